// Host runtime of libbrt: contexts, plans (problem normalisation, chunking, device buffers),
// HIP-graph capture/replay and the C ABI declared in include/brt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "brt.h"
#include "brt_api.h"
#include "brt_internal.h"

using namespace brt;

namespace {

// The calling thread's last error message: a fixed buffer, so that recording an error never allocates.
thread_local char g_err[512];

int vfail(int code, const char* fmt, va_list ap) {
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  return code;
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vfail(code, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(BRT_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool is_fin(double v) { return std::isfinite(v); }

template <typename Real>
PdeT<Real> to_device(const brt_problem& p, const Norm& n) {
  PdeT<Real> d;
  std::memset(&d, 0, sizeof(d));
  d.sigma = (Real)n.sigma;
  d.inv_lambda = (Real)n.inv_lambda;
  d.mu = (Real)n.mu;
  d.inv_q = (Real)(1.0 / n.q);
  d.q_lo = (uint32_t)(n.Q - 1);  // Q >= 1
  d.s_scale = n.Q < (1ull << 32) ? (Real)(1.0 / (4294967296.0 - (double)n.Q)) : (Real)0;
  d.K = n.K;
  d.jpack = 0;
  for (uint32_t i = 0; i < n.K; ++i) {
    d.jpack |= n.J[i] << (4 * i);
    d.omega[i] = (Real)n.omega[i];
  }
  d.u0_nterms = p.u0_nterms;
  d.cmod = p.coef_mod;
  d.cm_pow = p.coef_mod_pow;
  d.cm_bx = (Real)p.coef_mod_beta[0];
  d.cm_by = (Real)(p.dim == 2 ? p.coef_mod_beta[1] : 0.0);
  d.cm_t0 = (Real)p.coef_mod_t0;
  d.drift_on = (p.drift[0] != 0.0 || p.drift[1] != 0.0) ? 1u : 0u;
  d.drift[0] = (Real)p.drift[0];
  d.drift[1] = (Real)(p.dim == 2 ? p.drift[1] : 0.0);
  d.sde = p.sde;
  if (p.sde == BRT_SDE_EULER) {
    d.dlin[0] = (Real)p.drift_lin[0];
    d.dlin[1] = (Real)(p.dim == 2 ? p.drift_lin[1] : 0.0);
    d.sig_amp = (Real)p.sigma_amp;
    d.sig_k = p.sigma_amp != 0.0 ? (Real)(1.0 / (2.0 * p.sigma_width * p.sigma_width)) : (Real)0;
    d.inv_h = (Real)(1.0 / p.sde_dt);
  }
  for (int i = 0; i < kMaxU0Params; ++i) d.u0[i] = (Real)p.u0_params[i];
  if (p.u0_kind == BRT_U0_GAUSS_SUM)
    for (uint32_t k = 0; k < p.u0_nterms; ++k) {
      const double s = p.u0_params[4 * k + 3];
      d.u0[4 * k + 3] = (Real)(1.0 / (2.0 * s * s));
    }
  return d;
}

}  // namespace

namespace brt {

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vfail(code, fmt, ap);
  va_end(ap);
  return code;
}

// Strategy A normalisation of one problem (Sec. 2.1): u = v e^{mu t}, mu = c_1 + lambda, clock Exp(lambda),
// arity uniform over the K non-zero non-linear terms, vertex weight K c_j / lambda e^{(j-1) mu tau}.
Norm normalize(const brt_problem& p, const brt_mc& mc) {
  Norm n;
  n.sigma = std::sqrt(2.0 * p.diffusion);
  // With c_1 itself modulated, c_1(x, t) u cannot be absorbed into the prefactor: it joins the terms
  // chosen at a split as a branching with one child.
  const bool lin = p.coef_mod == BRT_COEF_MOD_GAUSS_TIME_ALL;
  const double c1 = lin ? 0.0 : p.coef[1];  // the part of c_1 in the prefactor e^{mu t}
  for (uint32_t j = 0; j < 8; ++j)
    if ((j != 1 || lin) && p.coef[j] != 0.0) n.J[n.K++] = j;
  if (n.K == 0) {
    n.lambda = 0.0;
    n.inv_lambda = 0.0;
    n.mu = c1;
  } else if (mc.strategy == BRT_STRATEGY_B) {
    // Strategy B: u = v e^{c_1 t}; a vertex carries tau K c_j / (1 - q) e^{(j-1) c_1 tau'}.  q is the
    // coin's realised leaf probability floor(q 2^32) / 2^32, so the weights match the coin exactly.
    n.q = std::floor(mc.q * 4294967296.0) * 0x1p-32;
    n.mu = c1;
    for (uint32_t i = 0; i < n.K; ++i) n.omega[i] = (double)n.K * p.coef[n.J[i]] / (1.0 - n.q);
  } else {
    n.lambda = mc.lambda;
    n.inv_lambda = 1.0 / mc.lambda;
    n.mu = c1 + mc.lambda;
    for (uint32_t i = 0; i < n.K; ++i) n.omega[i] = (double)n.K * p.coef[n.J[i]] / mc.lambda;
  }
  n.Q = (uint64_t)std::floor(n.q * 4294967296.0);  // exact: q 2^32 is a scaling by a power of two
  return n;
}

size_t pde_bytes(int precision) { return precision == 32 ? sizeof(PdeT<float>) : sizeof(PdeT<double>); }

uint32_t u0_param_count(uint32_t u0_kind, uint32_t nterms) {
  switch (u0_kind) {
    case BRT_U0_CONST: return 1;
    case BRT_U0_LOGISTIC: return 6;
    case BRT_U0_GAUSS_SUM: return 4 * nterms;
    default: return 3;
  }
}

template <typename Real>
static uint32_t family_stride_t(uint32_t u0_kind, const void* recs, size_t n) {
  if (n < 2) return 0;
  // records compared byte by byte (their padding is zero: to_device clears every record), so they are
  // copied with memcpy, which keeps the padding bytes
  const unsigned char* r = static_cast<const unsigned char*>(recs);
  PdeT<Real> first;
  std::memcpy(&first, r, sizeof(first));
  std::memset(first.u0, 0, sizeof(first.u0));
  first.u0_nterms = 0;
  uint32_t stride = 1;
  for (size_t i = 0; i < n; ++i) {
    PdeT<Real> x;
    std::memcpy(&x, r + i * sizeof(PdeT<Real>), sizeof(x));
    stride = std::max(stride, u0_param_count(u0_kind, x.u0_nterms));
    std::memset(x.u0, 0, sizeof(x.u0));
    x.u0_nterms = 0;
    if (std::memcmp(&x, &first, sizeof(x)) != 0) return 0;
  }
  return std::min<uint32_t>(stride, (uint32_t)kMaxU0Params);
}

uint32_t family_u0_stride(int precision, uint32_t u0_kind, const void* recs, size_t n) {
  return precision == 32 ? family_stride_t<float>(u0_kind, recs, n) : family_stride_t<double>(u0_kind, recs, n);
}

void pde_to_device(const brt_problem& p, const Norm& n, int precision, void* dst) {
  if (precision == 32) {
    const PdeT<float> d = to_device<float>(p, n);
    std::memcpy(dst, &d, sizeof(d));
  } else {
    const PdeT<double> d = to_device<double>(p, n);
    std::memcpy(dst, &d, sizeof(d));
  }
}

// Expected nodes per tree (cost model for ordering work): with arities uniform over J the number of
// lineages grows like e^{lambda (abar - 1) t}.
double est_nodes(const Norm& n, const brt_mc& mc, double t) {
  if (n.K == 0) return 1.0;
  double abar = 0;
  for (uint32_t i = 0; i < n.K; ++i) abar += n.J[i];
  abar /= n.K;
  double v;
  if (std::fabs(abar - 1.0) < 1e-9)
    v = 1.0 + n.lambda * t;
  else
    v = 1.0 + abar / (abar - 1.0) * std::expm1(std::min(50.0, n.lambda * (abar - 1.0) * t));
  if (mc.prune) v = std::min(v, 1.0 + abar * (mc.max_order + 1));
  return std::max(1.0, std::min(v, (double)mc.node_cap));
}

}  // namespace brt

struct brt_plan {
  brt_ctx* ctx = nullptr;
  int precision = 32, dim = 1, u0_kind = 0;
  uint32_t n_problems = 0, n_points = 0, n_bins = 0;
  uint32_t cmod = 0;  // some problem has variable coefficients
  uint32_t u0_stride = 0;  // > 0: the problems differ only in their initial data (a family launch)
  uint64_t total_trees = 0;
  brt_mc mc{};
  std::vector<PointRec> points;
  std::vector<Chunk> chunks;
  std::vector<Segment> segs;
  // device
  PointRec* d_points = nullptr;
  Chunk* d_chunks = nullptr;
  Segment* d_segs = nullptr;
  void* d_pdes = nullptr;
  uint32_t* d_counter = nullptr;
  unsigned long long* d_depth = nullptr;
  double* d_tree_f = nullptr;
  uint32_t* d_tree_meta = nullptr;
  void* d_spill = nullptr;
  Partial* d_partials = nullptr;
  unsigned long long* d_seg_nodes = nullptr;
  int grid = 0, waves_per_block = 4, stack_depth = 0, spill_depth = 0;
  // graph cache
  hipGraphExec_t graph = nullptr;
  brt_out graph_out{};
  hipStream_t graph_stream = nullptr;
  bool use_graph = true;
  uint64_t graph_captures = 0;  // graphs instantiated
  uint64_t graph_replays = 0;   // hipGraphLaunch calls (the first launch of a new graph included)
  uint64_t direct_runs = 0;     // runs enqueued kernel by kernel
  // per-kernel timing mode: events before the walk and after walk, reduce and finalize
  bool timing = false;
  std::vector<std::array<hipEvent_t, 4>> ev_pool;
  size_t ev_used = 0;
};

extern "C" {

int brt_version(void) { return 10000; }

const char* brt_last_error(void) { return g_err; }

int brt_create(brt_ctx** out, int device) {
  return brt::api_guard("brt_create", [&]() -> int {
    if (!out) return fail(BRT_E_ARG, "brt_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(BRT_E_ARG, "brt_create: device %d of %d", device, ndev);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    brt_ctx* c = new (std::nothrow) brt_ctx;
    if (!c) return fail(BRT_E_NOMEM, "brt_create: host allocation");
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    c->launch.struct_size = sizeof(brt_launch);
    c->launch.waves_per_block = 4;
    c->launch.blocks_per_cu = 0;
    c->launch.chunk_trees = 1024;
    c->launch.stack_depth = 0;
    // the allocation-free entry point's scratch array: its address on this device, looked up once
    int rc = noalloc_init_device(device);
    if (!rc) rc = contour_init_device(device);  // the finalize's pole-test contour
    if (rc) {
      delete c;
      return rc;
    }
    *out = c;
    g_err[0] = '\0';
    return BRT_OK;
  });
}

void brt_destroy(brt_ctx* ctx) { delete ctx; }

int brt_set_launch(brt_ctx* ctx, const brt_launch* l) {
  return brt::api_guard("brt_set_launch", [&]() -> int {
    if (!ctx || !l || l->struct_size != sizeof(brt_launch)) return fail(BRT_E_ARG, "brt_set_launch: bad arguments");
    if (l->waves_per_block < 1 || l->waves_per_block > 4) return fail(BRT_E_ARG, "waves_per_block must be 1..4");
    if (l->chunk_trees < 64 || l->chunk_trees % 64 != 0 || l->chunk_trees > (1u << 24))
      return fail(BRT_E_ARG, "chunk_trees must be a multiple of 64 in [64, 2^24]");
    if (l->stack_depth > 255) return fail(BRT_E_ARG, "stack_depth must be <= 255");
    ctx->launch = *l;
    return BRT_OK;
  });
}

int brt_get_launch(brt_ctx* ctx, brt_launch* l) {
  return brt::api_guard("brt_get_launch", [&]() -> int {
    if (!ctx || !l) return fail(BRT_E_ARG, "brt_get_launch: NULL argument");
    *l = ctx->launch;
    return BRT_OK;
  });
}

int brt_problem_check(const brt_problem* p, const brt_mc* mc) {
  return brt::api_guard("brt_problem_check", [&]() -> int {
    if (!p || !mc) return fail(BRT_E_ARG, "problem/mc is NULL");
    if (p->struct_size != sizeof(brt_problem)) return fail(BRT_E_ARG, "brt_problem.struct_size mismatch");
    if (mc->struct_size != sizeof(brt_mc)) return fail(BRT_E_ARG, "brt_mc.struct_size mismatch");
    if (p->dim != 1 && p->dim != 2) return fail(BRT_E_ARG, "dim must be 1 or 2");
    if (!(p->diffusion > 0.0) || !is_fin(p->diffusion)) return fail(BRT_E_ARG, "diffusion must be > 0");
    for (int j = 0; j < 8; ++j)
      if (!is_fin(p->coef[j])) return fail(BRT_E_ARG, "coef[%d] is not finite", j);
    for (int j = 0; j < 40; ++j)
      if (!is_fin(p->u0_params[j])) return fail(BRT_E_ARG, "u0_params[%d] is not finite", j);
    switch (p->u0_kind) {
      case BRT_U0_CONST:
        break;
      case BRT_U0_LOGISTIC: {
        const double pw = p->u0_params[3];
        if (!(pw == 1.0 || pw == 2.0 || pw == 3.0 || pw == 4.0)) return fail(BRT_E_ARG, "logistic power must be 1..4");
        break;
      }
      case BRT_U0_GAUSS_SUM:
        if (p->u0_nterms < 1 || p->u0_nterms > 8) return fail(BRT_E_ARG, "gauss_sum needs 1..8 terms");
        for (uint32_t k = 0; k < p->u0_nterms; ++k)
          if (!(p->u0_params[4 * k + 3] > 0.0)) return fail(BRT_E_ARG, "gauss_sum width must be > 0");
        break;
      case BRT_U0_COS2_BUMP:
        if (!(p->u0_params[1] > 0.0) || (p->dim == 2 && !(p->u0_params[2] > 0.0)))
          return fail(BRT_E_ARG, "cos2_bump half-widths must be > 0");
        break;
      default:
        return fail(BRT_E_ARG, "unknown u0_kind %u", p->u0_kind);
    }
    switch (p->coef_mod) {
      case BRT_COEF_MOD_NONE:
        break;
      case BRT_COEF_MOD_GAUSS_TIME:
      case BRT_COEF_MOD_GAUSS_TIME_ALL:
        if (!(p->coef_mod_beta[0] >= 0.0) || !(p->coef_mod_beta[1] >= 0.0) || !is_fin(p->coef_mod_beta[0]) ||
            !is_fin(p->coef_mod_beta[1]))
          return fail(BRT_E_ARG, "coef_mod_beta must be finite and >= 0");
        if (p->coef_mod_pow > 1) return fail(BRT_E_ARG, "coef_mod_pow must be 0 or 1");
        if (p->coef_mod_pow == 1 && !(p->coef_mod_t0 > 0.0 && is_fin(p->coef_mod_t0)))
          return fail(BRT_E_ARG, "coef_mod_t0 must be > 0 with coef_mod_pow 1");
        break;
      default:
        return fail(BRT_E_ARG, "unknown coef_mod %u", p->coef_mod);
    }
    if (!is_fin(p->drift[0]) || !is_fin(p->drift[1])) return fail(BRT_E_ARG, "drift must be finite");
    if (p->dim == 1 && p->drift[1] != 0.0) return fail(BRT_E_ARG, "drift[1] must be 0 in 1-D");
    if (p->sde == BRT_SDE_EXACT) {
      if (p->drift_lin[0] != 0.0 || p->drift_lin[1] != 0.0 || p->sigma_amp != 0.0)
        return fail(BRT_E_ARG, "drift_lin and sigma_amp need sde = BRT_SDE_EULER");
    } else if (p->sde == BRT_SDE_EULER) {
      if (!(p->sde_dt >= 1e-6) || !is_fin(p->sde_dt)) return fail(BRT_E_ARG, "sde_dt must be finite and >= 1e-6");
      if (!is_fin(p->drift_lin[0]) || !is_fin(p->drift_lin[1])) return fail(BRT_E_ARG, "drift_lin must be finite");
      if (p->dim == 1 && p->drift_lin[1] != 0.0) return fail(BRT_E_ARG, "drift_lin[1] must be 0 in 1-D");
      if (!(p->sigma_amp > -1.0) || !is_fin(p->sigma_amp)) return fail(BRT_E_ARG, "sigma_amp must be finite and > -1");
      if (p->sigma_amp != 0.0 && (!(p->sigma_width > 0.0) || !is_fin(p->sigma_width)))
        return fail(BRT_E_ARG, "sigma_width must be finite and > 0");
    } else {
      return fail(BRT_E_ARG, "unknown sde %u", p->sde);
    }
    if (mc->precision != 32 && mc->precision != 64) return fail(BRT_E_ARG, "precision must be 32 or 64");
    // An Euler edge takes ceil(s / h) steps; an FP32 path's edge duration s differs from its FP64 value by a
    // rounding, which can change the step count (and the tree) at a step boundary: only FP64 paths step.
    if (p->sde == BRT_SDE_EULER && mc->precision != 64)
      return fail(BRT_E_ARG, "Euler-Maruyama paths (sde = BRT_SDE_EULER) need precision 64");
    if (!(mc->lambda > 0.0) || !is_fin(mc->lambda)) return fail(BRT_E_ARG, "lambda must be > 0");
    if (mc->max_order > 126) return fail(BRT_E_ARG, "max_order must be <= 126");
    if (mc->node_cap < 1 || mc->node_cap > kMaxNodeCap) return fail(BRT_E_ARG, "node_cap must be in [1, 2^21-1]");
    if (mc->pade_L + mc->pade_M > mc->max_order) return fail(BRT_E_ARG, "pade_L + pade_M must be <= max_order");
    if (mc->pade_M > 16) return fail(BRT_E_ARG, "pade_M must be <= 16");
    if (mc->strategy != BRT_STRATEGY_A && mc->strategy != BRT_STRATEGY_B) return fail(BRT_E_ARG, "unknown strategy");
    if (mc->strategy == BRT_STRATEGY_B) {
      if (!(mc->q >= 1e-9 && mc->q <= 1.0)) return fail(BRT_E_ARG, "Strategy B needs 1e-9 <= q <= 1");
      double abar = 0.0;
      uint32_t K = 0;
      for (uint32_t j = 0; j < 8; ++j)
        if (j != 1 && p->coef[j] != 0.0) {
          abar += j;
          K += 1;
        }
      if (K > 0 && mc->q >= 1.0) return fail(BRT_E_ARG, "Strategy B with a non-linear term needs q < 1");
      if (K > 0 && !mc->prune && (1.0 - mc->q) * abar / K >= 1.0)
        return fail(BRT_E_ARG, "Strategy B without pruning needs subcritical trees: (1 - q) * mean arity < 1");
    }
    return BRT_OK;
  });
}

}  // extern "C"

static void plan_free(brt_plan* p) {
  if (!p) return;
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  for (auto& e : p->ev_pool)
    for (hipEvent_t ev : e) (void)hipEventDestroy(ev);
  (void)hipFree(p->d_points);
  (void)hipFree(p->d_chunks);
  (void)hipFree(p->d_segs);
  (void)hipFree(p->d_pdes);
  (void)hipFree(p->d_counter);
  (void)hipFree(p->d_depth);
  (void)hipFree(p->d_tree_f);
  (void)hipFree(p->d_tree_meta);
  (void)hipFree(p->d_spill);
  (void)hipFree(p->d_partials);
  (void)hipFree(p->d_seg_nodes);
  delete p;
}

template <typename T>
static int upload(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  if (hipMalloc(reinterpret_cast<void**>(dst), bytes) != hipSuccess)
    return fail(BRT_E_NOMEM, "hipMalloc(%zu) failed", bytes);
  if (!v.empty()) HIP_TRY(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return BRT_OK;
}

extern "C" int brt_plan_create(brt_ctx* ctx, uint32_t n_problems, const brt_problem* problems, const brt_mc* mc,
                    const brt_points* pts, brt_plan** out) {
  return brt::api_guard("brt_plan_create", [&]() -> int {
    if (!ctx || !problems || !mc || !pts || !out) return fail(BRT_E_ARG, "brt_plan_create: NULL argument");
    *out = nullptr;
    if (pts->struct_size != sizeof(brt_points)) return fail(BRT_E_ARG, "brt_points.struct_size mismatch");
    if (n_problems < 1 || n_problems > (uint32_t)kMaxProblems)
      return fail(BRT_E_ARG, "n_problems must be 1..%d", kMaxProblems);
    for (uint32_t i = 0; i < n_problems; ++i) {
      int rc = brt_problem_check(&problems[i], mc);
      if (rc) return rc;
      if (problems[i].dim != problems[0].dim || problems[i].u0_kind != problems[0].u0_kind)
        return fail(BRT_E_ARG, "all problems of a plan must share dim and u0_kind");
    }
    if (pts->n > 0 && (!pts->x || !pts->t || !pts->n_trees)) return fail(BRT_E_ARG, "points: NULL array");
    HIP_TRY(hipSetDevice(ctx->device));

    brt_plan* p = new (std::nothrow) brt_plan;
    if (!p) return fail(BRT_E_NOMEM, "host allocation");
    p->ctx = ctx;
    p->precision = (int)mc->precision;
    p->dim = (int)problems[0].dim;
    p->u0_kind = (int)problems[0].u0_kind;
    p->n_problems = n_problems;
    for (uint32_t i = 0; i < n_problems; ++i) p->cmod |= general_coefficients(problems[i]) ? 1u : 0u;
    p->n_points = pts->n;
    p->n_bins = mc->max_order + 2;
    p->mc = *mc;

    std::vector<Norm> norms(n_problems);
    for (uint32_t i = 0; i < n_problems; ++i) norms[i] = normalize(problems[i], *mc);

    // points
    const uint32_t dim = (uint32_t)p->dim;
    p->points.resize(pts->n);
    std::vector<double> cost(pts->n, 1.0);
    uint64_t base = 0;
    for (uint32_t i = 0; i < pts->n; ++i) {
      const uint32_t pid = pts->problem_id ? pts->problem_id[i] : 0u;
      if (pid >= n_problems) {
        plan_free(p);
        return fail(BRT_E_ARG, "point %u: problem_id %u out of range", i, pid);
      }
      const double t = pts->t[i];
      if (!(t >= 0.0) || !is_fin(t)) {
        plan_free(p);
        return fail(BRT_E_ARG, "point %u: t must be finite and >= 0", i);
      }
      if (pts->n_trees[i] > 0xffffffffull) {
        plan_free(p);
        return fail(BRT_E_ARG, "point %u: at most 2^32-1 trees", i);
      }
      PointRec& r = p->points[i];
      std::memset(&r, 0, sizeof(r));
      for (uint32_t d = 0; d < dim; ++d) {
        r.x[d] = pts->x[(size_t)i * dim + d];
        if (!is_fin(r.x[d])) {
          plan_free(p);
          return fail(BRT_E_ARG, "point %u: x is not finite", i);
        }
      }
      r.t = t;
      const Norm& nz = norms[pid];
      r.theta = nz.K > 0 ? std::exp(-nz.lambda * t) : 1.0;
      r.mu = nz.mu;
      r.tree_base = base;
      r.n_trees = (uint32_t)pts->n_trees[i];
      r.point_id = pts->point_id ? pts->point_id[i] : i;
      r.tree_first = pts->tree_first ? pts->tree_first[i] : 0u;
      r.n_total = r.n_trees;
      r.out_row = i;
      if ((uint64_t)r.tree_first + r.n_trees > 0xffffffffull) {
        plan_free(p);
        return fail(BRT_E_ARG, "point %u: tree_first + n_trees exceeds 2^32-1", i);
      }
      r.pde = pid;
      base += r.n_trees;
      cost[i] = est_nodes(nz, *mc, t);
    }
    p->total_trees = base;

    // walker chunks, most expensive first (longest-processing-time order)
    const uint32_t ct = ctx->launch.chunk_trees;
    std::vector<uint32_t> order(pts->n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });
    // (64-bit range counters: a point's tree count reaches 2^32 - 1, where a 32-bit counter would wrap)
    const uint32_t seg_trees = plan_seg_trees(p->total_trees);
    try {
      for (uint32_t i : order) {
        const uint64_t n = p->points[i].n_trees;
        for (uint64_t b0 = 0; b0 < n; b0 += ct)
          p->chunks.push_back(Chunk{i, (uint32_t)b0, (uint32_t)std::min<uint64_t>(n, b0 + ct), 0u});
      }
      // reduction segments, in point order
      for (uint32_t i = 0; i < pts->n; ++i) {
        PointRec& r = p->points[i];
        r.seg_begin = (uint32_t)p->segs.size();
        for (uint64_t b0 = 0; b0 < r.n_trees; b0 += seg_trees)
          p->segs.push_back(Segment{i, (uint32_t)b0, (uint32_t)std::min<uint64_t>(r.n_trees, b0 + seg_trees),
                                    (uint32_t)p->segs.size()});
        r.seg_count = (uint32_t)p->segs.size() - r.seg_begin;
      }
    } catch (const std::bad_alloc&) {
      plan_free(p);
      return fail(BRT_E_NOMEM, "plan: host allocation of the chunk and segment tables");
    }

    // Stack depth: with pruning a lineage holds at most max_order vertices with children still to
    // start; without pruning the depth is capped at kMaxDepthUnpruned (deeper trees are flagged).  The
    // top levels live in LDS, the rest in a per-thread global spill area.
    const uint32_t needed = mc->prune ? std::max(1u, mc->max_order) : kMaxDepthUnpruned;
    const uint32_t lds_levels = ctx->launch.stack_depth ? ctx->launch.stack_depth : kDefaultLdsLevels;
    p->stack_depth = (int)std::min(needed, lds_levels);
    p->spill_depth = (int)(needed - (uint32_t)p->stack_depth);
    p->waves_per_block = (int)ctx->launch.waves_per_block;

    int rc = BRT_OK;
    if (p->precision == 32) {
      std::vector<PdeT<float>> tab(n_problems);
      for (uint32_t i = 0; i < n_problems; ++i) tab[i] = to_device<float>(problems[i], norms[i]);
      p->u0_stride = family_u0_stride(32, (uint32_t)p->u0_kind, tab.data(), tab.size());
      rc = upload(reinterpret_cast<PdeT<float>**>(&p->d_pdes), tab);
    } else {
      std::vector<PdeT<double>> tab(n_problems);
      for (uint32_t i = 0; i < n_problems; ++i) tab[i] = to_device<double>(problems[i], norms[i]);
      p->u0_stride = family_u0_stride(64, (uint32_t)p->u0_kind, tab.data(), tab.size());
      rc = upload(reinterpret_cast<PdeT<double>**>(&p->d_pdes), tab);
    }
    if (!rc) rc = upload(&p->d_points, p->points);
    if (!rc) rc = upload(&p->d_chunks, p->chunks);
    if (!rc) rc = upload(&p->d_segs, p->segs);
    if (rc) {
      plan_free(p);
      return rc;
    }
    const size_t nb3 = (size_t)(p->n_bins + 3);
    if (hipMalloc(reinterpret_cast<void**>(&p->d_counter), 64) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&p->d_depth), 64) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&p->d_partials), std::max<size_t>(1, p->segs.size()) * nb3 * sizeof(Partial)) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&p->d_seg_nodes),
                  std::max<size_t>(1, p->segs.size()) * sizeof(unsigned long long)) != hipSuccess) {
      plan_free(p);
      return fail(BRT_E_NOMEM, "plan scratch allocation failed");
    }
    HIP_TRY(hipMemset(p->d_depth, 0, 64));

    // persistent grid: as many blocks as are resident at once
    int bpc = (int)ctx->launch.blocks_per_cu;
    int maxb = walk_max_blocks_per_cu(p->precision, p->dim, p->u0_kind, (int)p->n_problems, p->stack_depth, p->waves_per_block,
                                   (int)p->mc.strategy, (int)p->u0_stride);
    while (maxb <= 0 && p->waves_per_block > 1) {  // shrink the block until its LDS fits
      p->waves_per_block -= 1;
      maxb = walk_max_blocks_per_cu(p->precision, p->dim, p->u0_kind, (int)p->n_problems, p->stack_depth, p->waves_per_block,
                                   (int)p->mc.strategy, (int)p->u0_stride);
    }
    if (maxb <= 0) {
      plan_free(p);
      return fail(BRT_E_ARG, "launch settings do not fit the device (stack_depth %d, %d waves per block)",
                  p->stack_depth, p->waves_per_block);
    }
    if (bpc == 0 || bpc > maxb) bpc = maxb;
    p->grid = std::max(1, std::min<int>(bpc * ctx->n_cu, (int)std::max<size_t>(1, p->chunks.size())));
    if (p->spill_depth > 0) {
      const size_t bytes = (size_t)p->grid * p->waves_per_block * kWave * p->spill_depth *
                           stack_entry_size(p->precision, p->dim);
      if (hipMalloc(&p->d_spill, bytes) != hipSuccess) {
        plan_free(p);
        return fail(BRT_E_NOMEM, "stack spill area: hipMalloc(%zu)", bytes);
      }
    }
    *out = p;
    g_err[0] = '\0';
    return BRT_OK;
  });
}

extern "C" {
int brt_plan_info(const brt_plan* p, uint32_t* n_points, uint64_t* n_trees, uint32_t* n_bins, uint32_t* n_chunks);
}

// (called from entry points, which turn exceptions into status codes)
static int ensure_records(brt_plan* p) {
  if (p->d_tree_f) return BRT_OK;
  const size_t n = std::max<uint64_t>(1, p->total_trees);
  const size_t fb = n * sizeof(double);
  if (hipMalloc(reinterpret_cast<void**>(&p->d_tree_f), fb) != hipSuccess) return fail(BRT_E_NOMEM, "tree records: hipMalloc(%zu)", fb);
  if (hipMalloc(reinterpret_cast<void**>(&p->d_tree_meta), n * 4) != hipSuccess)
    return fail(BRT_E_NOMEM, "tree records: hipMalloc(%zu)", n * 4);
  return BRT_OK;
}

static int enqueue(brt_plan* p, const brt_out* o, hipStream_t s) {
  double* tf = reinterpret_cast<double*>(o->tree_f);
  uint32_t* tm = o->tree_meta;
  if (!tf || !tm) {
    int rc = ensure_records(p);
    if (rc) return rc;
    tf = p->d_tree_f;
    tm = p->d_tree_meta;
  }
  std::array<hipEvent_t, 4>* ev = nullptr;
  if (p->timing) {
    if (p->ev_used == p->ev_pool.size()) {
      std::array<hipEvent_t, 4> e{};
      for (auto& x : e) HIP_TRY(hipEventCreate(&x));
      p->ev_pool.push_back(e);
    }
    ev = &p->ev_pool[p->ev_used++];
  }
  HIP_TRY(launch_reset(p->d_counter, p->d_depth, s));
  if (ev) HIP_TRY(hipEventRecord((*ev)[0], s));
  if (!p->chunks.empty()) {
    WalkArgs w{};
    w.points = p->d_points;
    w.chunks = p->d_chunks;
    w.n_chunks = (uint32_t)p->chunks.size();
    w.n_problems = p->n_problems;
    w.pdes = p->d_pdes;
    w.chunk_counter = p->d_counter;
    w.depth_counter = p->d_depth;
    w.tree_f = tf;
    w.tree_meta = tm;
    w.key0 = (uint32_t)(p->mc.seed & 0xffffffffull);
    w.key1 = (uint32_t)(p->mc.seed >> 32);
    w.max_order = p->mc.max_order;
    w.prune = p->mc.prune;
    w.node_cap = p->mc.node_cap;
    w.strategy = p->mc.strategy;
    w.cmod = p->cmod;
    w.stack_depth = (uint32_t)p->stack_depth;
    w.spill_depth = (uint32_t)p->spill_depth;
    w.spill = p->d_spill;
    w.n_threads = (uint32_t)(p->grid * p->waves_per_block * kWave);
    w.u0_stride = p->u0_stride;
    HIP_TRY(launch_walk(p->precision, p->dim, p->u0_kind, w, p->grid, p->waves_per_block, s));
  }
  if (ev) HIP_TRY(hipEventRecord((*ev)[1], s));
  ReduceArgs r{};
  r.points = p->d_points;
  r.segs = p->d_segs;
  r.n_segs = (uint32_t)p->segs.size();
  r.tree_f = tf;
  r.tree_meta = tm;
  r.partials = p->d_partials;
  r.seg_nodes = p->d_seg_nodes;
  r.n_bins = p->n_bins;
  HIP_TRY(launch_reduce(r, s));
  if (ev) HIP_TRY(hipEventRecord((*ev)[2], s));
  FinalizeArgs f{};
  f.points = p->d_points;
  f.n_points = p->n_points;
  f.partials = p->d_partials;
  f.seg_nodes = p->d_seg_nodes;
  f.n_bins = p->n_bins;
  f.pade_L = p->mc.pade_L;
  f.pade_M = p->mc.pade_M;
  f.u = o->u;
  f.se = o->se;
  f.psum = o->psum;
  f.coef = o->coef;
  f.coef_var = o->coef_var;
  f.hist = reinterpret_cast<unsigned long long*>(o->hist);
  f.s1 = o->s1;
  f.s2 = o->s2;
  f.nodes = reinterpret_cast<unsigned long long*>(o->nodes);
  f.flags = o->flags;
  f.pade_diag = o->pade_diag;
  HIP_TRY(launch_finalize(f, s));
  if (ev) HIP_TRY(hipEventRecord((*ev)[3], s));
  return BRT_OK;
}

extern "C" {

int brt_plan_execute(brt_plan* p, const brt_out* o, void* stream) {
  return brt::api_guard("brt_plan_execute", [&]() -> int {
    if (!p || !o) return fail(BRT_E_ARG, "brt_plan_execute: NULL argument");
    if (o->struct_size != sizeof(brt_out)) return fail(BRT_E_ARG, "brt_out.struct_size mismatch");
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!s || !p->use_graph || p->timing) {
      const int rc = enqueue(p, o, s);
      if (!rc) p->direct_runs += 1;
      return rc;
    }
    if (p->graph && p->graph_stream == s && std::memcmp(&p->graph_out, o, sizeof(brt_out)) == 0) {
      HIP_TRY(hipGraphLaunch(p->graph, s));
      p->graph_replays += 1;
      return BRT_OK;
    }
    if (p->graph) {
      (void)hipGraphExecDestroy(p->graph);
      p->graph = nullptr;
    }
    if (!o->tree_f || !o->tree_meta) {
      int rc = ensure_records(p);  // allocate outside the capture
      if (rc) return rc;
    }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = enqueue(p, o, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(BRT_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      p->graph = nullptr;
      return fail(BRT_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    p->graph_out = *o;
    p->graph_stream = s;
    p->graph_captures += 1;
    HIP_TRY(hipGraphLaunch(p->graph, s));
    p->graph_replays += 1;
    return BRT_OK;
  });
}

int brt_plan_set_graph(brt_plan* p, int enable) {
  return brt::api_guard("brt_plan_set_graph", [&]() -> int {
    if (!p) return fail(BRT_E_ARG, "brt_plan_set_graph: NULL plan");
    p->use_graph = enable != 0;
    return BRT_OK;
  });
}

int brt_plan_graph_stats(const brt_plan* p, uint64_t* captures, uint64_t* replays, uint64_t* direct) {
  return brt::api_guard("brt_plan_graph_stats", [&]() -> int {
    if (!p) return fail(BRT_E_ARG, "brt_plan_graph_stats: NULL plan");
    if (captures) *captures = p->graph_captures;
    if (replays) *replays = p->graph_replays;
    if (direct) *direct = p->direct_runs;
    return BRT_OK;
  });
}

int brt_plan_info(const brt_plan* p, uint32_t* n_points, uint64_t* n_trees, uint32_t* n_bins, uint32_t* n_chunks) {
  return brt::api_guard("brt_plan_info", [&]() -> int {
    if (!p) return fail(BRT_E_ARG, "brt_plan_info: NULL plan");
    if (n_points) *n_points = p->n_points;
    if (n_trees) *n_trees = p->total_trees;
    if (n_bins) *n_bins = p->n_bins;
    if (n_chunks) *n_chunks = (uint32_t)p->chunks.size();
    return BRT_OK;
  });
}

int brt_plan_depth_exceeded(brt_plan* p, uint64_t* count) {
  return brt::api_guard("brt_plan_depth_exceeded", [&]() -> int {
    if (!p || !count) return fail(BRT_E_ARG, "NULL argument");
    unsigned long long v = 0;
    HIP_TRY(hipMemcpy(&v, p->d_depth, sizeof(v), hipMemcpyDeviceToHost));
    *count = v;
    return BRT_OK;
  });
}

int brt_plan_set_timing(brt_plan* p, int enable) {
  return brt::api_guard("brt_plan_set_timing", [&]() -> int {
    if (!p) return fail(BRT_E_ARG, "brt_plan_set_timing: NULL plan");
    p->timing = enable != 0;
    p->ev_used = 0;
    return BRT_OK;
  });
}

int brt_plan_get_timing(brt_plan* p, double* ms, uint64_t* runs) {
  return brt::api_guard("brt_plan_get_timing", [&]() -> int {
    if (!p || !ms) return fail(BRT_E_ARG, "brt_plan_get_timing: NULL argument");
    double acc[3] = {0, 0, 0};
    for (size_t i = 0; i < p->ev_used; ++i) {
      auto& e = p->ev_pool[i];
      HIP_TRY(hipEventSynchronize(e[3]));
      for (int k = 0; k < 3; ++k) {
        float v = 0.f;
        HIP_TRY(hipEventElapsedTime(&v, e[k], e[k + 1]));
        acc[k] += v;
      }
    }
    for (int k = 0; k < 3; ++k) ms[k] = acc[k];
    if (runs) *runs = p->ev_used;
    p->ev_used = 0;
    return BRT_OK;
  });
}

void brt_plan_destroy(brt_plan* p) { plan_free(p); }

int brt_solve(brt_ctx* ctx, uint32_t n_problems, const brt_problem* problems, const brt_mc* mc,
              const brt_points* points, const brt_out* out, void* stream) {
  return brt::api_guard("brt_solve", [&]() -> int {
    brt_plan* p = nullptr;
    int rc = brt_plan_create(ctx, n_problems, problems, mc, points, &p);
    if (rc) return rc;
    p->use_graph = false;
    rc = enqueue(p, out, reinterpret_cast<hipStream_t>(stream));
    if (!rc) {
      hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
      if (e != hipSuccess) rc = fail(BRT_E_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    uint64_t deep = 0;
    if (!rc) rc = brt_plan_depth_exceeded(p, &deep);
    plan_free(p);
    if (!rc && deep) rc = fail(BRT_E_RANGE, "%llu trees exceeded the stack depth", (unsigned long long)deep);
    return rc;
  });
}

}  // extern "C"
