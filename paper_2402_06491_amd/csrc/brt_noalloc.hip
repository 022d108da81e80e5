// brt_solve_noalloc (include/brt.h): the one-shot solve without any device or host allocation, for
// callers that cannot allocate.  Everything brt_solve would allocate (the problem table, point records,
// work chunks, reduction segments and partials, counters and, unless the caller supplies them, the tree
// records) lives in one file-scope device array, `scratch`, of kScratchBytes; the host side builds its
// tables in fixed file-scope arrays.  Both are shared by every call on a device: a mutex serialises the
// calls (each one waits for its stream before it returns), so calls that would overlap run one after the
// other.  The kernels are the ones of brt_solve, with the walker's whole stack in LDS (no spill area).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "brt.h"
#include "brt_api.h"
#include "brt_internal.h"

using namespace brt;

namespace {

constexpr uint32_t kNaMaxPoints = BRT_NOALLOC_MAX_POINTS;
constexpr uint64_t kNaMaxTrees = BRT_NOALLOC_MAX_TREES;
constexpr uint32_t kNaMaxOrder = BRT_NOALLOC_MAX_ORDER;
constexpr uint32_t kNaMaxBins = kNaMaxOrder + 2;
constexpr uint32_t kNaMaxChunks = (uint32_t)(kNaMaxTrees / 64) + kNaMaxPoints;  // chunks hold >= 64 trees
constexpr uint32_t kNaMaxSegs = (uint32_t)(kNaMaxTrees / kPlanSegMin) + kNaMaxPoints;
constexpr int kNaMaxDevices = 64;

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kOffPdes = 0;
constexpr size_t kOffPoints = align256(kOffPdes + (size_t)kMaxProblems * sizeof(PdeT<double>));
constexpr size_t kOffChunks = align256(kOffPoints + (size_t)kNaMaxPoints * sizeof(PointRec));
constexpr size_t kOffSegs = align256(kOffChunks + (size_t)kNaMaxChunks * sizeof(Chunk));
constexpr size_t kOffCounter = align256(kOffSegs + (size_t)kNaMaxSegs * sizeof(Segment));
constexpr size_t kOffDepth = kOffCounter + 64;
constexpr size_t kOffPartials = align256(kOffDepth + 64);
constexpr size_t kOffSegNodes = align256(kOffPartials + (size_t)kNaMaxSegs * (kNaMaxBins + 3) * sizeof(Partial));
constexpr size_t kOffTreeF = align256(kOffSegNodes + (size_t)kNaMaxSegs * sizeof(unsigned long long));
constexpr size_t kOffTreeMeta = align256(kOffTreeF + (size_t)kNaMaxTrees * sizeof(double));
constexpr size_t kScratchBytes = align256(kOffTreeMeta + (size_t)kNaMaxTrees * sizeof(uint32_t));
static_assert(kScratchBytes <= (size_t(60) << 20), "the scratch array is meant to stay near 55 MiB");

// The device scratch array.  In host code its name is only a handle for hipGetSymbolAddress: the device
// address of each GPU's copy is looked up once (noalloc_init_device) and used everywhere instead.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;                         // serialises the calls (they share the arrays below and `scratch`)
void* g_scratch[kNaMaxDevices] = {};     // device address of `scratch` on each device

// host-side tables of one call
unsigned char h_pdes[(size_t)kMaxProblems * sizeof(PdeT<double>)];
PointRec h_points[kNaMaxPoints];
Chunk h_chunks[kNaMaxChunks];
Segment h_segs[kNaMaxSegs];
double h_cost[kNaMaxPoints];
uint32_t h_order[kNaMaxPoints];
Norm h_norm[kMaxProblems];

int na_fail(int code, const char* what) { return set_error(code, "brt_solve_noalloc: %s", what); }

#define NA_TRY(expr)                                                                                 \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return set_error(BRT_E_DEVICE, "brt_solve_noalloc: %s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

namespace brt {

int noalloc_init_device(int device) {
  if (device < 0 || device >= kNaMaxDevices) return set_error(BRT_E_DEVICE, "device %d: no scratch slot", device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return BRT_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return set_error(BRT_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  g_scratch[device] = ptr;
  return BRT_OK;
}

}  // namespace brt

extern "C" int brt_solve_noalloc(brt_ctx* ctx, uint32_t n_problems, const brt_problem* problems, const brt_mc* mc,
                                 const brt_points* pts, const brt_out* o, void* stream) {
  return brt::api_guard("brt_solve_noalloc", [&]() -> int {
    if (!ctx || !problems || !mc || !pts || !o) return na_fail(BRT_E_ARG, "NULL argument");
    if (pts->struct_size != sizeof(brt_points)) return na_fail(BRT_E_ARG, "brt_points.struct_size mismatch");
    if (o->struct_size != sizeof(brt_out)) return na_fail(BRT_E_ARG, "brt_out.struct_size mismatch");
    if (n_problems < 1 || n_problems > (uint32_t)kMaxProblems) return na_fail(BRT_E_ARG, "n_problems must be 1..64");
    for (uint32_t i = 0; i < n_problems; ++i) {
      const int rc = brt_problem_check(&problems[i], mc);
      if (rc) return rc;
      if (problems[i].dim != problems[0].dim || problems[i].u0_kind != problems[0].u0_kind)
        return na_fail(BRT_E_ARG, "all problems must share dim and u0_kind");
    }
    if (!mc->prune || mc->max_order < 1 || mc->max_order > kNaMaxOrder)
      return na_fail(BRT_E_ARG, "needs pruning and 1 <= max_order <= BRT_NOALLOC_MAX_ORDER (the walker's stack is all in LDS)");
    if (pts->n > kNaMaxPoints) return na_fail(BRT_E_ARG, "more than BRT_NOALLOC_MAX_POINTS points");
    if (pts->n > 0 && (!pts->x || !pts->t || !pts->n_trees)) return na_fail(BRT_E_ARG, "points: NULL array");
    if (ctx->device < 0 || ctx->device >= kNaMaxDevices) return na_fail(BRT_E_ARG, "device out of range");
    uint64_t total = 0;
    for (uint32_t i = 0; i < pts->n; ++i) {
      if (pts->n_trees[i] > 0xffffffffull) return na_fail(BRT_E_ARG, "at most 2^32-1 trees per point");
      total += pts->n_trees[i];
    }
    if (total > kNaMaxTrees) return na_fail(BRT_E_ARG, "more than BRT_NOALLOC_MAX_TREES trees in one call");

    std::lock_guard<std::mutex> lk(g_mu);
    unsigned char* base = static_cast<unsigned char*>(g_scratch[ctx->device]);
    if (!base) return na_fail(BRT_E_DEVICE, "scratch address unknown on this device");
    NA_TRY(hipSetDevice(ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    const int precision = (int)mc->precision, dim = (int)problems[0].dim, u0_kind = (int)problems[0].u0_kind;
    const uint32_t B = mc->max_order + 2;
    const size_t pb = pde_bytes(precision);
    for (uint32_t i = 0; i < n_problems; ++i) {
      h_norm[i] = normalize(problems[i], *mc);
      pde_to_device(problems[i], h_norm[i], precision, h_pdes + i * pb);
    }
    // points
    uint64_t tree_base = 0;
    for (uint32_t i = 0; i < pts->n; ++i) {
      const uint32_t pid = pts->problem_id ? pts->problem_id[i] : 0u;
      if (pid >= n_problems) return na_fail(BRT_E_ARG, "problem_id out of range");
      const double t = pts->t[i];
      if (!(t >= 0.0) || !std::isfinite(t)) return na_fail(BRT_E_ARG, "t must be finite and >= 0");
      PointRec& r = h_points[i];
      std::memset(&r, 0, sizeof(r));
      for (int d = 0; d < dim; ++d) {
        r.x[d] = pts->x[(size_t)i * dim + d];
        if (!std::isfinite(r.x[d])) return na_fail(BRT_E_ARG, "x is not finite");
      }
      const Norm& nz = h_norm[pid];
      r.t = t;
      r.theta = nz.K > 0 ? std::exp(-nz.lambda * t) : 1.0;
      r.mu = nz.mu;
      r.tree_base = tree_base;
      r.n_trees = (uint32_t)pts->n_trees[i];
      r.point_id = pts->point_id ? pts->point_id[i] : i;
      r.tree_first = pts->tree_first ? pts->tree_first[i] : 0u;
      if ((uint64_t)r.tree_first + r.n_trees > 0xffffffffull) return na_fail(BRT_E_ARG, "tree_first + n_trees exceeds 2^32-1");
      r.n_total = r.n_trees;
      r.out_row = i;
      r.pde = pid;
      tree_base += r.n_trees;
      h_cost[i] = est_nodes(nz, *mc, t);
      h_order[i] = i;
    }
    // chunks, most expensive points first (ties by index, so the order does not depend on the sort)
    std::sort(h_order, h_order + pts->n,
              [](uint32_t a, uint32_t b) { return h_cost[a] > h_cost[b] || (h_cost[a] == h_cost[b] && a < b); });
    const uint32_t ct = ctx->launch.chunk_trees;
    uint32_t nc = 0, ns = 0;
    for (uint32_t k = 0; k < pts->n; ++k) {
      const uint32_t i = h_order[k];
      const uint64_t n = h_points[i].n_trees;
      for (uint64_t b0 = 0; b0 < n; b0 += ct) {
        if (nc == kNaMaxChunks) return na_fail(BRT_E_ARG, "too many work chunks");
        h_chunks[nc++] = Chunk{i, (uint32_t)b0, (uint32_t)std::min<uint64_t>(n, b0 + ct), 0u};
      }
    }
    // reduction segments, in point order
    const uint32_t seg_trees = plan_seg_trees(total);
    for (uint32_t i = 0; i < pts->n; ++i) {
      PointRec& r = h_points[i];
      r.seg_begin = ns;
      for (uint64_t b0 = 0; b0 < r.n_trees; b0 += seg_trees) {
        if (ns == kNaMaxSegs) return na_fail(BRT_E_ARG, "too many reduction segments");
        h_segs[ns] = Segment{i, (uint32_t)b0, (uint32_t)std::min<uint64_t>(r.n_trees, b0 + seg_trees), ns};
        ++ns;
      }
      r.seg_count = ns - r.seg_begin;
    }
    // the walker's whole stack in LDS: with pruning a lineage holds at most max_order open vertices
    const int stack_depth = (int)std::max(1u, mc->max_order);
    int wpb = (int)ctx->launch.waves_per_block;
    int maxb = walk_max_blocks_per_cu(precision, dim, u0_kind, (int)n_problems, stack_depth, wpb, (int)mc->strategy);
    while (maxb <= 0 && wpb > 1) {
      wpb -= 1;
      maxb = walk_max_blocks_per_cu(precision, dim, u0_kind, (int)n_problems, stack_depth, wpb, (int)mc->strategy);
    }
    if (maxb <= 0) return na_fail(BRT_E_ARG, "the walker's stack does not fit in LDS");
    int bpc = (int)ctx->launch.blocks_per_cu;
    if (bpc == 0 || bpc > maxb) bpc = maxb;
    const int grid = std::max(1, std::min<int>(bpc * ctx->n_cu, (int)std::max<uint32_t>(1u, nc)));

    void* d_pdes = base + kOffPdes;
    PointRec* d_points = reinterpret_cast<PointRec*>(base + kOffPoints);
    Chunk* d_chunks = reinterpret_cast<Chunk*>(base + kOffChunks);
    Segment* d_segs = reinterpret_cast<Segment*>(base + kOffSegs);
    uint32_t* d_counter = reinterpret_cast<uint32_t*>(base + kOffCounter);
    unsigned long long* d_depth = reinterpret_cast<unsigned long long*>(base + kOffDepth);
    Partial* d_partials = reinterpret_cast<Partial*>(base + kOffPartials);
    unsigned long long* d_seg_nodes = reinterpret_cast<unsigned long long*>(base + kOffSegNodes);
    double* tf = o->tree_f ? reinterpret_cast<double*>(o->tree_f) : reinterpret_cast<double*>(base + kOffTreeF);
    uint32_t* tm = o->tree_meta ? o->tree_meta : reinterpret_cast<uint32_t*>(base + kOffTreeMeta);

    NA_TRY(hipMemcpyAsync(d_pdes, h_pdes, n_problems * pb, hipMemcpyHostToDevice, s));
    if (pts->n) NA_TRY(hipMemcpyAsync(d_points, h_points, pts->n * sizeof(PointRec), hipMemcpyHostToDevice, s));
    if (nc) NA_TRY(hipMemcpyAsync(d_chunks, h_chunks, nc * sizeof(Chunk), hipMemcpyHostToDevice, s));
    if (ns) NA_TRY(hipMemcpyAsync(d_segs, h_segs, ns * sizeof(Segment), hipMemcpyHostToDevice, s));
    NA_TRY(launch_reset(d_counter, d_depth, s));
    if (nc) {
      WalkArgs w{};
      w.points = d_points;
      w.chunks = d_chunks;
      w.n_chunks = nc;
      w.n_problems = n_problems;
      w.pdes = d_pdes;
      w.chunk_counter = d_counter;
      w.depth_counter = d_depth;
      w.tree_f = tf;
      w.tree_meta = tm;
      w.spill = nullptr;
      w.key0 = (uint32_t)(mc->seed & 0xffffffffull);
      w.key1 = (uint32_t)(mc->seed >> 32);
      w.max_order = mc->max_order;
      w.prune = mc->prune;
      w.node_cap = mc->node_cap;
      w.strategy = mc->strategy;
      uint32_t cmod = 0;
      for (uint32_t i = 0; i < n_problems; ++i) cmod |= general_coefficients(problems[i]) ? 1u : 0u;
      w.cmod = cmod;
      w.stack_depth = (uint32_t)stack_depth;
      w.spill_depth = 0;
      w.n_threads = (uint32_t)(grid * wpb * kWave);
      NA_TRY(launch_walk(precision, dim, u0_kind, w, grid, wpb, s));
    }
    ReduceArgs r{};
    r.points = d_points;
    r.segs = d_segs;
    r.n_segs = ns;
    r.tree_f = tf;
    r.tree_meta = tm;
    r.partials = d_partials;
    r.seg_nodes = d_seg_nodes;
    r.n_bins = B;
    NA_TRY(launch_reduce(r, s));
    FinalizeArgs f{};
    f.points = d_points;
    f.n_points = pts->n;
    f.partials = d_partials;
    f.seg_nodes = d_seg_nodes;
    f.n_bins = B;
    f.pade_L = mc->pade_L;
    f.pade_M = mc->pade_M;
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
    NA_TRY(launch_finalize(f, s));
    NA_TRY(hipStreamSynchronize(s));
    unsigned long long deep = 0;
    NA_TRY(hipMemcpy(&deep, d_depth, sizeof(deep), hipMemcpyDeviceToHost));
    if (deep) return set_error(BRT_E_RANGE, "brt_solve_noalloc: %llu trees exceeded the stack depth", deep);
    return BRT_OK;
  });
}
