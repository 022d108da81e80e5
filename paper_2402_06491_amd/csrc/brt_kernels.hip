// HIP tree walker of the random-tree Monte Carlo (Strategy A, Sec. 2.1) for gfx950.
//
//  walk_kernel  persistent, work-stealing: one tree per lane, one node per loop iteration, an
//               explicit per-lane DFS stack (LDS, then a per-thread global spill area), idle lanes
//               refilled from the wave's chunk with ballot/popcount; one record (value, splits,
//               nodes, flags) per tree.
//
// The moment reduction and the FP64 finalize are in brt_moments.hip.  Nothing here is a dense
// contraction, so there is no MFMA work: the kernel is bound by VALU issue (Philox's 32x32->64
// integer multiplies and the transcendentals of Box-Muller, the clock and the weights).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "brt_internal.h"

namespace brt {

// ------------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64 multiplies and
// xors, with the Weyl key schedule.  The key is wave-uniform (kernel argument), so its schedule runs
// on the scalar unit.
// ------------------------------------------------------------------------------------------------
struct U4 {
  uint32_t a, b, c, d;
};

// Three-input xor in one VALU instruction: gfx950's v_bitop3_b32 with truth table 0x96
// (a ^ b ^ c); the compiler otherwise emits two v_xor_b32.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// The same block for a counter (c0, c1, c2, 0) whose first round's product of c2 is given with its xor:
// h1 = hi(M1 c2) ^ c1 ^ k0 and l1 = lo(M1 c2).  The walker's counters (node, tree, point id, 0) keep
// (tree, point id) through a whole tree, so that half of the first round is done once per tree.
__device__ __forceinline__ U4 philox4x32_10_tree(uint32_t c0, uint32_t h1, uint32_t l1, uint32_t k0, uint32_t k1) {
  const uint64_t q = (uint64_t)0xD2511F53u * (uint64_t)c0;
  uint32_t a0 = h1, a1 = l1, a2 = (uint32_t)(q >> 32) ^ k1, a3 = (uint32_t)q;
  k0 += 0x9E3779B9u;
  k1 += 0xBB67AE85u;
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)a0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)a2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), a1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), a3, k1);
    a1 = (uint32_t)p1;
    a3 = (uint32_t)p0;
    a0 = n0;
    a2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{a0, a1, a2, a3};
}

// ------------------------------------------------------------------------------------------------
// Precision-dependent elementary functions.
// FP32: hardware log2/exp2/sqrt/sin/cos/rcp (v_log_f32, v_exp_f32, v_sqrt_f32, v_sin_f32, v_cos_f32,
// v_rcp_f32; the sin/cos units take their argument in revolutions, which is exactly the Box-Muller
// angle u2).  FP64: the device math library.
// ------------------------------------------------------------------------------------------------
template <typename Real>
struct Math;

template <>
struct Math<float> {
  static __device__ __forceinline__ float ln(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
  static __device__ __forceinline__ float ex(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
  static __device__ __forceinline__ float sq(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  // sin and cos of 2*pi*u for u in [0, 1)
  static __device__ __forceinline__ void sincos_rev(float u, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
  }
  static __device__ __forceinline__ float cos_rev(float u) { return __builtin_amdgcn_cosf(u); }
  static __device__ __forceinline__ float cos_half_pi(float v) {  // cos(pi v / 2) = cos(2 pi (v/4))
    return __builtin_amdgcn_cosf(0.25f * v);
  }
};

template <>
struct Math<double> {
  static __device__ __forceinline__ double ln(double x) { return log(x); }
  static __device__ __forceinline__ double ex(double x) { return exp(x); }
  static __device__ __forceinline__ double sq(double x) { return sqrt(x); }
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
  static __device__ __forceinline__ void sincos_rev(double u, double* s, double* c) { sincospi(2.0 * u, s, c); }
  static __device__ __forceinline__ double cos_rev(double u) { return cospi(2.0 * u); }
  static __device__ __forceinline__ double cos_half_pi(double v) { return cospi(0.5 * v); }
};

// ------------------------------------------------------------------------------------------------
// Initial data g at the end of a leaf path.
// ------------------------------------------------------------------------------------------------
// The problem constants the node step reads every time.  With one problem per launch they are loaded
// once, before the loop, and stay in scalar registers; with several they come from the LDS table.
template <typename Real>
struct HotC {
  Real sigma, inv_lambda, mu, inv_q, s_scale;
  uint32_t K, jpack, q_lo, cmod, cm_pow, drift_on, sde;
  Real cm_bx, cm_by, cm_t0, drift0, drift1;
  Real dlin0, dlin1, sig_amp, sig_k, inv_h;  // a general L (Euler-Maruyama edges)
  Real g[6];  // first initial-data parameters (the logistic family's A, s, x0, p, n0, n1)
  Real omega0;  // the first term's vertex weight (the only one when K == 1)
};

template <typename Real>
__device__ __forceinline__ HotC<Real> hot_of(const PdeT<Real>& pd) {
  HotC<Real> h;
  h.sigma = pd.sigma;
  h.inv_lambda = pd.inv_lambda;
  h.mu = pd.mu;
  h.inv_q = pd.inv_q;
  h.s_scale = pd.s_scale;
  h.K = pd.K;
  h.jpack = pd.jpack;
  h.q_lo = pd.q_lo;
  h.cmod = pd.cmod;
  h.cm_pow = pd.cm_pow;
  h.cm_bx = pd.cm_bx;
  h.cm_by = pd.cm_by;
  h.cm_t0 = pd.cm_t0;
  h.drift_on = pd.drift_on;
  h.drift0 = pd.drift[0];
  h.drift1 = pd.drift[1];
  h.sde = pd.sde;
  h.dlin0 = pd.dlin[0];
  h.dlin1 = pd.dlin[1];
  h.sig_amp = pd.sig_amp;
  h.sig_k = pd.sig_k;
  h.inv_h = pd.inv_h;
  for (int i = 0; i < 6; ++i) h.g[i] = pd.u0[i];
  h.omega0 = pd.omega[0];
  return h;
}

// Logistic initial data A (1 + e^{s (n.x - x0)})^{-p}, split around its exponential; g = (A, s, x0, p, n0, n1).
template <typename Real, int DIM>
__device__ __forceinline__ Real logistic_arg(const Real* g, const Real* x) {
  Real nx = x[0] * g[4];
  if constexpr (DIM == 2) nx += x[1] * g[5];
  return g[1] * (nx - g[2]);
}

template <typename Real>
__device__ __forceinline__ Real logistic_finish(const Real* g, Real e) {
  const Real base = Math<Real>::rcp((Real)1 + e);
  Real r = base;
  const int pw = (int)g[3];
  for (int i = 1; i < pw; ++i) r *= base;
  return g[0] * r;
}

template <typename Real, int DIM, int U0>
__device__ __forceinline__ Real eval_g(const Real* p, uint32_t nterms, const Real* x) {
  if constexpr (U0 == 0) {
    return p[0];
  } else if constexpr (U0 == 1) {
    return logistic_finish<Real>(p, Math<Real>::ex(logistic_arg<Real, DIM>(p, x)));
  } else if constexpr (U0 == 2) {
    Real acc = 0;
    for (uint32_t k = 0; k < nterms; ++k) {
      const Real* q = p + 4 * k;
      const Real dx = x[0] - q[1];
      Real r2 = dx * dx;
      if constexpr (DIM == 2) {
        const Real dy = x[1] - q[2];
        r2 += dy * dy;
      }
      acc += q[0] * Math<Real>::ex(-r2 * q[3]);  // q[3] holds 1/(2 s^2) on the device
    }
    return acc;
  } else {
    const Real ax = x[0] < 0 ? -x[0] : x[0];
    if (ax > p[1]) return 0;
    const Real cx = Math<Real>::cos_half_pi(x[0] / p[1]);
    Real v = p[0] * cx * cx;
    if constexpr (DIM == 2) {
      const Real ay = x[1] < 0 ? -x[1] : x[1];
      if (ay > p[2]) return 0;
      const Real cy = Math<Real>::cos_half_pi(x[1] / p[2]);
      v *= cy * cy;
    }
    return v;
  }
}

// One edge of a general L = sigma(x)^2/2 Lap + b(x) . grad (Sec. 2.1's SDE, the Euler scheme of Sec. 2.4):
// n = ceil(dt / h) (at most kMaxEulerSteps) equal Euler-Maruyama steps, which end at the edge's end (its branching time), with
// b(x) = drift + dlin x and sigma(x) = sigma (1 + sig_amp e^{-sig_k |x|^2}).  Step 0 uses the node's own
// normals (radius r0, angle cos/sin c0, s0), step k the Philox block (node, tree, point, k).
template <typename Real, int DIM>
__device__ __forceinline__ void euler_edge(const HotC<Real>& hc, const Real* x, Real dt, Real r0, Real c0, Real s0,
                                           uint32_t node, uint32_t tree, uint32_t pid, uint32_t k0, uint32_t k1,
                                           Real* out) {
  const Real nf = ceil(dt * hc.inv_h);
  const uint32_t n = nf < (Real)1 ? 1u : nf > (Real)kMaxEulerSteps ? kMaxEulerSteps : (uint32_t)nf;
  const Real h = dt / (Real)n, sh = Math<Real>::sq(h);
  Real y0 = x[0], y1 = DIM == 2 ? x[1] : (Real)0;
  Real za = r0 * c0, zb = r0 * s0;
  for (uint32_t k = 0; k < n; ++k) {
    if (k > 0) {
      const U4 v = philox4x32_10(node, tree, pid, k, k0, k1);
      const Real u1 = ((Real)v.c + (Real)0.5) * (Real)0x1p-32;
      const Real u2 = (Real)v.d * (Real)0x1p-32;
      const Real r = Math<Real>::sq((Real)-2 * Math<Real>::ln(u1));
      Real sn, cs;
      Math<Real>::sincos_rev(u2, &sn, &cs);
      za = r * cs;
      zb = r * sn;
    }
    Real r2 = y0 * y0;
    if constexpr (DIM == 2) r2 += y1 * y1;
    const Real sg = hc.sigma * ((Real)1 + hc.sig_amp * Math<Real>::ex(-hc.sig_k * r2));
    const Real i0 = (hc.drift0 + hc.dlin0 * y0) * h + sg * sh * za;
    const Real i1 = (hc.drift1 + hc.dlin1 * y1) * h + sg * sh * zb;
    y0 += i0;
    if constexpr (DIM == 2) y1 += i1;
  }
  out[0] = y0;
  out[1] = DIM == 2 ? y1 : x[1];
}

template <typename Real, int DIM>
__host__ __device__ constexpr size_t stack_entry_bytes() {
  return sizeof(double) + (DIM + 1) * sizeof(Real) + 1;
}

// LDS bytes of one stack level of one lane.  Strategy A keeps the lineage's clock product (the time left
// follows from it, t + ln(P)/lambda); Strategy B, which has no clock, keeps the time left instead.
template <typename Real, int DIM, int STRAT>
__host__ __device__ constexpr size_t stack_lds_entry_bytes() {
  return (STRAT == 0 ? sizeof(double) : sizeof(Real)) + DIM * sizeof(Real) + 1;
}

// LDS bytes of a launch's problem table: n full records, or (u0_stride > 0, a family of problems that
// differ only in their initial data) the first problem's record, then every problem's number of
// initial-data terms and its first u0_stride initial-data parameters.
__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }
template <typename Real>
__host__ __device__ constexpr size_t pde_table_bytes(int n, int u0_stride = 0) {
  return u0_stride == 0 ? align16((size_t)n * sizeof(PdeT<Real>))
                        : align16(sizeof(PdeT<Real>)) + align16((size_t)n * sizeof(uint32_t)) +
                              align16((size_t)n * (size_t)u0_stride * sizeof(Real));
}

// Wave-uniform copies (scalar registers) of values loaded from a wave-uniform address.
__device__ __forceinline__ uint32_t rfl_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t rfl_u64(uint64_t v) {
  return ((uint64_t)rfl_u32((uint32_t)(v >> 32)) << 32) | rfl_u32((uint32_t)v);
}
__device__ __forceinline__ double rfl_f64(double v) { return __builtin_bit_cast(double, rfl_u64(__builtin_bit_cast(uint64_t, v))); }
// An empty statement that reads a register: the compiler completes the load that wrote it first.
__device__ __forceinline__ void consume(double v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void consume(float v) { asm volatile("" ::"v"(v)); }

// ------------------------------------------------------------------------------------------------
// Per-lane DFS stack.  An entry is pushed for each vertex that still has children to start: the
// state its children depart from (clock product P, position, time left) and the number of children
// not yet started.  The top `lds_depth` levels live in LDS (structure of arrays, one slot per lane so
// lanes never conflict); deeper levels go to the thread's own slice of a global spill area.
// ------------------------------------------------------------------------------------------------
#define BRT_LDS __attribute__((address_space(3)))

template <typename Real, int DIM, int STRAT>
struct Stack {
  // LDS pointers carry their address space so that the compiler keeps ds_* instructions for them
  // instead of merging both tiers into generic (flat) accesses through a selected pointer.  LDS levels
  // hold P (Strategy A) or T (Strategy B), never both; the spill levels keep the full layout.
  BRT_LDS double* P;   // [lds_depth][64], Strategy A
  BRT_LDS Real* X;     // [DIM][lds_depth][64]
  BRT_LDS Real* T;     // [lds_depth][64], Strategy B
  BRT_LDS uint8_t* R;  // [lds_depth][64]
  double* gP;          // this thread's spill levels: [spill_depth]
  Real* gX;            // [DIM][spill_depth]
  Real* gT;            // [spill_depth]
  uint8_t* gR;         // [spill_depth]
  uint32_t lds_depth, spill_depth, lane;

  __device__ __forceinline__ void push(uint32_t sp, double p, const Real* x, Real t, uint32_t rem) {
    if (sp < lds_depth) {
      const uint32_t o = sp * kWave + lane;
      if constexpr (STRAT == 0) P[o] = p;
      else T[o] = t;
      X[o] = x[0];
      if constexpr (DIM == 2) X[lds_depth * kWave + o] = x[1];
      R[o] = (uint8_t)rem;
    } else {
      const uint32_t o = sp - lds_depth;
      if constexpr (STRAT == 0) gP[o] = p;
      else gT[o] = t;
      gX[o] = x[0];
      if constexpr (DIM == 2) gX[spill_depth + o] = x[1];
      gR[o] = (uint8_t)rem;
    }
  }
  // Read the top entry (level sp-1) into the departure state (P for Strategy A, whose time left the
  // caller derives from it; the time left for Strategy B); returns the number of children still to
  // start after the one about to be visited, and stores it back.
  __device__ __forceinline__ uint32_t top(uint32_t sp, double* p, Real* x, Real* t) {
    const uint32_t lv = sp - 1;
    uint32_t rem;
    if (lv < lds_depth) {
      const uint32_t o = lv * kWave + lane;
      if constexpr (STRAT == 0) *p = P[o];
      else *t = T[o];
      x[0] = X[o];
      if constexpr (DIM == 2) x[1] = X[lds_depth * kWave + o];
      rem = (uint32_t)R[o] - 1u;
      R[o] = (uint8_t)rem;
    } else {
      const uint32_t o = lv - lds_depth;
      if constexpr (STRAT == 0) *p = gP[o];
      else *t = gT[o];
      x[0] = gX[o];
      if constexpr (DIM == 2) x[1] = gX[spill_depth + o];
      rem = (uint32_t)gR[o] - 1u;
      gR[o] = (uint8_t)rem;
      // Consume the loaded values in this (rare) branch: the wait for them is then placed here, and
      // the common path, where the merged values are used, waits on no memory counter (which on this
      // architecture also counts the record stores).
      if constexpr (STRAT == 0) consume(*p);
      else consume(*t);
      consume(x[0]);
      if constexpr (DIM == 2) consume(x[1]);
    }
    return rem;
  }
};

// ------------------------------------------------------------------------------------------------
// The walker.  TAB: kOneProblem, the problem constants are loop invariants; kProblemTable, several
// problems, each lane reads its tree's problem from the LDS table; kFamily, several problems that differ
// only in their initial data (the constants of the node step are loop invariants, a leaf reads its
// problem's initial-data parameters from the LDS table).  MODE bit 0 (STRAT): Strategy A (0, Sec. 2.1) or B (1, Sec. 2.2);
// bit 1 (CMOD): some problem of the launch has variable coefficients or a drift, so the variants for
// constant coefficients and L = a Lap carry no trace of them.
// ------------------------------------------------------------------------------------------------
template <typename Real, int DIM, int U0, int TAB, int MODE>
__global__ __launch_bounds__(kMaxWalkThreads) void walk_kernel(WalkArgs a) {
  constexpr bool MULTI = TAB == kProblemTable;
  constexpr int STRAT = MODE & 1;
  constexpr bool CMOD = (MODE & 2) != 0;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  // problem table -> LDS
  PdeT<Real>* pdes = reinterpret_cast<PdeT<Real>*>(smem);
  const uint32_t u0s = TAB == kFamily ? a.u0_stride : 0u;
  uint32_t* fam_nt = reinterpret_cast<uint32_t*>(smem + align16(sizeof(PdeT<Real>)));
  Real* fam_u0 = reinterpret_cast<Real*>(smem + align16(sizeof(PdeT<Real>)) + align16(a.n_problems * sizeof(uint32_t)));
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.pdes);
    uint32_t* dst = reinterpret_cast<uint32_t*>(smem);
    const uint32_t words = (uint32_t)((TAB == kFamily ? 1u : a.n_problems) * sizeof(PdeT<Real>) / 4);
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
    if constexpr (TAB == kFamily) {
      const PdeT<Real>* gp = reinterpret_cast<const PdeT<Real>*>(a.pdes);
      for (uint32_t i = threadIdx.x; i < a.n_problems; i += blockDim.x) fam_nt[i] = gp[i].u0_nterms;
      for (uint32_t i = threadIdx.x; i < a.n_problems * u0s; i += blockDim.x) fam_u0[i] = gp[i / u0s].u0[i % u0s];
    }
  }
  __syncthreads();

  const uint32_t lane = __lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  Stack<Real, DIM, STRAT> st;
  {
    const uint32_t depth = a.stack_depth;
    unsigned char* wbase = smem + pde_table_bytes<Real>((int)a.n_problems, (int)u0s) +
                           (size_t)wave * depth * kWave * stack_lds_entry_bytes<Real, DIM, STRAT>();
    // Strategy A: [P double][X DIM reals][R bytes]; Strategy B: [X DIM reals][T reals][R bytes]
    st.P = (BRT_LDS double*)(wbase);
    st.X = STRAT == 0 ? (BRT_LDS Real*)(st.P + depth * kWave) : (BRT_LDS Real*)(wbase);
    st.T = st.X + DIM * depth * kWave;
    st.R = STRAT == 0 ? (BRT_LDS uint8_t*)(st.X + DIM * depth * kWave) : (BRT_LDS uint8_t*)(st.T + depth * kWave);
    // spill area: per thread, stride-1 levels (deep levels are rare, so coalescing does not matter)
    const size_t gtid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t sd = (size_t)a.spill_depth * a.n_threads;
    const size_t me = gtid * a.spill_depth;
    st.gP = reinterpret_cast<double*>(a.spill) + me;
    st.gX = reinterpret_cast<Real*>(reinterpret_cast<double*>(a.spill) + sd) + DIM * me;
    st.gT = reinterpret_cast<Real*>(reinterpret_cast<double*>(a.spill) + sd) + DIM * sd + me;
    st.gR = reinterpret_cast<uint8_t*>(reinterpret_cast<Real*>(reinterpret_cast<double*>(a.spill) + sd) + (DIM + 1) * sd) + me;
    st.lds_depth = depth;
    st.spill_depth = a.spill_depth;
    st.lane = lane;
  }
  const uint32_t max_depth = a.stack_depth + a.spill_depth;

  // one problem: its constants loaded once (uniform, scalar registers)
  const HotC<Real> h0 = hot_of(*reinterpret_cast<const PdeT<Real>*>(a.pdes));
  const uint32_t node_cap = a.node_cap;
  const uint32_t max_order = a.max_order;
  const bool prune = a.prune != 0;

  // Wave-uniform chunk cursor and the constants of the chunk's point, held in scalar registers: a
  // refill copies them into the new lanes without touching memory.  The index of the chunk after
  // the current one is requested as soon as the current one starts.
  uint32_t c_next = 0, c_end = 0;
  bool more = true;
  uint32_t c_pid = 0, c_pde = 0, c_tfirst = 0, c_ph = 0, c_pl = 0;
  uint64_t c_base = 0;
  double c_theta = 1.0;
  Real c_t = 0, c_x0 = 0, c_x1 = 0;
  uint32_t next_raw = 0;
  if (lane == 0) next_raw = atomicAdd(a.chunk_counter, 1u);

  // which lanes hold a tree (wave-uniform, in scalar registers)
  uint64_t amask = 0;
  // The variants with general coefficients leave the node step early on lanes without a tree (a
  // divergent continue), after which the lanes' copies of a carried mask would differ: they rebuild
  // the mask from this per-lane flag at the top of every step instead, where all lanes have met.
  bool live = false;
  // per-lane tree state
  uint32_t tree = 0, node = 0, ne = 0, flags = 0, sp = 0, pid = 0, pde_lane = 0;
  uint32_t ph = 0, pl = 0;  // the tree's share of the first Philox round (philox4x32_10_tree)
  uint64_t rec = 0;
  double P = 1.0, theta = 1.0;
  double F = 1.0;  // running product of the tree's factors (FP64 for range: weights reach e^{32} per vertex)
  Real tau = 0;
  Real troot = 0;  // the point's time: Strategy A derives a sibling's time left from it and the clock product
  Real x[2] = {0, 0};

  while (true) {
    // ---- refill: idle lanes take trees from the wave's chunk; at most one chunk switch per
    // iteration (lanes left without a tree at a chunk boundary wait one node step).  Which lanes hold
    // a tree is the wave-uniform mask `amask` (scalar registers); a lane reads its bit through
    // inverse_ballot. ----
    if constexpr (CMOD) amask = __ballot(live);
    const uint64_t need = ~amask;
    if (need != 0 && more) {
      if (c_next == c_end) {
        const uint32_t ci = __builtin_amdgcn_readfirstlane(next_raw);
        if (ci >= a.n_chunks) {
          more = false;
        } else {
          if (lane == 0) next_raw = atomicAdd(a.chunk_counter, 1u);
          const Chunk ch = a.chunks[ci];
          c_next = __builtin_amdgcn_readfirstlane(ch.begin);
          c_end = __builtin_amdgcn_readfirstlane(ch.end);
          const uint32_t point = __builtin_amdgcn_readfirstlane(ch.point);
          // The point's constants are made wave-uniform here, so that the loads complete at the chunk
          // switch: a load still pending in a vector register would make later code wait on the
          // counter that also counts the record stores (vmcnt), in every node step.
          const PointRec& pr = a.points[point];
          c_pid = rfl_u32(pr.point_id);
          const uint64_t pq = (uint64_t)0xCD9E8D57u * (uint64_t)c_pid;  // the first Philox round's point part
          c_ph = (uint32_t)(pq >> 32) ^ a.key0;
          c_pl = (uint32_t)pq;
          c_pde = rfl_u32(pr.pde);
          c_tfirst = rfl_u32(pr.tree_first);
          c_base = rfl_u64(pr.tree_base);
          c_theta = rfl_f64(pr.theta);
          c_t = (Real)rfl_f64(pr.t);
          c_x0 = (Real)rfl_f64(pr.x[0]);
          c_x1 = (Real)rfl_f64(pr.x[1]);
        }
      }
      if (more) {
        const uint32_t avail = c_end - c_next;
        const uint32_t cnt = (uint32_t)__popcll(need);
        const uint32_t take = cnt < avail ? cnt : avail;
        // the lane's rank among the idle lanes; the `take` lowest idle lanes get the next trees
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
        const uint64_t got = need & __ballot(rank < take);
        if (__builtin_amdgcn_inverse_ballot_w64(got)) {
          tree = c_tfirst + c_next + rank;
          pid = c_pid;
          ph = c_ph ^ tree;
          pl = c_pl;
          pde_lane = c_pde;
          rec = c_base + c_next + rank;
          theta = c_theta;
          tau = c_t;
          troot = c_t;
          x[0] = c_x0;
          x[1] = c_x1;
          P = 1.0;
          F = 1.0;
          node = 0;
          ne = 0;
          flags = 0;
          sp = 0;
          live = true;
        }
        amask |= got;
        c_next += take;
      }
    }
    // No lane holds a tree only when the chunks are used up (or the wave met an empty chunk: it then
    // takes one guarded step on stale state and refills again).
    if (amask == 0 && !more) break;
    const bool active = __builtin_amdgcn_inverse_ballot_w64(amask);
    // Lanes without a tree step along on their stale state (no memory effects: push, pop and record
    // are guarded), which keeps the node step free of a divergent exit; the variants with general
    // coefficients skip them, as their Euler edges take a data-dependent number of steps.
    if constexpr (CMOD) {
      if (!active) continue;
    }

    const PdeT<Real>& pd = pdes[MULTI ? pde_lane : 0u];  // per-arity weights and the other data families
    const HotC<Real> hc = MULTI ? hot_of(pd) : h0;

    // ---- one node of this lane's tree ----
    // Vertex and leaf quantities are computed for every lane and chosen with selects; only the stack
    // push, the stack pop and the record write are divergent.
    const bool capped = node >= node_cap;
    const U4 w = philox4x32_10_tree(node, ph, pl, a.key0, a.key1);
    double Pn = P;
    bool vertex;
    Real S;     // time from the node's start to its split
    Real tau2;  // time left after the split
    if constexpr (STRAT == 0) {
      // Strategy A: Exp(lambda) clock; vertex iff the lineage's product of uniforms exceeds theta
      const double U = fma((double)w.a, 0x1p-32, 0x1p-33);  // (w0 + 1/2) 2^-32, exact
      Pn = P * U;
      vertex = !capped && Pn > theta;
      S = -Math<Real>::ln((Real)U) * hc.inv_lambda;
      tau2 = tau - S;
      tau2 = tau2 < (Real)0 ? (Real)0 : tau2;
    } else {
      // Strategy B: coin w0 >= Q; the split comes after the fraction V = (w0 - Q + 1/2)/(2^32 - Q)
      // of tau.  tau (1 - V) comes from the complementary count 2^32 - w0 - 1/2, free of the
      // cancellation of tau - S near V = 1 (it multiplies the weights of the vertex's children).
      vertex = !capped && w.a > hc.q_lo;
      const Real ts = tau * hc.s_scale;
      S = ((Real)(w.a - hc.q_lo - 1u) + (Real)0.5) * ts;
      tau2 = ((Real)(~w.a) + (Real)0.5) * ts;
    }

    // Box-Muller radius and the Brownian scale under one square root: sigma sqrt(-2 ln(u1) dt) with
    // dt = S on the way to a split, tau to a leaf
    const Real u1 = ((Real)w.c + (Real)0.5) * (Real)0x1p-32;
    const Real u2 = (Real)w.d * (Real)0x1p-32;
    // 1-D paths use the cosine half of the Box-Muller pair only (an Euler edge's first step in 2-D uses both)
    Real sn = 0, cs;
    if constexpr (DIM == 2)
      Math<Real>::sincos_rev(u2, &sn, &cs);
    else
      cs = Math<Real>::cos_rev(u2);
    const Real dt = vertex ? S : tau;
    const Real sdr = hc.sigma * Math<Real>::sq((Real)-2 * Math<Real>::ln(u1) * dt);
    Real xn[2];
    xn[0] = x[0] + sdr * cs;
    xn[1] = DIM == 2 ? x[1] + sdr * sn : x[1];
    if constexpr (CMOD) {
      if (hc.sde) {
        // a general L: the edge is integrated by Euler-Maruyama steps instead
        euler_edge<Real, DIM>(hc, x, dt, Math<Real>::sq((Real)-2 * Math<Real>::ln(u1)), cs, sn, node, tree, pid, a.key0,
                              a.key1, xn);
      } else if (hc.drift_on) {
        // constant drift: the edge also moves by b dt (exact for L = a Lap + b . grad)
        xn[0] += hc.drift0 * dt;
        if constexpr (DIM == 2) xn[1] += hc.drift1 * dt;
      }
    }

    // one exponential per node: the vertex weight e^{(alpha-1) mu tau'} or, for logistic initial
    // data, e^{s (n.x - x0)} at the leaf
    const uint32_t idx = __umulhi(w.b, hc.K);
    const uint32_t alpha = (hc.jpack >> (4 * idx)) & 15u;
    Real earg = (Real)((int)alpha - 1) * hc.mu * tau2;
    // variable coefficients: c_j exp(-bx x^2 - by y^2) (tau' + t0)^(-pow) at the split, folded into the
    // vertex's exponential
    Real cscale = (Real)1;
    if constexpr (CMOD) {
      if (hc.cmod) {
        earg -= hc.cm_bx * (xn[0] * xn[0]) + (DIM == 2 ? hc.cm_by * (xn[1] * xn[1]) : (Real)0);
        if (hc.cm_pow) cscale = (Real)1 / (tau2 + hc.cm_t0);
      }
    }
    // the initial data's parameters: the lane's problem's (a family's table) or the problem's
    const Real* g;
    if constexpr (TAB == kFamily)
      g = fam_u0 + pde_lane * u0s;
    else if constexpr (U0 == 1)
      g = hc.g;
    else
      g = pd.u0;
    if constexpr (U0 == 1) earg = vertex ? earg : logistic_arg<Real, DIM>(g, xn);
    const Real E = Math<Real>::ex(earg);
    // Strategy B's vertex weight carries the time left tau (eta(t) = t) and its leaves divide by q
    const Real wscale = (STRAT == 1 ? tau : (Real)1) * cscale;
    const Real lscale = STRAT == 1 ? hc.inv_q : (Real)1;
    // the chosen term's weight from the table; with logistic initial data, one problem and one non-linear
    // term it is a loop invariant (the other families keep the table read: there the branch around it
    // costs the walker registers)
    Real factor;
    if constexpr (U0 == 1) {
      Real om;
      if (!MULTI && hc.K == 1)
        om = hc.omega0;
      else
        om = pd.omega[idx];
      factor = vertex ? wscale * om * E : lscale * logistic_finish<Real>(g, E);
    } else {
      if (vertex)
        factor = wscale * pd.omega[idx] * E;
      else
        factor = lscale * eval_g<Real, DIM, U0>(g, TAB == kFamily ? fam_nt[pde_lane] : pd.u0_nterms, xn);
    }

    ne += vertex ? 1u : 0u;
    const bool ovf = vertex && prune && ne > max_order;
    const bool vok = vertex && !ovf;
    flags |= (capped ? kMetaCapped : 0u) | (ovf ? kMetaOverflow : 0u);
    node += capped ? 0u : 1u;
    F *= (double)factor;
    bool done = capped || ovf;
    if (active && vok && alpha >= 2) {
      if (sp == max_depth) {
        flags |= kMetaDepth;
        done = true;
      } else {
        st.push(sp, Pn, xn, tau2, alpha - 1);
        sp += 1;
      }
    }
    const bool cont = vok && alpha > 0;  // the vertex's first child departs from the split point
    x[0] = cont ? xn[0] : x[0];
    if constexpr (DIM == 2) x[1] = cont ? xn[1] : x[1];
    P = cont ? Pn : P;
    tau = cont ? tau2 : tau;
    const bool branch_end = active && !done && !cont;  // a leaf, or a vertex without children
    if (branch_end) {
      if (sp == 0) {
        done = true;
      } else {
        const uint32_t rem = st.top(sp, &P, x, &tau);
        if (rem == 0) sp -= 1;
        if constexpr (STRAT == 0) {
          // the time left at the split: the point's time less the lineage's exponential times, which
          // sum to -ln(P)/lambda
          const Real tl = troot + Math<Real>::ln((Real)P) * hc.inv_lambda;
          tau = tl < (Real)0 ? (Real)0 : tl;
        }
      }
    }
    const bool fin = active && done;
    if (fin) {
      a.tree_f[rec] = flags ? 0.0 : F;
      a.tree_meta[rec] = (ne < 255u ? ne : 255u) | flags | (node << kMetaNodesShift);
      if (flags & kMetaDepth) atomicAdd(a.depth_counter, 1ull);
    }
    if constexpr (CMOD) {
      if (fin) live = false;
    } else {
      amask &= ~__ballot(fin);
    }
  }
}

__global__ void reset_kernel(uint32_t* chunk_counter, unsigned long long* depth_counter) {
  if (threadIdx.x == 0) {
    *chunk_counter = 0u;
    *depth_counter = 0ull;
  }
}

// ------------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------------
size_t stack_entry_size(int precision, int dim) {
  if (precision == 32) return dim == 1 ? stack_entry_bytes<float, 1>() : stack_entry_bytes<float, 2>();
  return dim == 1 ? stack_entry_bytes<double, 1>() : stack_entry_bytes<double, 2>();
}

template <typename Real>
static size_t lds_entry(int dim, int strategy) {
  if (dim == 1) return strategy ? stack_lds_entry_bytes<Real, 1, 1>() : stack_lds_entry_bytes<Real, 1, 0>();
  return strategy ? stack_lds_entry_bytes<Real, 2, 1>() : stack_lds_entry_bytes<Real, 2, 0>();
}

size_t walk_lds_bytes(int precision, int dim, int stack_depth, int waves_per_block, int n_problems, int strategy,
                      int u0_stride) {
  const size_t sd = (size_t)stack_depth * kWave * waves_per_block;
  const int us = n_problems > 1 ? u0_stride : 0;
  if (precision == 32) return pde_table_bytes<float>(n_problems, us) + sd * lds_entry<float>(dim, strategy);
  return pde_table_bytes<double>(n_problems, us) + sd * lds_entry<double>(dim, strategy);
}

template <typename Real, int DIM, int U0, int TAB, int MODE>
static const void* walk_ptr() {
  return reinterpret_cast<const void*>(&walk_kernel<Real, DIM, U0, TAB, MODE>);
}

template <typename Real, int DIM, int TAB, int MODE>
static const void* walk_ptr_u0(int u0) {
  switch (u0) {
    case 0: return walk_ptr<Real, DIM, 0, TAB, MODE>();
    case 1: return walk_ptr<Real, DIM, 1, TAB, MODE>();
    case 2: return walk_ptr<Real, DIM, 2, TAB, MODE>();
    default: return walk_ptr<Real, DIM, 3, TAB, MODE>();
  }
}

template <typename Real, int DIM, int MODE>
static const void* walk_ptr_tab(int u0, int tab) {
  switch (tab) {
    case kOneProblem: return walk_ptr_u0<Real, DIM, kOneProblem, MODE>(u0);
    case kProblemTable: return walk_ptr_u0<Real, DIM, kProblemTable, MODE>(u0);
    default: return walk_ptr_u0<Real, DIM, kFamily, MODE>(u0);
  }
}

template <typename Real, int DIM>
static const void* walk_ptr_m(int u0, int tab, int mode) {
  switch (mode) {
    case 0: return walk_ptr_tab<Real, DIM, 0>(u0, tab);
    case 1: return walk_ptr_tab<Real, DIM, 1>(u0, tab);
    case 2: return walk_ptr_tab<Real, DIM, 2>(u0, tab);
    default: return walk_ptr_tab<Real, DIM, 3>(u0, tab);
  }
}

// The table mode of a launch of n problems (u0_stride > 0: they form a family).
static int walk_tab(int n_problems, int u0_stride) {
  return n_problems <= 1 ? kOneProblem : (u0_stride > 0 ? kFamily : kProblemTable);
}

static const void* walk_fn(int precision, int dim, int u0, int tab, int mode) {
  if (precision == 32)
    return dim == 1 ? walk_ptr_m<float, 1>(u0, tab, mode) : walk_ptr_m<float, 2>(u0, tab, mode);
  return dim == 1 ? walk_ptr_m<double, 1>(u0, tab, mode) : walk_ptr_m<double, 2>(u0, tab, mode);
}

int walk_max_blocks_per_cu(int precision, int dim, int u0_kind, int n_problems, int stack_depth, int waves_per_block,
                           int strategy, int u0_stride) {
  int nb = 0;
  const size_t lds = walk_lds_bytes(precision, dim, stack_depth, waves_per_block, n_problems, strategy, u0_stride);
  const int tab = walk_tab(n_problems, u0_stride);
  // the smaller occupancy of the strategy's variants with and without variable coefficients, so a grid
  // sized by it stays resident
  int best = 1 << 30;
  for (int mode = strategy; mode < 4; mode += 2) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_fn(precision, dim, u0_kind, tab, mode),
                                                     waves_per_block * kWave, lds) != hipSuccess)
      return 0;
    best = nb < best ? nb : best;
  }
  return best;
}

hipError_t launch_reset(uint32_t* chunk_counter, unsigned long long* depth_counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, chunk_counter, depth_counter);
  return hipGetLastError();
}

hipError_t launch_walk(int precision, int dim, int u0_kind, const WalkArgs& a, int grid, int waves_per_block,
                       hipStream_t s) {
  const size_t lds = walk_lds_bytes(precision, dim, (int)a.stack_depth, waves_per_block, (int)a.n_problems,
                                    (int)a.strategy, (int)a.u0_stride);
  const void* fn = walk_fn(precision, dim, u0_kind, walk_tab((int)a.n_problems, (int)a.u0_stride),
                           (int)(a.strategy | (a.cmod ? 2u : 0u)));
  void* args[] = {const_cast<WalkArgs*>(&a)};
  return hipLaunchKernel(fn, dim3(grid), dim3(waves_per_block * kWave), args, lds, s);
}

}  // namespace brt
