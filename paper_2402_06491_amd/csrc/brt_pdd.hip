// Domain decomposition tail (Sec. 3): interpolation of the Monte Carlo node values into boundary data
// (tensor-product not-a-knot cubic splines) and the decoupled subdomain solves (Crank-Nicolson in
// Peaceman-Rachford ADI form), FP64 throughout.
//
// Kernels
//   spline_rows_kernel  one thread per (line, node time): spline moments along the line
//   spline_s_kernel     one thread per (line, node time, fine node): values along the line
//   spline_t_kernel     one thread per (line, fine node): spline in time, written at every time level
//   init_field_kernel   u0 at every grid node, line data at level 0
//   adi_kernel          persistent cooperative launch through all time steps: per step an x phase and
//                       a y phase, each followed by a barrier (among the blocks of a die when the dies
//                       own whole subdomains, else over the grid); a work item is 32 lines of one
//                       subdomain (16 for lines of more than 512 unknowns) held in LDS by one block,
//                       each line's tridiagonal system solved by 32 threads (segments of consecutive
//                       unknowns joined by scans of their carries); the x phase also forms the y
//                       phase's right-hand sides.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "brt.h"
#include "brt_api.h"
#include "brt_internal.h"

using brt::set_error;

namespace {

constexpr uint32_t kMaxSub = 64;
constexpr uint32_t kMaxCells = 1024;
constexpr uint32_t kMaxNodesPerLine = 257;
constexpr uint32_t kMaxNt = 63;
constexpr double kBarrierSeconds = 5.0;
// Solver fields are stored with a row pitch of a multiple of 16 doubles and column 1 (the first
// interior column) on a 128-byte boundary, so that the solver's 16-column strips and 64-column row
// tiles map onto whole cache lines.
constexpr uint32_t kFieldLead = 15;  // doubles before column 0
constexpr uint32_t kXcds = 8;        // workgroups are dealt to the accelerator's dies round-robin
constexpr uint32_t kMaxGroups = 512;             // barrier groups of a launch
constexpr uint32_t kSyncWords = 4 + 2 * kMaxGroups;  // abort word, then arrivals and die mask per group

#define PDD_TRY(expr)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return set_error(BRT_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct LineDev {
  uint32_t orient;    // 0 vertical, 1 horizontal
  uint32_t k;         // index of the cut along x (vertical) or y (horizontal)
  uint32_t n_fine;    // fine nodes along the line
  uint32_t ns;        // interpolation nodes along the line
  uint64_t bd_off;    // offset (doubles) of time level 0 in the boundary data
  uint64_t node_off;  // index of the line's first node value
  double c;           // x of a vertical line, y of a horizontal one
  double s_lo;        // first position along the line
  double hs;          // node spacing
  double hf;          // fine spacing
};

struct U0Dev {
  uint32_t kind;
  uint32_t nterms;
  double p[40];
};

__device__ double u0_value(const U0Dev& u, double x, double y) {
  const double* p = u.p;
  switch (u.kind) {
    case BRT_U0_CONST:
      return p[0];
    case BRT_U0_LOGISTIC: {
      const double nx = x * p[4] + y * p[5];
      const double base = 1.0 / (1.0 + exp(p[1] * (nx - p[2])));
      double v = 1.0;
      for (int k = 0; k < (int)p[3]; ++k) v *= base;
      return p[0] * v;
    }
    case BRT_U0_GAUSS_SUM: {
      double tot = 0.0;
      for (uint32_t k = 0; k < u.nterms; ++k) {
        const double A = p[4 * k], cx = p[4 * k + 1], cy = p[4 * k + 2], s = p[4 * k + 3];
        tot += A * exp(-((x - cx) * (x - cx) + (y - cy) * (y - cy)) / (2.0 * s * s));
      }
      return tot;
    }
    default: {
      if (fabs(x) > p[1] || fabs(y) > p[2]) return 0.0;
      const double cxv = cos(M_PI * x / (2.0 * p[1]));
      const double cyv = cos(M_PI * y / (2.0 * p[2]));
      return p[0] * (cxv * cxv) * (cyv * cyv);
    }
  }
}

// Moments (second derivatives) of the not-a-knot spline through y[0..m-1] at spacing h, m >= 4.  With
// uniform nodes the not-a-knot conditions M0 = 2 M1 - M2 and M(m-1) = 2 M(m-2) - M(m-3) turn the first
// and last interior equations into 6 M1 = r1 and 6 M(m-2) = r(m-2); the rest is the (1, 4, 1) system.
__device__ void notaknot_moments(const double* y, size_t ys, double* M, size_t ms, double* cp, size_t cs,
                                 int m, double h) {
  const double k6 = 6.0 / (h * h);
  auto r = [&](int i) { return k6 * ((y[(i - 1) * ys] - 2.0 * y[i * ys]) + y[(i + 1) * ys]); };
  const double M1 = r(1) / 6.0;
  const double Mm2 = r(m - 2) / 6.0;
  M[1 * ms] = M1;
  M[(m - 2) * ms] = Mm2;
  if (m >= 5) {
    // unknowns i = 2..m-3
    double dprev = 0.0, cprev = 0.0;
    for (int i = 2; i <= m - 3; ++i) {
      double rhs = r(i);
      if (i == 2) rhs -= M1;
      if (i == m - 3) rhs -= Mm2;
      const double inv = 1.0 / (4.0 - (i == 2 ? 0.0 : cprev));
      const double c = inv;
      const double d = (rhs - (i == 2 ? 0.0 : dprev)) * inv;
      cp[i * cs] = c;
      M[i * ms] = d;
      cprev = c;
      dprev = d;
    }
    double xn = M[(m - 3) * ms];
    for (int i = m - 4; i >= 2; --i) {
      xn = M[i * ms] - cp[i * cs] * xn;
      M[i * ms] = xn;
    }
  }
  M[0] = 2.0 * M1 - M[2 * ms];
  M[(m - 1) * ms] = 2.0 * Mm2 - M[(m - 3) * ms];
}

// Value at s (relative to node 0) of the spline with values y and moments M; s beyond the ends uses
// the end intervals' cubics.
__device__ double spline_value(const double* y, size_t ys, const double* M, size_t ms, int m, double h, double s) {
  int i = (int)floor(s / h);
  i = i < 0 ? 0 : (i > m - 2 ? m - 2 : i);
  const double ds = s - i * h;
  const double y0 = y[i * ys], y1 = y[(i + 1) * ys];
  const double M0 = M[i * ms], M1 = M[(i + 1) * ms];
  const double b = (y1 - y0) / h - h * (2.0 * M0 + M1) / 6.0;
  return y0 + ds * (b + ds * (0.5 * M0 + ds * ((M1 - M0) / (6.0 * h))));
}

struct SplineArgs {
  const LineDev* lines;
  uint32_t n_lines;
  uint32_t rows;      // nt + 1
  uint32_t max_ns;
  uint32_t max_fine;
  const double* node_values;
  double* vals;       // [line][row][max_ns]
  double* mom;        // [line][row][max_ns]
  double* cp;         // [line][row][max_ns] scratch
  double* rowsv;      // [row][line][max_fine]: values along the line at the fine nodes
  double* tmom;       // [row][line][max_fine]
  double* tcp;        // [row][line][max_fine]
  double* bd;
  double ht;          // node time spacing T / nt
  double dt;          // fine time step
  uint32_t n_steps;
  U0Dev u0;
};

__global__ void spline_rows_kernel(SplineArgs a) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= a.n_lines * a.rows) return;
  const uint32_t l = id / a.rows, row = id % a.rows;
  const LineDev L = a.lines[l];
  const size_t base = (size_t)id * a.max_ns;
  double* y = a.vals + base;
  for (uint32_t i = 0; i < L.ns; ++i) {
    double v;
    if (row == 0) {
      const double s = L.s_lo + i * L.hs;
      v = L.orient == 0 ? u0_value(a.u0, L.c, s) : u0_value(a.u0, s, L.c);
    } else {
      v = a.node_values[L.node_off + (size_t)(row - 1) * L.ns + i];
    }
    y[i] = v;
  }
  notaknot_moments(y, 1, a.mom + base, 1, a.cp + base, 1, (int)L.ns, L.hs);
}

__global__ void spline_s_kernel(SplineArgs a) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lr = blockIdx.y;  // line * rows + row
  const uint32_t l = lr / a.rows, row = lr % a.rows;
  const LineDev L = a.lines[l];
  if (j >= L.n_fine) return;
  const size_t base = (size_t)lr * a.max_ns;
  const double v = spline_value(a.vals + base, 1, a.mom + base, 1, (int)L.ns, L.hs, j * L.hf);
  a.rowsv[((size_t)row * a.n_lines + l) * a.max_fine + j] = v;
}

__global__ void spline_t_kernel(SplineArgs a) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t l = blockIdx.y;
  const LineDev L = a.lines[l];
  if (j >= L.n_fine) return;
  const size_t stride = (size_t)a.n_lines * a.max_fine;  // between node times
  const size_t off = (size_t)l * a.max_fine + j;
  const double* y = a.rowsv + off;
  double* M = a.tmom + off;
  notaknot_moments(y, stride, M, stride, a.tcp + off, stride, (int)a.rows, a.ht);
  double* out = a.bd + L.bd_off + j;
  for (uint32_t n = 0; n <= a.n_steps; ++n)
    out[(size_t)n * L.n_fine] = spline_value(y, stride, M, stride, (int)a.rows, a.ht, n * a.dt);
}

struct FieldArgs {
  double* f0;
  double* f1;
  const double* bd;
  const LineDev* lines;
  uint32_t NX, NY, W, cx, cy, zero_outer;  // W: row pitch of the fields
  double x_lo, y_lo, hx, hy;
  int16_t vline[kMaxSub + 1];
  int16_t hline[kMaxSub + 1];
  U0Dev u0;
};

__global__ void init_field_kernel(FieldArgs a) {
  const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (uint64_t)(a.NX + 1) * (a.NY + 1)) return;
  const uint32_t i = (uint32_t)(id % (a.NX + 1)), j = (uint32_t)(id / (a.NX + 1));
  double v = u0_value(a.u0, a.x_lo + i * a.hx, a.y_lo + j * a.hy);
  const bool on_v = i % a.cx == 0 && a.vline[i / a.cx] >= 0;
  const bool on_h = j % a.cy == 0 && a.hline[j / a.cy] >= 0;
  if (on_v) {
    const LineDev& L = a.lines[a.vline[i / a.cx]];
    v = a.bd[L.bd_off + j];
  } else if (on_h) {
    const LineDev& L = a.lines[a.hline[j / a.cy]];
    v = a.bd[L.bd_off + i];
  } else if (a.zero_outer && (i == 0 || i == a.NX || j == 0 || j == a.NY)) {
    v = 0.0;
  }
  const size_t idx = (size_t)j * a.W + i;
  a.f0[idx] = v;
  a.f1[idx] = v;
}

struct AdiArgs {
  double* f0;
  double* f1;
  double* yrhs;         // the y phase's right-hand sides without boundary terms, written by the x phase
  const double* bd;
  const LineDev* lines;
  const double* inv_x;  // pivots' reciprocals of the x and the y lines, kSegs * S each, zero-padded
  const double* inv_y;
  uint32_t* sync;       // [2] abort; [4 + 2g] arrivals at, [5 + 2g] dies of the blocks of barrier group g
  uint64_t spin_limit;  // wall-clock ticks a barrier may wait
  double pcoef[8];      // f(u) = c1 u + m(x, y, t) sum_j pcoef_j u^j: the modulated part (pcoef_1 = 0 unless c_1 is modulated) ...
  const double* ex;     // ... scaled by ex[i] ey[j] (t_mid + t0)^-pow (all 1 with constant coefficients)
  const double* ey;
  uint32_t cm_pow;
  double cm_t0, c1, dt;
  double rx2, ry2, dt2;
  uint32_t W;           // row pitch of the fields (a multiple of 16)
  uint32_t px, py, cx, cy;
  uint32_t steps;
  uint32_t nblocks;
  uint32_t groups;      // barrier groups: 1 (the whole grid) or one per die, each owning whole subdomains
  uint32_t x_blk, y_blk;       // items per subdomain in the x and the y phase
  uint32_t n_vlines, bv, bh;   // data lines: vertical count; blocks of nodes per vertical / horizontal line
  uint32_t n_lines;
  int16_t vline[kMaxSub + 1];
  int16_t hline[kMaxSub + 1];
  uint32_t v_fine, h_fine;               // fine nodes of a vertical and of a horizontal line
  uint64_t bd_off[2 * (kMaxSub + 1)];    // boundary data offset of each line (doubles)
};

__device__ inline double reaction(const double* c, double u) {
  double f = 0.0;
  for (int j = 7; j >= 0; --j) f = f * u + c[j];
  return f;
}

// f at the extrapolated value ut for the node with modulation factor exy and the step's time factor tf
// (both 1 with constant coefficients): c_1 ut + (exy tf) P(ut), P the non-linear part.
__device__ inline double reaction_at(const AdiArgs& a, double ut, double exy, double tf) {
  return a.c1 * ut + (exy * tf) * reaction(a.pcoef, ut);
}

__device__ inline double time_factor(const AdiArgs& a, uint32_t n) {
  return a.cm_pow ? 1.0 / ((n + 0.5) * a.dt + a.cm_t0) : 1.0;
}

// Die (XCD) this wave runs on.
__device__ inline uint32_t xcc_id() {
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & 0xfu;
}

// Barrier of a group of blocks: cnt counts arrivals from the start of the launch, so the k-th barrier
// is passed when it reaches k * members (no reset between barriers).  Every block waits at most
// spin_limit wall-clock ticks; on a time-out, or when any block has timed out, it raises the abort
// word and returns false so that every block leaves the kernel.
//
// Fences.  With die_local set, every block of the group runs on one die, and all that the group's
// blocks read after a barrier was written by the group itself: the die's L2 is then the coherence
// point, so each wave waits until its stores are in L2 and the arriving side needs no L2 write-back.
// The CU's vector L1 may hold lines this CU read before the barrier and other CUs have rewritten
// since; the sweeps read every such field value with L1-bypassing loads (ldg2_c), so the leaving side
// needs no invalidate either.  Otherwise device-scope fences (L2 write-back and invalidation) order
// the phases.
__device__ bool group_barrier(uint32_t* cnt, uint32_t* abort_word, uint32_t members, uint32_t& gen, uint64_t spin_limit,
                              bool die_local, uint32_t* flag) {
  if (die_local) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ok = 1;
    if (!die_local) __threadfence();
    const uint32_t target = (gen + 1) * members;
    if (atomicAdd(cnt, 1u) != target - 1) {
      const uint64_t t0 = wall_clock64();
      // relaxed polling: an acquiring load would invalidate the caches on every poll while other
      // blocks still work; the fence below acquires once the count has reached the target
      while ((int32_t)(__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
        if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            wall_clock64() - t0 > spin_limit) {
          atomicExch(abort_word, 1u);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    if (!die_local) __threadfence();
    gen += 1;
    *flag = ok;
  }
  __syncthreads();
  return *flag != 0;
}

// Intermediate-level value on the vertical line kx at row y between levels n and n+1.
__device__ inline double ustar_line(const AdiArgs& a, uint32_t kx, uint32_t y, uint32_t n) {
  const int vl = a.vline[kx];
  if (vl < 0) return 0.0;
  const double* g0 = a.bd + a.bd_off[vl] + (size_t)n * a.v_fine;
  const double* g1 = g0 + a.v_fine;
  const double d0 = (g0[y - 1] - 2.0 * g0[y]) + g0[y + 1];
  const double d1 = (g1[y - 1] - 2.0 * g1[y]) + g1[y + 1];
  return 0.5 * (g0[y] + a.ry2 * d0) + 0.5 * (g1[y] - a.ry2 * d1);
}

// Value at level n on the horizontal line ky at column x (0 for an outer edge held at zero).
__device__ inline double hline_value(const AdiArgs& a, uint32_t ky, uint32_t x, uint32_t n) {
  const int hl = a.hline[ky];
  if (hl < 0) return 0.0;
  return a.bd[a.bd_off[hl] + (size_t)n * a.h_fine + x];
}

// A work item is L lines of one subdomain, solved by one block of 32 L threads with the lines resident
// in LDS (L = 32 for segments of 16 unknowns, 16 for segments of 32).  Three passes:
//   1. the right-hand sides, from coalesced global loads (x phase: threads along the positions of the
//      item's rows; y phase: L/2 column pairs x 64 row groups), into LDS [line][position];
//   2. the tridiagonal solves, kSegs threads per line, each owning S consecutive positions: a local
//      forward recurrence, a scan of the segments' affine carry maps over the line's lanes, the carry
//      applied, a local backward recurrence, a reverse scan, and the backward carry applied;
//   3. the solution back to global memory with the thread mapping of pass 1.
// In LDS a segment of S positions is followed by one pad double (conflict-free segment reads) and the
// line pitch is 4 mod 32 doubles (conflict-free column writes in the y phase).  The pivots' reciprocals
// of both directions stay in LDS for the whole launch, in the same segment layout.  Subdomains have at
// most kSegs * 32 cells per side.
constexpr int kSegs = 32;    // threads per line in pass 2; row groups of the y phase's passes 1 and 3
constexpr int kXBatch = 8;   // x phase: rows loaded together
constexpr int kYBatch = 4;   // y phase: positions per thread loaded together

template <int S>
struct AdiShape {
  static constexpr int lines = S == 16 ? 32 : 16;  // lines per item
  static constexpr int threads = lines * kSegs;    // threads per block
};

static_assert(kMaxCells - 1 <= (uint32_t)kSegs * 32, "the longest line must fit 32 segments of 32");

__host__ __device__ constexpr uint32_t seg_span(int S) { return (uint32_t)kSegs * (S + 1); }
__host__ __device__ constexpr uint32_t seg_pitch(int S) { return seg_span(S) + 4; }
__host__ __device__ constexpr int adi_lines(int S) { return S == 16 ? AdiShape<16>::lines : AdiShape<32>::lines; }
__host__ __device__ constexpr int adi_threads(int S) { return adi_lines(S) * kSegs; }
// LDS (doubles): the lines, the pivots' reciprocals of the x and the y lines, then the intermediate
// values on the item's two vertical data lines (scaled by r/2, then plain) and the coefficient
// modulation of its rows (x phase).
__host__ __device__ constexpr size_t adi_lds_doubles(int S) {
  return (size_t)adi_lines(S) * seg_pitch(S) + 2 * (size_t)seg_span(S) + 5 * (size_t)adi_lines(S);
}

template <int S>
__device__ inline uint32_t lds_pos(uint32_t p) {
  return p + p / S;
}

// Global accesses at a 32-bit byte offset from a base that is uniform over the block.
__device__ inline void stg(double* base, uint32_t byte_off, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// Two neighbouring columns in one access; only 8-byte alignment is assumed (multi-dword global
// accesses need dword alignment), so a pair may start at any column.
typedef double dpair __attribute__((ext_vector_type(2), aligned(8)));
__device__ inline dpair ldg2(const double* base, uint32_t byte_off) {
  return *reinterpret_cast<const dpair*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ inline void stg2(double* base, uint32_t byte_off, dpair v) {
  *reinterpret_cast<dpair*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// A pair of field values that other blocks of the group wrote since the last barrier, loaded past the
// CU's vector L1 (agent-scope coherent loads), so that leaving a die-local barrier needs no L1
// invalidate: the L1 may keep lines of the read-only data (boundary data, coefficient factors).
__device__ inline dpair ldg2_c(const double* base, uint32_t byte_off) {
  const unsigned long long* q =
      reinterpret_cast<const unsigned long long*>(reinterpret_cast<const char*>(base) + byte_off);
  const unsigned long long lo = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long hi = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return dpair{__longlong_as_double((long long)lo), __longlong_as_double((long long)hi)};
}
__device__ inline double ldg_c(const double* base, uint32_t byte_off) {
  const unsigned long long* q =
      reinterpret_cast<const unsigned long long*>(reinterpret_cast<const char*>(base) + byte_off);
  return __longlong_as_double((long long)__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Keeps the scheduler from hoisting the loads of a later batch above this point.
__device__ inline void batch_fence() { __builtin_amdgcn_sched_barrier(0); }

// The thread index, opaque to the compiler: per-thread offsets are then recomputed in each sweep
// instead of being hoisted out of the step loop and held in registers for the whole launch.
__device__ inline uint32_t thread_index() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Pass 2 on the lines at D (kSegs threads per line).  For a line of m unknowns with
// (1 + r) x_i - (r/2)(x_{i-1} + x_{i+1}) = d_i, Thomas' recurrences are d'_i = INV_i d_i + B_i d'_{i-1}
// and x_i = d'_i + B_i x_{i+1}, with INV_i the pivots' reciprocals and B_i = (r/2) INV_i (both zero
// beyond m, so padded unknowns solve to zero).  Segment j first runs the forward recurrence from a
// zero carry; d'_i = y_i + beta_i c_j then follows from the true carry c_j (d' at the end of segment
// j-1, from a scan of the maps c -> y_end + beta_end c) and the running product beta_i of the B's from
// the segment's start.  The backward recurrence likewise runs from a zero carry, and
// x_i = z_i + g_i x_in with g_i the product of the B's from i to the segment's end and x_in the
// solution just after the segment (a reverse scan of the maps x -> z_start + g_start x).
template <int S>
__device__ inline void solve_lines(double* __restrict__ D, uint32_t pitch, const double* __restrict__ inv, double half) {
  const uint32_t t = thread_index();
  const uint32_t j = t % kSegs;
  double* __restrict__ Dl = D + (t / kSegs) * pitch + j * (S + 1);
  const double* __restrict__ F = inv + j * (S + 1);
  double y[S];
  double acc = 0.0, beta = 1.0;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const double f = F[k];
    const double b = half * f;
    acc = fma(b, acc, Dl[k] * f);
    y[k] = acc;
    beta *= b;
  }
  double ca = acc, cb = beta;
#pragma unroll
  for (int d = 1; d < kSegs; d <<= 1) {
    const double a2 = __shfl_up(ca, d, kSegs), b2 = __shfl_up(cb, d, kSegs);
    if (j >= (uint32_t)d) {
      ca = fma(cb, a2, ca);
      cb *= b2;
    }
  }
  double c = __shfl_up(ca, 1, kSegs);
  if (j == 0) c = 0.0;
  double z = 0.0, g = 1.0;
  beta = 1.0;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    beta *= half * F[k];
    y[k] = fma(c, beta, y[k]);
  }
#pragma unroll
  for (int k = S - 1; k >= 0; --k) {
    const double b = half * F[k];
    z = fma(b, z, y[k]);
    y[k] = z;
    g *= b;
  }
  double xa = z, xg = g;
#pragma unroll
  for (int d = 1; d < kSegs; d <<= 1) {
    const double a2 = __shfl_down(xa, d, kSegs), g2 = __shfl_down(xg, d, kSegs);
    if (j + d < (uint32_t)kSegs) {
      xa = fma(xg, a2, xa);
      xg *= g2;
    }
  }
  double xin = __shfl_down(xa, 1, kSegs);
  if (j == kSegs - 1) xin = 0.0;
  g = 1.0;
#pragma unroll
  for (int k = S - 1; k >= 0; --k) {
    g *= half * F[k];
    Dl[k] = fma(g, xin, y[k]);
  }
}

// The x phase solves the x lines for the intermediate level u* and then forms, while u* is in LDS, the
// right-hand side of the y phase at every interior node except its boundary terms:
// u* + (r/2) d_xx u* + (dt/2) f, with f the reaction it used itself.  The y phase then reads one value
// per node instead of u*, its x neighbours, u^n and u^{n-1}.  (dt/2) f waits in the output array
// between the two passes (the same thread overwrites it; the lines stay in L2), not in registers.
template <int S>
__device__ void x_sweep(const AdiArgs& a, uint32_t item, uint32_t n, const double* __restrict__ cur,
                        const double* __restrict__ prev, double* __restrict__ smem) {
  constexpr int L = AdiShape<S>::lines, T = AdiShape<S>::threads;
  constexpr uint32_t M = (uint32_t)kSegs * S;
  constexpr uint32_t pitch = seg_pitch(S);
  // pass 1 and 3: threads along the position pairs; with more threads than pairs, row sets of R rows
  constexpr uint32_t NP = M / 2, sets = T >= (int)NP ? T / NP : 1, R = L / sets, pstep = sets > 1 ? NP : T;
  static_assert(pstep >= NP, "one position pair per thread");
  const uint32_t t = thread_index();
  const uint32_t h = sets > 1 ? t / NP : 0, pp = sets > 1 ? t % NP : t, r0 = h * R;
  const uint32_t sub = item / a.x_blk, blk = item % a.x_blk;
  const uint32_t sx = sub % a.px, sy = sub / a.px;
  const uint32_t ybase = sy * a.cy + 1 + blk * L;
  const uint32_t nrows = min((uint32_t)L, (sy + 1) * a.cy - ybase);  // lines of this item
  const uint32_t c0 = sx * a.cx, m = a.cx - 1, W = a.W;
  double* __restrict__ D = smem;                                  // [line][pitch]
  const double* __restrict__ INV = D + L * pitch;                 // x lines
  double* __restrict__ SB = D + L * pitch + 2 * seg_span(S);      // u* on the two vertical lines: scaled, plain
  double* __restrict__ EY = SB + 4 * L;                           // coefficient modulation of the item's rows
  const double tf = time_factor(a, n);
  const double* __restrict__ cur_b = cur + (size_t)(ybase - 1) * W + c0 + 1;  // row above the item
  const double* __restrict__ prev_b = prev + (size_t)ybase * W + c0 + 1;
  double* __restrict__ yr_b = a.yrhs + (size_t)ybase * W + c0 + 1;
  // Halo rows on the subdomain's horizontal data lines are read from the boundary data (level n), so a
  // subdomain never reads field values that another subdomain's solve writes.
  const int hl_top = blk == 0 ? a.hline[sy] : -1;
  const int hl_bot = ybase + nrows == (sy + 1) * a.cy ? a.hline[sy + 1] : -1;
  const double* __restrict__ top_b = hl_top >= 0 ? a.bd + a.bd_off[hl_top] + (size_t)n * a.h_fine + c0 + 1 : cur_b;
  const double* __restrict__ bot_b =
      hl_bot >= 0 ? a.bd + a.bd_off[hl_bot] + (size_t)n * a.h_fine + c0 + 1 : cur_b + (size_t)(nrows + 1) * W;
  auto cur_row = [&](uint32_t rel) {  // rel: row above the item = 0; clamped to nrows + 1
    return rel == 0 ? top_b : rel >= nrows + 1 ? bot_b : cur_b + (size_t)rel * W;
  };
  if (t < (uint32_t)L) {
    EY[t] = a.ey[min(ybase + t, ybase + nrows - 1)];
    if (t < nrows) {
      const uint32_t y = ybase + t;
      const double usl = ustar_line(a, sx, y, n), usr = ustar_line(a, sx + 1, y, n);
      SB[t] = a.rx2 * usl;
      SB[L + t] = a.rx2 * usr;
      SB[2 * L + t] = usl;
      SB[3 * L + t] = usr;
    }
  }
  __syncthreads();
  const uint32_t pa = 2 * pp, pb = pa + 1;  // the pair's positions (pb may be the line column)
  const uint32_t oa = lds_pos<S>(pa), ob = lds_pos<S>(pb);
  if (pa >= m) {
#pragma unroll
    for (uint32_t k = 0; k < R; ++k) {
      D[(r0 + k) * pitch + oa] = 0.0;
      D[(r0 + k) * pitch + ob] = 0.0;
    }
  } else {
    const uint32_t vo = 8 * pa;
    const dpair exv = ldg2(a.ex + c0 + 1, vo);
    dpair up = ldg2_c(cur_row(min(r0, nrows + 1)), vo), mid = ldg2_c(cur_row(min(r0 + 1, nrows + 1)), vo);
#pragma unroll
    for (uint32_t k0 = 0; k0 < R; k0 += kXBatch) {
      dpair cv[kXBatch], pv[kXBatch];
#pragma unroll
      for (int k = 0; k < kXBatch; ++k) {
        cv[k] = ldg2_c(cur_row(min(r0 + k0 + k + 2, nrows + 1)), vo);
        pv[k] = ldg2_c(prev_b + (size_t)min(r0 + k0 + k, nrows - 1) * W, vo);
      }
#pragma unroll
      for (int k = 0; k < kXBatch; ++k) {
        const uint32_t row = r0 + k0 + k;
        const dpair u = mid, dn = cv[k];
        const double ey = EY[row];
        const double fa = a.dt2 * reaction_at(a, 1.5 * u.x - 0.5 * pv[k].x, exv.x * ey, tf);
        const double fb = a.dt2 * reaction_at(a, 1.5 * u.y - 0.5 * pv[k].y, exv.y * ey, tf);
        double da = u.x + a.ry2 * ((up.x - 2.0 * u.x) + dn.x) + fa;
        double db = u.y + a.ry2 * ((up.y - 2.0 * u.y) + dn.y) + fb;
        if (row < nrows) {
          if (pb < m)
            stg2(yr_b + (size_t)row * W, 8 * pa, dpair{fa, fb});
          else
            stg(yr_b + (size_t)row * W, 8 * pa, fa);
        }
        if (pa == 0) da += SB[row];
        if (pa == m - 1) da += SB[L + row];
        if (pb == m - 1) db += SB[L + row];
        D[row * pitch + oa] = da;
        D[row * pitch + ob] = pb < m ? db : 0.0;
        up = mid;
        mid = dn;
      }
      batch_fence();
    }
  }
  __syncthreads();
  solve_lines<S>(D, pitch, INV, a.rx2);
  __syncthreads();
  if (pa < m) {
    const uint32_t ol = pa > 0 ? lds_pos<S>(pa - 1) : oa, orr = pb + 1 < m ? lds_pos<S>(pb + 1) : oa;
    dpair fv[R];
#pragma unroll
    for (uint32_t k = 0; k < R; ++k)
      fv[k] = r0 + k < nrows ? (pb < m ? ldg2_c(yr_b + (size_t)(r0 + k) * W, 8 * pa)
                                       : dpair{ldg_c(yr_b + (size_t)(r0 + k) * W, 8 * pa), 0.0})
                             : dpair{0.0, 0.0};
#pragma unroll
    for (uint32_t k = 0; k < R; ++k) {
      const uint32_t row = r0 + k;
      if (row >= nrows) continue;
      const double* Dr = D + row * pitch;
      const double usr = SB[3 * L + row];
      const double sa = Dr[oa];
      const double sl = pa > 0 ? Dr[ol] : SB[2 * L + row];
      const double sb = pb < m ? Dr[ob] : usr;
      const double ra = sa + a.rx2 * ((sl - 2.0 * sa) + sb) + fv[k].x;
      double* out = yr_b + (size_t)row * W;
      if (pb < m) {
        const double sr = pb + 1 < m ? Dr[orr] : usr;
        stg2(out, 8 * pa, dpair{ra, sb + a.rx2 * ((sa - 2.0 * sb) + sr) + fv[k].y});
      } else {
        stg(out, 8 * pa, ra);
      }
    }
  }
  __syncthreads();
}

// The y phase adds the boundary terms of the horizontal data lines (level n+1) to the right-hand sides
// the x phase left, solves the y lines and writes u^{n+1}.
template <int S>
__device__ void y_sweep(const AdiArgs& a, uint32_t item, uint32_t n, double* __restrict__ next,
                        double* __restrict__ smem) {
  constexpr int L = AdiShape<S>::lines, T = AdiShape<S>::threads;
  constexpr uint32_t pitch = seg_pitch(S);
  constexpr uint32_t P2 = L / 2, G = T / P2, npt = (uint32_t)kSegs * S / G;  // pairs per row, row groups, positions per thread
  const uint32_t t = thread_index();
  const uint32_t c = t % P2, q = t / P2;  // column pair, row group
  const uint32_t sub = item / a.y_blk, blk = item % a.y_blk;
  const uint32_t sx = sub % a.px, sy = sub / a.px;
  const uint32_t xfirst = sx * a.cx + 1 + blk * L;
  const uint32_t nl = min((uint32_t)L, (sx + 1) * a.cx - xfirst);
  const uint32_t cc = min(c, (nl - 1) / 2);
  const uint32_t x = xfirst + 2 * cc;   // first column of the pair (x + 1 exists: interior or the line column)
  const uint32_t r0 = sy * a.cy, m = a.cy - 1, W = a.W;
  double* __restrict__ D = smem;  // [line][pitch]
  const double* __restrict__ INV = D + L * pitch + seg_span(S);  // y lines
  const double* __restrict__ yr_b = a.yrhs + (size_t)r0 * W;
  double* __restrict__ next_b = next + (size_t)r0 * W;
  const double gb00 = a.ry2 * hline_value(a, sy, x, n + 1), gb01 = a.ry2 * hline_value(a, sy, x + 1, n + 1);
  const double gb10 = a.ry2 * hline_value(a, sy + 1, x, n + 1), gb11 = a.ry2 * hline_value(a, sy + 1, x + 1, n + 1);
  const uint32_t l0 = 2 * c, l1 = 2 * c + 1;
#pragma unroll
  for (uint32_t kb = 0; kb < npt; kb += kYBatch) {
    dpair rv[kYBatch];
#pragma unroll
    for (int k = 0; k < kYBatch; ++k) {
      const uint32_t p = min(q + G * (kb + k), m - 1);
      rv[k] = ldg2_c(yr_b, 8 * ((1 + p) * W + x));
    }
#pragma unroll
    for (int k = 0; k < kYBatch; ++k) {
      const uint32_t p = q + G * (kb + k);
      double d0 = rv[k].x, d1 = rv[k].y;
      if (p == 0) {
        d0 += gb00;
        d1 += gb01;
      }
      if (p == m - 1) {
        d0 += gb10;
        d1 += gb11;
      }
      const uint32_t o = lds_pos<S>(p);
      D[l0 * pitch + o] = p < m ? d0 : 0.0;
      D[l1 * pitch + o] = p < m ? d1 : 0.0;
    }
  }
  __syncthreads();
  solve_lines<S>(D, pitch, INV, a.ry2);
  __syncthreads();
  if (l0 < nl)
#pragma unroll 4
    for (uint32_t k = 0; k < npt; ++k) {
      const uint32_t p = q + G * k;
      if (p < m) {
        const uint32_t o = lds_pos<S>(p), off = 8 * ((1 + p) * W + x);
        if (l1 < nl)
          stg2(next_b, off, dpair{D[l0 * pitch + o], D[l1 * pitch + o]});
        else
          stg(next_b, off, D[l0 * pitch + o]);
      }
    }
  __syncthreads();
}

// Line nodes of level n+1 into the new field; a horizontal line leaves the nodes it shares with a
// vertical data line to that line.
__device__ void write_lines(const AdiArgs& a, uint32_t item, uint32_t n, double* next) {
  uint32_t l, blk;
  if (item < a.n_vlines * a.bv) {
    l = item / a.bv;
    blk = item % a.bv;
  } else {
    item -= a.n_vlines * a.bv;
    l = a.n_vlines + item / a.bh;
    blk = item % a.bh;
  }
  const LineDev& L = a.lines[l];
  const uint32_t j = blk * blockDim.x + threadIdx.x;
  if (j >= L.n_fine) return;
  const double v = a.bd[L.bd_off + (size_t)(n + 1) * L.n_fine + j];
  if (L.orient == 0) {
    next[(size_t)j * a.W + L.k * a.cx] = v;
  } else {
    if (j % a.cx == 0 && a.vline[j / a.cx] >= 0) return;
    next[(size_t)(L.k * a.cy) * a.W + j] = v;
  }
}

// Blocks are dealt to the dies round-robin (block b on die b mod 8).  With a grid that is a multiple
// of the die count, the blocks of die x, ranked r = b / 8, form `parts` consecutive parts of equal size
// (parts a multiple of 8; 8 parts: one per die).  Part k = x (parts / 8) + r / size holds the blocks
// that synchronise together when parts are barrier groups.
struct BlockPart {
  uint32_t part, rank, size;
};
__device__ inline BlockPart block_part(uint32_t parts) {
  const uint32_t b = blockIdx.x, size = gridDim.x / parts, r = b / kXcds;
  return {(b % kXcds) * (parts / kXcds) + r / size, r % size, size};
}

// Items of a phase taken by this block.  With a grid that is a multiple of the die count, the items
// are split into one contiguous range per part (the barrier groups when there are more than 8, else
// the dies) and dealt round-robin over the part's blocks: a group's blocks then take exactly the items
// of its subdomains, and the blocks of a die work on neighbouring strips at the same time and share
// the halo lines in its L2.
struct ItemRange {
  uint32_t begin, end, stride;
};
__device__ inline ItemRange block_items(uint32_t n_items, uint32_t groups) {
  if (gridDim.x % kXcds != 0) return {blockIdx.x, n_items, gridDim.x};
  const uint32_t parts = groups > kXcds ? groups : kXcds;
  const BlockPart p = block_part(parts);
  return {(uint32_t)((uint64_t)n_items * p.part / parts) + p.rank, (uint32_t)((uint64_t)n_items * (p.part + 1) / parts),
          p.size};
}

template <int S>
__global__ __launch_bounds__(AdiShape<S>::threads) void adi_kernel(AdiArgs a) {
  extern __shared__ double smem[];
  __shared__ uint32_t barrier_ok;
  uint32_t gen = 0;
  const uint32_t nsub = a.px * a.py;
  uint32_t* const bar = a.sync + 4 + 2 * (a.groups > 1 ? block_part(a.groups).part : 0u);
  const uint32_t members = gridDim.x / a.groups;
  const uint32_t x_items = nsub * a.x_blk;
  const uint32_t y_items = nsub * a.y_blk;
  const uint32_t l_items = a.n_vlines * a.bv + (a.n_lines - a.n_vlines) * a.bh;
  {  // pivots' reciprocals of both directions into LDS, segment layout
    constexpr uint32_t M = (uint32_t)kSegs * S;
    double* inv = smem + AdiShape<S>::lines * seg_pitch(S);
    for (uint32_t i = threadIdx.x; i < M; i += AdiShape<S>::threads) {
      inv[lds_pos<S>(i)] = a.inv_x[i];
      inv[seg_span(S) + lds_pos<S>(i)] = a.inv_y[i];
    }
    __syncthreads();
  }
  // Items of a phase cost the same (equal subdomains), so they are dealt statically: no counter
  // traffic between the barriers.
  const ItemRange xr = block_items(x_items, a.groups), yr = block_items(y_items, a.groups);
  // Which dies the group's blocks run on: one bit per die, complete after the group's first barrier.
  if (threadIdx.x == 0) atomicOr(bar + 1, 1u << xcc_id());
  if (!group_barrier(bar, a.sync + 2, members, gen, a.spin_limit, false, &barrier_ok)) return;
  const bool die_local = __popc(__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 1;
  for (uint32_t n = 0; n < a.steps; ++n) {
    const double* cur = (n & 1) ? a.f1 : a.f0;
    double* prev = (n & 1) ? a.f0 : a.f1;  // holds u^{n-1}; receives u^{n+1}
    for (uint32_t it = xr.begin; it < xr.end; it += xr.stride) x_sweep<S>(a, it, n, cur, prev, smem);
    if (!group_barrier(bar, a.sync + 2, members, gen, a.spin_limit, die_local, &barrier_ok)) return;
    for (uint32_t it = yr.begin; it < yr.end; it += yr.stride) y_sweep<S>(a, it, n, prev, smem);
    for (uint32_t it = blockIdx.x; it < l_items; it += gridDim.x) write_lines(a, it, n, prev);
    if (!group_barrier(bar, a.sync + 2, members, gen, a.spin_limit, die_local, &barrier_ok)) return;
  }
}

}  // namespace

struct brt_pdd {
  brt_ctx* ctx = nullptr;
  brt_problem prob{};
  brt_pdd_grid g{};
  int device = 0, n_cu = 0;
  uint32_t NX = 0, NY = 0, W = 0, max_ns = 0, max_fine = 0, n_vlines = 0;  // W: field row pitch
  double hx = 0, hy = 0, dt = 0, rx = 0, ry = 0;
  std::vector<LineDev> lines;
  int16_t vline[kMaxSub + 1];
  int16_t hline[kMaxSub + 1];
  uint64_t n_nodes = 0, bd_doubles = 0;
  U0Dev u0{};
  // device
  LineDev* d_lines = nullptr;
  double* d_bd = nullptr;
  double* d_f[3] = {nullptr, nullptr, nullptr};
  double* d_fac = nullptr;
  double* d_spl = nullptr;  // vals, mom, cp, rowsv, tmom, tcp
  uint32_t* d_sync = nullptr;
  double* d_node_u = nullptr;
  double* d_exy = nullptr;  // variable coefficients: e^{-bx x_i^2} (NX+1), then e^{-by y_j^2} (NY+1)
  size_t spl_rows = 0, spl_fine = 0;
  // Monte Carlo plan of the nodes (built on first run, rebuilt when mc or the tree count change)
  brt_plan* plan = nullptr;
  brt_mc plan_mc{};
  uint64_t plan_trees = 0;
  hipEvent_t ev[6] = {};
  bool recorded[3] = {false, false, false};
  uint32_t last_groups = 0;  // barrier groups of the last solve
  int grid = 0;
  int seg = 16;    // unknowns per segment of the solver's line solves
  size_t lds = 0;  // dynamic LDS of the solver launch (bytes)
};

namespace {

void pdd_free(brt_pdd* p) {
  if (!p) return;
  if (p->plan) brt_plan_destroy(p->plan);
  (void)hipFree(p->d_lines);
  (void)hipFree(p->d_bd);
  for (double* f : p->d_f) (void)hipFree(f);
  (void)hipFree(p->d_fac);
  (void)hipFree(p->d_spl);
  (void)hipFree(p->d_sync);
  (void)hipFree(p->d_node_u);
  (void)hipFree(p->d_exy);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

// Reciprocals of the Thomas pivots of (1 + r) x_i - (r/2)(x_{i-1} + x_{i+1}) = d_i, i < m, padded
// with zeros to kSegs * S entries.
void pivot_reciprocals(double r, uint32_t m, int S, double* inv) {
  const double diag = 1.0 + r, half = 0.5 * r;
  for (uint32_t i = 0; i < (uint32_t)kSegs * S; ++i) inv[i] = i < m ? 1.0 / (i == 0 ? diag : diag - half * half * inv[i - 1]) : 0.0;
}

// Segment length of the solver: the smallest of 16 and 32 that covers the longer side.
int seg_length(const brt_pdd_grid& g) { return std::max(g.cx, g.cy) - 1 <= (uint32_t)kSegs * 16 ? 16 : 32; }

const void* adi_kernel_ptr(int S) {
  return S == 16 ? reinterpret_cast<const void*>(&adi_kernel<16>) : reinterpret_cast<const void*>(&adi_kernel<32>);
}

}  // namespace

extern "C" {

int brt_pdd_create(brt_ctx* ctx, const brt_problem* prob, const brt_pdd_grid* grid, brt_pdd** out) {
  return brt::api_guard("brt_pdd_create", [&]() -> int {
    if (!ctx || !prob || !grid || !out) return set_error(BRT_E_ARG, "brt_pdd_create: NULL argument");
    *out = nullptr;
    if (prob->struct_size != sizeof(brt_problem)) return set_error(BRT_E_ARG, "brt_problem.struct_size mismatch");
    if (grid->struct_size != sizeof(brt_pdd_grid)) return set_error(BRT_E_ARG, "brt_pdd_grid.struct_size mismatch");
    const brt_pdd_grid& g = *grid;
    if (prob->dim != 2) return set_error(BRT_E_ARG, "pdd: the problem must be 2-D");
    if (!(prob->diffusion > 0.0) || !std::isfinite(prob->diffusion)) return set_error(BRT_E_ARG, "pdd: diffusion must be > 0");
    for (double c : prob->coef)
      if (!std::isfinite(c)) return set_error(BRT_E_ARG, "pdd: non-finite coefficient");
    if (prob->u0_kind > BRT_U0_COS2_BUMP) return set_error(BRT_E_ARG, "pdd: unknown u0_kind");
    if (prob->coef_mod > BRT_COEF_MOD_GAUSS_TIME_ALL) return set_error(BRT_E_ARG, "pdd: unknown coef_mod");
    if (prob->drift[0] != 0.0 || prob->drift[1] != 0.0 || prob->sde != BRT_SDE_EXACT)
      return set_error(BRT_E_ARG, "pdd: the subdomain solver takes L = a Lap (no drift, constant sigma)");
    if (prob->coef_mod != BRT_COEF_MOD_NONE &&
        (!(prob->coef_mod_beta[0] >= 0.0) || !(prob->coef_mod_beta[1] >= 0.0) || prob->coef_mod_pow > 1 ||
         (prob->coef_mod_pow == 1 && !(prob->coef_mod_t0 > 0.0))))
      return set_error(BRT_E_ARG, "pdd: invalid variable-coefficient parameters");
    if (prob->u0_kind == BRT_U0_GAUSS_SUM && (prob->u0_nterms < 1 || prob->u0_nterms > 8))
      return set_error(BRT_E_ARG, "pdd: gauss_sum needs 1..8 terms");
    if (!(g.x_hi > g.x_lo) || !(g.y_hi > g.y_lo) || !std::isfinite(g.x_lo + g.x_hi + g.y_lo + g.y_hi))
      return set_error(BRT_E_ARG, "pdd: empty or non-finite domain");
    if (g.px < 1 || g.py < 1 || g.px > kMaxSub || g.py > kMaxSub) return set_error(BRT_E_ARG, "pdd: px, py must be 1..64");
    if (g.cx < 2 || g.cy < 2 || g.cx > kMaxCells || g.cy > kMaxCells) return set_error(BRT_E_ARG, "pdd: cx, cy must be 2..1024");
    if (!(g.T > 0.0) || !std::isfinite(g.T)) return set_error(BRT_E_ARG, "pdd: T must be > 0");
    if (g.n_steps < 1 || g.n_steps > (1u << 20)) return set_error(BRT_E_ARG, "pdd: n_steps must be 1..2^20");
    if (g.ns_x < 4 || g.ns_y < 4 || g.ns_x > kMaxNodesPerLine || g.ns_y > kMaxNodesPerLine)
      return set_error(BRT_E_ARG, "pdd: ns_x, ns_y must be 4..257");
    if (g.nt < 3 || g.nt > kMaxNt) return set_error(BRT_E_ARG, "pdd: nt must be 3..63");
    if (g.outer != BRT_PDD_OUTER_LINES && g.outer != BRT_PDD_OUTER_ZERO) return set_error(BRT_E_ARG, "pdd: unknown outer");
    if (g.outer == BRT_PDD_OUTER_ZERO && g.px == 1 && g.py == 1)
      return set_error(BRT_E_ARG, "pdd: no lines (one subdomain with zero outer edges)");

    brt_pdd* p = new (std::nothrow) brt_pdd;
    if (!p) return set_error(BRT_E_NOMEM, "pdd: host allocation");
    p->ctx = ctx;
    p->prob = *prob;
    p->g = g;
    p->NX = g.px * g.cx;
    p->NY = g.py * g.cy;
    p->hx = (g.x_hi - g.x_lo) / p->NX;
    p->hy = (g.y_hi - g.y_lo) / p->NY;
    p->dt = g.T / g.n_steps;
    p->rx = prob->diffusion * p->dt / (p->hx * p->hx);
    p->ry = prob->diffusion * p->dt / (p->hy * p->hy);
    p->u0.kind = prob->u0_kind;
    p->u0.nterms = prob->u0_nterms;
    std::memcpy(p->u0.p, prob->u0_params, sizeof(p->u0.p));
    for (auto& v : p->vline) v = -1;
    for (auto& v : p->hline) v = -1;
    const bool edges = g.outer == BRT_PDD_OUTER_LINES;
    uint64_t node_off = 0, bd_off = 0;
    for (int orient = 0; orient < 2; ++orient) {
      const uint32_t parts = orient == 0 ? g.px : g.py;
      for (uint32_t k = 0; k <= parts; ++k) {
        if (!edges && (k == 0 || k == parts)) continue;
        LineDev L{};
        L.orient = (uint32_t)orient;
        L.k = k;
        if (orient == 0) {
          L.c = g.x_lo + k * (g.x_hi - g.x_lo) / g.px;
          L.n_fine = p->NY + 1;
          L.ns = g.ns_y;
          L.s_lo = g.y_lo;
          L.hs = (g.y_hi - g.y_lo) / (g.ns_y - 1);
          L.hf = p->hy;
          p->vline[k] = (int16_t)p->lines.size();
          p->n_vlines += 1;
        } else {
          L.c = g.y_lo + k * (g.y_hi - g.y_lo) / g.py;
          L.n_fine = p->NX + 1;
          L.ns = g.ns_x;
          L.s_lo = g.x_lo;
          L.hs = (g.x_hi - g.x_lo) / (g.ns_x - 1);
          L.hf = p->hx;
          p->hline[k] = (int16_t)p->lines.size();
        }
        L.node_off = node_off;
        L.bd_off = bd_off;
        node_off += (uint64_t)g.nt * L.ns;
        bd_off += (uint64_t)(g.n_steps + 1) * L.n_fine;
        p->lines.push_back(L);
      }
    }
    p->n_nodes = node_off;
    p->bd_doubles = bd_off;
    p->max_ns = std::max(g.ns_x, g.ns_y);
    p->max_fine = std::max(p->NX, p->NY) + 1;
    p->W = (p->NX + 1 + 15) & ~15u;
    const size_t field = (size_t)p->W * (p->NY + 1) + kFieldLead + 1;
    const double bytes = 8.0 * ((double)p->bd_doubles + 3.0 * (double)field);
    if (bytes > 128e9) {
      pdd_free(p);
      return set_error(BRT_E_ARG, "pdd: grid needs %.1f GB of device memory (limit 128 GB)", bytes / 1e9);
    }
    int rc = BRT_OK;
    auto dev_alloc = [&](void** ptr, size_t n) {
      if (rc != BRT_OK) return;
      if (hipMalloc(ptr, n) != hipSuccess) rc = set_error(BRT_E_NOMEM, "pdd: device allocation of %zu bytes", n);
    };
    if (hipGetDevice(&p->device) != hipSuccess) rc = set_error(BRT_E_DEVICE, "pdd: no device");
    hipDeviceProp_t prop;
    if (rc == BRT_OK && hipGetDeviceProperties(&prop, p->device) != hipSuccess) rc = set_error(BRT_E_DEVICE, "pdd: device query");
    if (rc == BRT_OK) p->n_cu = prop.multiProcessorCount;
    const uint32_t rows = g.nt + 1;
    p->spl_rows = (size_t)p->lines.size() * rows * p->max_ns;
    p->spl_fine = (size_t)rows * p->lines.size() * p->max_fine;
    dev_alloc((void**)&p->d_lines, sizeof(LineDev) * p->lines.size());
    dev_alloc((void**)&p->d_bd, 8 * p->bd_doubles);
    for (double*& f : p->d_f) dev_alloc((void**)&f, 8 * field);
    p->seg = seg_length(g);
    dev_alloc((void**)&p->d_fac, 8 * 2 * (size_t)kSegs * p->seg);
    dev_alloc((void**)&p->d_spl, 8 * (3 * p->spl_rows + 3 * p->spl_fine));
    dev_alloc((void**)&p->d_sync, 4 * (size_t)kSyncWords);
    dev_alloc((void**)&p->d_node_u, 8 * std::max<uint64_t>(p->n_nodes, 1));
    dev_alloc((void**)&p->d_exy, 8 * (size_t)(p->NX + 1 + p->NY + 1));
    for (hipEvent_t& e : p->ev)
      if (rc == BRT_OK && hipEventCreate(&e) != hipSuccess) rc = set_error(BRT_E_DEVICE, "pdd: event creation");
    if (rc == BRT_OK) {
      std::vector<double> fac(2 * (size_t)kSegs * p->seg);
      pivot_reciprocals(p->rx, g.cx - 1, p->seg, fac.data());
      pivot_reciprocals(p->ry, g.cy - 1, p->seg, fac.data() + (size_t)kSegs * p->seg);
      std::vector<double> exy(p->NX + 1 + p->NY + 1, 1.0);
      if (prob->coef_mod != BRT_COEF_MOD_NONE) {
        for (uint32_t i = 0; i <= p->NX; ++i) {
          const double x = g.x_lo + i * p->hx;
          exy[i] = std::exp(-prob->coef_mod_beta[0] * x * x);
        }
        for (uint32_t j = 0; j <= p->NY; ++j) {
          const double y = g.y_lo + j * p->hy;
          exy[p->NX + 1 + j] = std::exp(-prob->coef_mod_beta[1] * y * y);
        }
      }
      if (hipMemcpy(p->d_exy, exy.data(), 8 * exy.size(), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(p->d_fac, fac.data(), 8 * fac.size(), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(p->d_lines, p->lines.data(), sizeof(LineDev) * p->lines.size(), hipMemcpyHostToDevice) != hipSuccess)
        rc = set_error(BRT_E_DEVICE, "pdd: upload");
    }
    if (rc == BRT_OK) {
      int per_cu = 0;
      p->lds = 8 * adi_lds_doubles(p->seg);
      if (hipFuncSetAttribute(adi_kernel_ptr(p->seg), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)p->lds) != hipSuccess)
        rc = set_error(BRT_E_DEVICE, "pdd: solver LDS of %zu bytes", p->lds);
      if (rc == BRT_OK &&
          (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adi_kernel_ptr(p->seg), adi_threads(p->seg),
                                                        p->lds) != hipSuccess ||
           per_cu < 1))
        rc = set_error(BRT_E_DEVICE, "pdd: solver occupancy query (LDS %zu bytes)", p->lds);
      const uint32_t nsub = g.px * g.py;
      const uint32_t lines = adi_lines(p->seg);
      const uint32_t x_items = nsub * ((g.cy - 1 + lines - 1) / lines);
      const uint32_t y_items = nsub * ((g.cx - 1 + lines - 1) / lines);
      const uint64_t cap = (uint64_t)per_cu * p->n_cu;
      const uint64_t items = std::max(x_items, y_items);
      if (nsub % kXcds == 0 && cap >= kXcds) {
        // Die-local barriers (the subdomains split over the dies): the fewest rounds of items over all
        // resident blocks, dealt evenly, a multiple of the die count.  On the 4 x 4 x 512^2 workload a
        // step takes 54 us at 256 blocks of 1024 threads (one item per block and phase), 61 at 128 and
        // 65-67 at 160 or 192 (uneven rounds).
        const uint64_t cap8 = cap / kXcds * kXcds;
        const uint64_t rounds = (items + cap8 - 1) / cap8;
        p->grid = (int)std::min<uint64_t>(cap8, ((items + rounds - 1) / rounds + kXcds - 1) / kXcds * kXcds);
      } else {
        // One barrier over the grid, with device-scope fences: half the compute units, a multiple of the
        // die count (a step of that workload took 76 us at 128 blocks and 88 at 256 with these fences:
        // more blocks lengthen every block's memory latency and add L2 write-backs at the barriers).
        const uint64_t half = std::max<uint64_t>(kXcds, (uint64_t)p->n_cu / 2 / kXcds * kXcds);
        p->grid = (int)std::min<uint64_t>({items, half, cap});
      }
    }
    if (rc != BRT_OK) {
      pdd_free(p);
      return rc;
    }
    *out = p;
    return BRT_OK;
  });
}

int brt_pdd_nodes(const brt_pdd* p, double* xy, double* t, uint64_t* n) {
  return brt::api_guard("brt_pdd_nodes", [&]() -> int {
    if (!p || !n) return set_error(BRT_E_ARG, "brt_pdd_nodes: NULL argument");
    *n = p->n_nodes;
    uint64_t i = 0;
    for (const LineDev& L : p->lines) {
      for (uint32_t k = 1; k <= p->g.nt; ++k) {
        const double tk = k * p->g.T / p->g.nt;
        for (uint32_t s = 0; s < L.ns; ++s, ++i) {
          const double pos = L.s_lo + s * L.hs;
          if (xy) {
            xy[2 * i] = L.orient == 0 ? L.c : pos;
            xy[2 * i + 1] = L.orient == 0 ? pos : L.c;
          }
          if (t) t[i] = tk;
        }
      }
    }
    return BRT_OK;
  });
}

int brt_pdd_lines(const brt_pdd* p, uint32_t* n_lines, uint32_t* orient, double* coord, uint32_t* n_fine) {
  return brt::api_guard("brt_pdd_lines", [&]() -> int {
    if (!p || !n_lines) return set_error(BRT_E_ARG, "brt_pdd_lines: NULL argument");
    *n_lines = (uint32_t)p->lines.size();
    for (size_t l = 0; l < p->lines.size(); ++l) {
      if (orient) orient[l] = p->lines[l].orient;
      if (coord) coord[l] = p->lines[l].c;
      if (n_fine) n_fine[l] = p->lines[l].n_fine;
    }
    return BRT_OK;
  });
}

int brt_pdd_interpolate(brt_pdd* p, const double* node_values, void* stream) {
  return brt::api_guard("brt_pdd_interpolate", [&]() -> int {
    if (!p || !node_values) return set_error(BRT_E_ARG, "brt_pdd_interpolate: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    SplineArgs a{};
    a.lines = p->d_lines;
    a.n_lines = (uint32_t)p->lines.size();
    a.rows = p->g.nt + 1;
    a.max_ns = p->max_ns;
    a.max_fine = p->max_fine;
    a.node_values = node_values;
    a.vals = p->d_spl;
    a.mom = a.vals + p->spl_rows;
    a.cp = a.mom + p->spl_rows;
    a.rowsv = a.cp + p->spl_rows;
    a.tmom = a.rowsv + p->spl_fine;
    a.tcp = a.tmom + p->spl_fine;
    a.bd = p->d_bd;
    a.ht = p->g.T / p->g.nt;
    a.dt = p->dt;
    a.n_steps = p->g.n_steps;
    a.u0 = p->u0;
    PDD_TRY(hipEventRecord(p->ev[2], s));
    const uint32_t nr = a.n_lines * a.rows;
    spline_rows_kernel<<<(nr + 63) / 64, 64, 0, s>>>(a);
    PDD_TRY(hipGetLastError());
    spline_s_kernel<<<dim3((p->max_fine + 255) / 256, nr), 256, 0, s>>>(a);
    PDD_TRY(hipGetLastError());
    spline_t_kernel<<<dim3((p->max_fine + 255) / 256, a.n_lines), 256, 0, s>>>(a);
    PDD_TRY(hipGetLastError());
    PDD_TRY(hipEventRecord(p->ev[3], s));
    p->recorded[1] = true;
    return BRT_OK;
  });
}

int brt_pdd_boundary(const brt_pdd* p, uint32_t line, double* dst, void* stream) {
  return brt::api_guard("brt_pdd_boundary", [&]() -> int {
    if (!p || !dst) return set_error(BRT_E_ARG, "brt_pdd_boundary: NULL argument");
    if (line >= p->lines.size()) return set_error(BRT_E_ARG, "brt_pdd_boundary: no line %u", line);
    const LineDev& L = p->lines[line];
    PDD_TRY(hipMemcpyAsync(dst, p->d_bd + L.bd_off, 8 * (size_t)(p->g.n_steps + 1) * L.n_fine, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return BRT_OK;
  });
}

int brt_pdd_solve(brt_pdd* p, uint32_t steps, double* field, void* stream) {
  return brt::api_guard("brt_pdd_solve", [&]() -> int {
    if (!p || !field) return set_error(BRT_E_ARG, "brt_pdd_solve: NULL argument");
    if (steps < 1 || steps > p->g.n_steps) return set_error(BRT_E_ARG, "brt_pdd_solve: steps must be 1..%u", p->g.n_steps);
    hipStream_t s = (hipStream_t)stream;
    const brt_pdd_grid& g = p->g;
    PDD_TRY(hipEventRecord(p->ev[4], s));
    FieldArgs fa{};
    fa.f0 = p->d_f[0] + kFieldLead;
    fa.f1 = p->d_f[1] + kFieldLead;
    fa.W = p->W;
    fa.bd = p->d_bd;
    fa.lines = p->d_lines;
    fa.NX = p->NX;
    fa.NY = p->NY;
    fa.cx = g.cx;
    fa.cy = g.cy;
    fa.zero_outer = g.outer == BRT_PDD_OUTER_ZERO;
    fa.x_lo = g.x_lo;
    fa.y_lo = g.y_lo;
    fa.hx = p->hx;
    fa.hy = p->hy;
    std::memcpy(fa.vline, p->vline, sizeof(fa.vline));
    std::memcpy(fa.hline, p->hline, sizeof(fa.hline));
    fa.u0 = p->u0;
    const uint64_t n_field = (uint64_t)(p->NX + 1) * (p->NY + 1);
    init_field_kernel<<<(unsigned)((n_field + 255) / 256), 256, 0, s>>>(fa);
    PDD_TRY(hipGetLastError());
    PDD_TRY(hipMemsetAsync(p->d_sync, 0, 4 * (size_t)kSyncWords, s));

    AdiArgs a{};
    a.f0 = p->d_f[0] + kFieldLead;
    a.f1 = p->d_f[1] + kFieldLead;
    a.yrhs = p->d_f[2] + kFieldLead;
    a.bd = p->d_bd;
    a.lines = p->d_lines;
    a.inv_x = p->d_fac;
    a.inv_y = p->d_fac + (size_t)kSegs * p->seg;
    a.sync = p->d_sync;
    int rate_khz = 0;
    PDD_TRY(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, p->device));
    a.spin_limit = (uint64_t)(kBarrierSeconds * 1e3 * (rate_khz > 0 ? rate_khz : 100000));
    // f = c_1 u + m(x, y, t) P(u): P holds the modulated terms, c_1 among them when it is modulated too
    const bool lin = p->prob.coef_mod == BRT_COEF_MOD_GAUSS_TIME_ALL;
    for (int j = 0; j < 8; ++j) a.pcoef[j] = p->prob.coef[j];
    a.pcoef[1] = lin ? p->prob.coef[1] : 0.0;
    const bool cmod = p->prob.coef_mod != BRT_COEF_MOD_NONE;
    a.cm_pow = cmod ? p->prob.coef_mod_pow : 0u;
    a.cm_t0 = p->prob.coef_mod_t0;
    a.c1 = lin ? 0.0 : p->prob.coef[1];
    a.dt = p->dt;
    a.ex = p->d_exy;
    a.ey = p->d_exy + p->NX + 1;
    a.rx2 = 0.5 * p->rx;
    a.ry2 = 0.5 * p->ry;
    a.dt2 = 0.5 * p->dt;
    a.W = p->W;
    a.px = g.px;
    a.py = g.py;
    a.cx = g.cx;
    a.cy = g.cy;
    a.steps = steps;
    a.nblocks = (uint32_t)p->grid;
    // Subdomains are decoupled, so blocks that own whole subdomains in both phases synchronise among
    // themselves only: one group per subdomain when the grid splits evenly over them (a group then waits
    // only for the blocks of its own subdomain), else one per die, else one over the grid.
    const uint32_t nsub = g.px * g.py, grid = (uint32_t)p->grid;
    a.groups = nsub % kXcds != 0 || grid % kXcds != 0 ? 1u : grid % nsub == 0 && nsub <= kMaxGroups ? nsub : kXcds;
    p->last_groups = a.groups;
    const uint32_t lines = adi_lines(p->seg), threads = adi_threads(p->seg);
    a.x_blk = (g.cy - 1 + lines - 1) / lines;
    a.y_blk = (g.cx - 1 + lines - 1) / lines;
    a.n_vlines = p->n_vlines;
    a.bv = (p->NY + 1 + threads - 1) / threads;
    a.bh = (p->NX + 1 + threads - 1) / threads;
    a.n_lines = (uint32_t)p->lines.size();
    std::memcpy(a.vline, p->vline, sizeof(a.vline));
    std::memcpy(a.hline, p->hline, sizeof(a.hline));
    a.v_fine = p->NY + 1;
    a.h_fine = p->NX + 1;
    for (size_t l = 0; l < p->lines.size(); ++l) a.bd_off[l] = p->lines[l].bd_off;
    void* kargs[] = {&a};
    PDD_TRY(hipLaunchCooperativeKernel(adi_kernel_ptr(p->seg), dim3(p->grid), dim3(threads), kargs,
                                       (unsigned)p->lds, s));
    const double* result = ((steps & 1) ? p->d_f[1] : p->d_f[0]) + kFieldLead;
    PDD_TRY(hipMemcpy2DAsync(field, 8 * (size_t)(p->NX + 1), result, 8 * (size_t)p->W, 8 * (size_t)(p->NX + 1), p->NY + 1,
                             hipMemcpyDeviceToDevice, s));
    PDD_TRY(hipEventRecord(p->ev[5], s));
    p->recorded[2] = true;
    return BRT_OK;
  });
}

int brt_pdd_run(brt_pdd* p, const brt_mc* mc, uint64_t trees_per_node, double* node_u, double* field, void* stream) {
  return brt::api_guard("brt_pdd_run", [&]() -> int {
    if (!p || !mc || !field) return set_error(BRT_E_ARG, "brt_pdd_run: NULL argument");
    if (mc->struct_size != sizeof(brt_mc)) return set_error(BRT_E_ARG, "brt_mc.struct_size mismatch");
    if (trees_per_node < 1 || trees_per_node > 0xffffffffull) return set_error(BRT_E_ARG, "brt_pdd_run: trees_per_node must be 1..2^32-1");
    hipStream_t s = (hipStream_t)stream;
    if (p->plan && (std::memcmp(&p->plan_mc, mc, sizeof(brt_mc)) != 0 || p->plan_trees != trees_per_node)) {
      brt_plan_destroy(p->plan);
      p->plan = nullptr;
    }
    if (!p->plan) {
      std::vector<double> xy(2 * p->n_nodes), t(p->n_nodes);
      std::vector<uint64_t> nt(p->n_nodes, trees_per_node);
      uint64_t n = 0;
      brt_pdd_nodes(p, xy.data(), t.data(), &n);
      brt_points pts{};
      pts.struct_size = sizeof(pts);
      pts.n = (uint32_t)n;
      pts.x = xy.data();
      pts.t = t.data();
      pts.n_trees = nt.data();
      const int rc = brt_plan_create(p->ctx, 1, &p->prob, mc, &pts, &p->plan);
      if (rc != BRT_OK) {
        p->plan = nullptr;
        return rc;
      }
      p->plan_mc = *mc;
      p->plan_trees = trees_per_node;
    }
    double* u = node_u ? node_u : p->d_node_u;
    brt_out o{};
    o.struct_size = sizeof(o);
    o.u = u;
    PDD_TRY(hipEventRecord(p->ev[0], s));
    int rc = brt_plan_execute(p->plan, &o, stream);
    if (rc != BRT_OK) return rc;
    PDD_TRY(hipEventRecord(p->ev[1], s));
    p->recorded[0] = true;
    rc = brt_pdd_interpolate(p, u, stream);
    if (rc != BRT_OK) return rc;
    return brt_pdd_solve(p, p->g.n_steps, field, stream);
  });
}

int brt_pdd_get_barrier(brt_pdd* p, uint32_t* groups, uint32_t* die_local) {
  return brt::api_guard("brt_pdd_get_barrier", [&]() -> int {
    if (!p || !groups || !die_local) return set_error(BRT_E_ARG, "brt_pdd_get_barrier: NULL argument");
    *groups = *die_local = 0;
    if (!p->recorded[2]) return BRT_OK;
    PDD_TRY(hipEventSynchronize(p->ev[5]));
    uint32_t w[kSyncWords];
    PDD_TRY(hipMemcpy(w, p->d_sync, sizeof(w), hipMemcpyDeviceToHost));
    *groups = p->last_groups;
    for (uint32_t g = 0; g < p->last_groups; ++g) *die_local += __builtin_popcount(w[5 + 2 * g]) == 1 ? 1u : 0u;
    return BRT_OK;
  });
}

int brt_pdd_get_timing(brt_pdd* p, double* ms) {
  return brt::api_guard("brt_pdd_get_timing", [&]() -> int {
    if (!p || !ms) return set_error(BRT_E_ARG, "brt_pdd_get_timing: NULL argument");
    for (int k = 0; k < 3; ++k) {
      ms[k] = 0.0;
      if (!p->recorded[k]) continue;
      PDD_TRY(hipEventSynchronize(p->ev[2 * k + 1]));
      float v = 0.f;
      PDD_TRY(hipEventElapsedTime(&v, p->ev[2 * k], p->ev[2 * k + 1]));
      ms[k] = v;
    }
    p->recorded[0] = false;
    uint32_t abort_word = 0;
    PDD_TRY(hipMemcpy(&abort_word, p->d_sync + 2, 4, hipMemcpyDeviceToHost));
    if (abort_word) return set_error(BRT_E_DEVICE, "pdd: the solver's grid barrier timed out");
    return BRT_OK;
  });
}

void brt_pdd_destroy(brt_pdd* p) { pdd_free(p); }

}  // extern "C"
