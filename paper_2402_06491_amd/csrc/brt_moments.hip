// Moment reduction and FP64 finalize of the random-tree Monte Carlo (gfx950).
//
//  reduce_kernel    one wave per segment of one point's trees: per-bin count, sum F, sum F^2 with
//                   per-lane LDS accumulators (each lane sums its own records in index order) and a
//                   fixed-order wave reduction, so the result does not depend on scheduling.
//  finalize_kernel  one wave per point, FP64: Neumaier-compensated sums over the point's segments,
//                   coefficients a_n = e^{mu t} S1_n / N (the sample mean of the functional, Sec. 2.4)
//                   and their variances, the [L/M] Pade approximant at z = 1 (Sec. 2.1 end) by LU with
//                   partial pivoting, and its delta-method standard error from the exact gradient of
//                   the approximant with respect to the coefficients.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "brt_internal.h"

namespace brt {

constexpr int kRedGroup = 16;  // moment bins accumulated per pass over a segment
constexpr int kRedBatch = 32;  // records loaded per lane before they are accumulated
constexpr uint32_t kAbsent = 0xffffffffu;  // marks a batch slot past the end of the segment (no real
                                           // record has every flag bit set)

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Partials layout per segment: bins 0..B-1 (B-1 is the tail, Ne > max_order without pruning) with
// moments, then counts of overflow, capped and depth-exceeded trees.
__global__ __launch_bounds__(64) void reduce_kernel(ReduceArgs a) {
  __shared__ double ls1[kRedGroup][kWave];
  __shared__ double ls2[kRedGroup][kWave];
  __shared__ uint32_t lcnt[kRedGroup][kWave];

  const uint32_t seg = blockIdx.x;
  const uint32_t lane = threadIdx.x;
  const Segment sg = a.segs[seg];
  const PointRec& pr = a.points[sg.point];
  const double* F = a.tree_f + pr.tree_base;
  const uint32_t* M = a.tree_meta + pr.tree_base;
  const uint32_t B = a.n_bins;
  Partial* out = a.partials + (size_t)sg.out * (B + 3);

  unsigned long long nodes = 0;
  uint32_t n_ovf = 0, n_cap = 0, n_dep = 0;
  for (uint32_t g0 = 0; g0 < B; g0 += kRedGroup) {
    for (int k = 0; k < kRedGroup; ++k) {
      ls1[k][lane] = 0.0;
      ls2[k][lane] = 0.0;
      lcnt[k][lane] = 0u;
    }
    bool above = false;
    // records are loaded kRedBatch at a time so that many loads are in flight per lane; each lane
    // still adds its records in increasing index order
    for (uint32_t i0 = sg.begin + lane; i0 < sg.end; i0 += kWave * kRedBatch) {
      uint32_t mb[kRedBatch];
      double fb[kRedBatch];
#pragma unroll
      for (int j = 0; j < kRedBatch; ++j) {
        const uint32_t i = i0 + j * kWave;
        mb[j] = i < sg.end ? M[i] : kAbsent;
        fb[j] = i < sg.end ? F[i] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < kRedBatch; ++j) {
      const uint32_t m = mb[j];
      const double f = fb[j];
      if (m == kAbsent) continue;
      if (g0 == 0) {
        nodes += (unsigned long long)(m >> kMetaNodesShift);
        n_ovf += (m >> 8) & 1u;
        n_cap += (m >> 9) & 1u;
        n_dep += (m >> 10) & 1u;
      }
      if (m & (kMetaOverflow | kMetaCapped | kMetaDepth)) continue;
      const uint32_t ne = m & kMetaNeMask;
      const uint32_t bin = ne < B - 1 ? ne : B - 1;
      if (bin >= g0 && bin < g0 + kRedGroup) {
        const uint32_t k = bin - g0;
        ls1[k][lane] += f;
        ls2[k][lane] += f * f;
        lcnt[k][lane] += 1u;
      }
      above |= bin >= g0 + kRedGroup;
      }
    }
    for (int k = 0; k < kRedGroup; ++k) {
      const uint32_t b = g0 + k;
      const double v1 = wave_sum_f64(ls1[k][lane]);
      const double v2 = wave_sum_f64(ls2[k][lane]);
      const unsigned long long c = wave_sum_u64((unsigned long long)lcnt[k][lane]);
      if (lane == 0 && b < B) {
        out[b].count = c;
        out[b].s1 = v1;
        out[b].s2 = v2;
      }
    }
    if (__ballot(above) == 0) {
      for (uint32_t b = g0 + kRedGroup + lane; b < B; b += kWave) {
        out[b].count = 0;
        out[b].s1 = 0.0;
        out[b].s2 = 0.0;
      }
      break;
    }
  }
  nodes = wave_sum_u64(nodes);
  const unsigned long long o = wave_sum_u64(n_ovf), c = wave_sum_u64(n_cap), d = wave_sum_u64(n_dep);
  if (lane == 0) {
    a.seg_nodes[sg.out] = nodes;
    out[B] = Partial{o, 0.0, 0.0};
    out[B + 1] = Partial{c, 0.0, 0.0};
    out[B + 2] = Partial{d, 0.0, 0.0};
  }
}

constexpr int kMaxBins = 128;  // B = max_order + 2 <= 128
constexpr int kMaxPadeM = 16;

// LU factorisation with partial pivoting, in place (row-major M x M, multipliers below the
// diagonal), perm[i] = original row now at position i.  Singular when an entry is not finite or the
// smallest pivot magnitude is at most 1e-13 times the largest.
__device__ bool lu_factor(double* T, int M, int* perm) {
  double pmax = 0.0, pmin = 1e308;
  for (int i = 0; i < M; ++i) perm[i] = i;
  for (int c = 0; c < M; ++c) {
    int piv = c;
    double best = fabs(T[c * M + c]);
    for (int r = c + 1; r < M; ++r) {
      const double v = fabs(T[r * M + c]);
      if (v > best || !(v == v)) {
        best = v;
        piv = r;
      }
    }
    if (!(best == best) || best > 1.7e308) return false;
    if (piv != c) {
      for (int j = 0; j < M; ++j) {
        const double tmp = T[c * M + j];
        T[c * M + j] = T[piv * M + j];
        T[piv * M + j] = tmp;
      }
      const int tp = perm[c];
      perm[c] = perm[piv];
      perm[piv] = tp;
    }
    if (best == 0.0) return false;
    pmax = best > pmax ? best : pmax;
    pmin = best < pmin ? best : pmin;
    for (int r = c + 1; r < M; ++r) {
      const double l = T[r * M + c] / T[c * M + c];
      T[r * M + c] = l;
      for (int j = c + 1; j < M; ++j) T[r * M + j] -= l * T[c * M + j];
    }
  }
  return pmin > 1e-13 * pmax;
}

struct PadeResult {
  double value;
  int L, M;       // degrees used
  bool lowered;
};

// [L/M] at z = 1 of sum_n a_n z^n.  The denominator q (q_0 = 1) satisfies
// sum_{j=0}^{M} q_j a_{k-j} = 0 for k = L+1..L+M (a_i = 0 for i < 0); with partial sums
// A_m = a_0 + ... + a_m the value is sum_j q_j A_{L-j} / sum_j q_j.  A singular system moves to
// [L+1/M-1] (same total order), down to M = 0 (the partial sum).  On return T holds the LU factors
// (M x M), perm the pivoting and q the denominator.
__device__ PadeResult pade(const double* a, int L, int M, double* q, double* T, int* perm) {
  PadeResult r{0.0, L, M, false};
  while (true) {
    q[0] = 1.0;
    if (M == 0) break;
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        const int k = L + i - j;  // T_{ij} = a_{L+i-j}, i, j = 1..M
        T[i * M + j] = k >= 0 ? a[k] : 0.0;
      }
    bool ok = lu_factor(T, M, perm);
    for (int i = 0; ok && i < M; ++i)
      if (!(fabs(a[L + 1 + i]) <= 1.7e308)) ok = false;
    if (ok) {
      double y[kMaxPadeM];
      for (int i = 0; i < M; ++i) {  // forward: L y = P (-b)
        double s = -a[L + 1 + perm[i]];
        for (int j = 0; j < i; ++j) s -= T[i * M + j] * y[j];
        y[i] = s;
      }
      for (int i = M - 1; i >= 0; --i) {  // backward: U q = y
        double s = y[i];
        for (int j = i + 1; j < M; ++j) s -= T[i * M + j] * q[j + 1];
        q[i + 1] = s / T[i * M + i];
      }
      break;
    }
    L += 1;
    M -= 1;
    r.lowered = true;
  }
  double num = 0.0, den = 0.0;
  for (int j = 0; j <= M; ++j) {
    double A = 0.0;
    for (int i = 0; i <= L - j; ++i) A += a[i];
    num += q[j] * A;
    den += q[j];
  }
  r.value = num / den;
  r.L = L;
  r.M = M;
  return r;
}

// Gradient g_k = d value / d a_k (k = 0..L+M) of the approximant returned by pade().  With
// D = sum_j q_j and c_j = (A_{L-j} - value)/D, solve T^T y = c; then
//   g_k = [k <= L] sum_{j=0}^{min(M, L-k)} q_j / D  -  sum_{i=1}^{M} y_i q_{L+i-k}  (0 <= L+i-k <= M).
__device__ void pade_gradient(const double* a, const PadeResult& r, const double* q, const double* T,
                              const int* perm, double* g) {
  const int L = r.L, M = r.M;
  double D = 0.0;
  for (int j = 0; j <= M; ++j) D += q[j];
  double y[kMaxPadeM];
  if (M > 0) {
    double v[kMaxPadeM];
    for (int i = 0; i < M; ++i) {  // U^T v = c
      double A = 0.0;
      for (int m = 0; m <= L - (i + 1); ++m) A += a[m];
      double s = (A - r.value) / D;
      for (int j = 0; j < i; ++j) s -= T[j * M + i] * v[j];
      v[i] = s / T[i * M + i];
    }
    double w[kMaxPadeM];
    for (int i = M - 1; i >= 0; --i) {  // L^T w = v
      double s = v[i];
      for (int j = i + 1; j < M; ++j) s -= T[j * M + i] * w[j];
      w[i] = s;
    }
    for (int i = 0; i < M; ++i) y[perm[i]] = w[i];  // P y = w
  }
  for (int k = 0; k <= L + M; ++k) {
    double gk = 0.0;
    if (k <= L) {
      const int jm = (L - k) < M ? (L - k) : M;
      for (int j = 0; j <= jm; ++j) gk += q[j];
      gk /= D;
    }
    for (int i = 1; i <= M; ++i) {
      const int j = L + i - k;
      if (j >= 0 && j <= M) gk -= y[i - 1] * q[j];
    }
    g[k] = gk;
  }
}

__global__ __launch_bounds__(64) void finalize_kernel(FinalizeArgs a) {
  __shared__ double coef[kMaxBins];
  __shared__ double m1[kMaxBins];
  __shared__ double m2[kMaxBins];
  __shared__ double grad[kMaxBins];
  __shared__ double T[kMaxPadeM * kMaxPadeM];
  __shared__ double q[kMaxPadeM + 1];
  __shared__ int perm[kMaxPadeM];
  __shared__ unsigned long long extra[3];

  const uint32_t p = blockIdx.x;
  const uint32_t lane = threadIdx.x;
  const PointRec& pr = a.points[p];
  const uint32_t row = pr.out_row;  // output row of this point
  const uint32_t B = a.n_bins;
  const uint32_t NB = B + 3;
  const double N = (double)pr.n_total;
  const double scale = exp(pr.mu * pr.t);

  for (uint32_t b = lane; b < NB; b += kWave) {
    // Neumaier-compensated sums over the point's segments, in segment order
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    unsigned long long cnt = 0;
    for (uint32_t s = 0; s < pr.seg_count; ++s) {
      const Partial& pt = a.partials[(size_t)(pr.seg_begin + s) * NB + b];
      cnt += pt.count;
      const double t1 = s1 + pt.s1;
      c1 += fabs(s1) >= fabs(pt.s1) ? (s1 - t1) + pt.s1 : (pt.s1 - t1) + s1;
      s1 = t1;
      const double t2 = s2 + pt.s2;
      c2 += fabs(s2) >= fabs(pt.s2) ? (s2 - t2) + pt.s2 : (pt.s2 - t2) + s2;
      s2 = t2;
    }
    s1 += c1;
    s2 += c2;
    if (a.hist) a.hist[(size_t)row * NB + b] = cnt;
    if (b < B) {
      if (a.s1) a.s1[(size_t)row * B + b] = s1;
      if (a.s2) a.s2[(size_t)row * B + b] = s2;
      const double mm1 = N > 0 ? s1 / N : 0.0;
      const double mm2 = N > 0 ? s2 / N : 0.0;
      m1[b] = mm1;
      m2[b] = mm2;
      coef[b] = scale * mm1;
      const double var = N > 1 ? scale * scale * (mm2 - mm1 * mm1) / (N - 1.0) : 0.0;
      if (a.coef) a.coef[(size_t)row * B + b] = scale * mm1;
      if (a.coef_var) a.coef_var[(size_t)row * B + b] = var;
    } else {
      extra[b - B] = cnt;
    }
  }
  __syncthreads();
  unsigned long long nodes = 0;
  for (uint32_t s = lane; s < pr.seg_count; s += kWave) nodes += a.seg_nodes[pr.seg_begin + s];
  nodes = wave_sum_u64(nodes);

  if (lane == 0) {
    uint32_t fl = 0;
    if (extra[0] > 0) fl |= BRT_FLAG_OVERFLOW;
    if (extra[1] > 0) fl |= BRT_FLAG_CAPPED;
    if (extra[2] > 0) fl |= BRT_FLAG_DEPTH;
    double psum = 0.0;
    for (uint32_t b = 0; b < B; ++b) psum += coef[b];
    const PadeResult r = pade(coef, (int)a.pade_L, (int)a.pade_M, q, T, perm);
    if (r.lowered) fl |= BRT_FLAG_LOWERED;
    // pole test: Q(0) = 1; flag a value <= 1e-8 anywhere on [0, 1]
    for (int k = 1; k <= 64; ++k) {
      const double z = k / 64.0;
      double qz = 0.0, zp = 1.0;
      for (int j = 0; j <= r.M; ++j) {
        qz += q[j] * zp;
        zp *= z;
      }
      if (!(qz > 1e-8)) {
        fl |= BRT_FLAG_POLE;
        break;
      }
    }
    // delta method: Var(u) = sum_kl g_k g_l Cov(a_k, a_l) with
    // Cov(a_k, a_l) = scale^2 (delta_kl m2_k - m1_k m1_l) / (N - 1)
    pade_gradient(coef, r, q, T, perm, grad);
    double gg = 0.0, gm = 0.0;
    for (int k = 0; k <= r.L + r.M; ++k) {
      gg += grad[k] * grad[k] * m2[k];
      gm += grad[k] * m1[k];
    }
    const double var = N > 1 ? scale * scale * (gg - gm * gm) / (N - 1.0) : 0.0;
    if (a.u) a.u[row] = r.value;
    if (a.se) a.se[row] = sqrt(var > 0.0 ? var : 0.0);
    if (a.psum) a.psum[row] = psum;
    if (a.flags) a.flags[row] = fl;
    if (a.nodes) a.nodes[row] = nodes;
  }
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  if (a.n_segs == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(a.n_segs), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  if (a.n_points == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(a.n_points), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

}  // namespace brt
