// Moment reduction and FP64 finalize of the random-tree Monte Carlo (gfx950).
//
//  reduce_kernel    one wave per segment of one point's trees: per-bin count, compensated
//                   (double-double) sum of F and plain sum of F*F, each lane adding its records in index
//                   order, the lanes joined by a fixed butterfly.
//  finalize_kernel  one wave per point, FP64: the point's segment sums joined exactly (integer digit
//                   words) and rounded once, so the result does not depend on the order of the segments,
//                   coefficients a_n = e^{mu t} S1_n / N (the sample mean of the functional, Sec. 2.4)
//                   and their variances, the [L/M] Pade approximant at z = 1 (Sec. 2.1 end) with its
//                   degrees chosen by the singular values of the denominator's linear conditions (one-sided
//                   Jacobi) and its denominator by LU with partial pivoting, its delta-method standard error
//                   and sensitivity from the exact gradient of the approximant with respect to the
//                   coefficients, the neighbouring orders [L-1/M] and [L/M-1] (Sec. 2.4 judges an
//                   approximant across numbers of coefficients), and a count of its poles near [0, 1]
//                   by the argument principle.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "brt_internal.h"

namespace brt {

constexpr int kRedGroup = 16;   // bins accumulated per pass over a segment (per-lane sums in LDS)
static_assert(kSegTrees <= 65535, "per-lane counts are 16-bit");
constexpr int kRedBatch = 32;   // records loaded per lane before they are accumulated
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

// A finite double v as sign, significand and position: |v| = m 2^(p - 1074) with m < 2^53 and p >= 0
// (p = biased exponent - 1 for normal numbers, 0 for subnormal ones).
__host__ __device__ __forceinline__ void split_double(double v, uint32_t* p, uint64_t* m, bool* neg) {
  uint64_t bits;
  memcpy(&bits, &v, sizeof(bits));
  const uint32_t e = (uint32_t)(bits >> 52) & 0x7ffu;
  const uint64_t frac = bits & ((1ull << 52) - 1);
  *neg = (bits >> 63) != 0;
  *m = e ? (frac | (1ull << 52)) : frac;
  *p = e ? e - 1 : 0;
}

// The three signed digits that add v (finite, nonzero) to a digit-word accumulator at words k, k+1, k+2.
__host__ __device__ __forceinline__ void digits_of(double v, uint32_t* k, unsigned long long* d) {
  uint32_t p;
  uint64_t m;
  bool neg;
  split_double(v, &p, &m, &neg);
  *k = p >> 5;
  const uint32_t sh = p & 31u;
  const uint64_t lo = m << sh;
  const uint64_t hi = sh ? (m >> (64 - sh)) : 0ull;
  const uint64_t d0 = lo & 0xffffffffull, d1 = lo >> 32, d2 = hi;
  d[0] = neg ? (unsigned long long)(0ull - d0) : d0;  // two's complement: adding it subtracts the digit
  d[1] = neg ? (unsigned long long)(0ull - d1) : d1;
  d[2] = neg ? (unsigned long long)(0ull - d2) : d2;
}

// The digit words of one sum (kAccWords signed words, word k weighing 2^(32k - 1074), word k at
// w[k * stride]) rounded once to the nearest double, ties to even; special = the non-finite values seen
// (bit 0 +inf, bit 1 -inf, bit 2 NaN).
__host__ __device__ double acc_round(const unsigned long long* w, int stride, unsigned long long special) {
  if (special & 4ull) return NAN;
  if ((special & 3ull) == 3ull) return NAN;
  if (special & 1ull) return INFINITY;
  if (special & 2ull) return -INFINITY;
  // carry-propagate into 32-bit digits; the final carry is the sign (0 or -1)
  uint32_t dg[kAccWords];
  long long carry = 0;
  for (int k = 0; k < kAccWords; ++k) {
    const long long t = (long long)w[(size_t)k * stride] + carry;
    dg[k] = (uint32_t)((unsigned long long)t & 0xffffffffull);
    carry = t >> 32;
  }
  const bool neg = carry < 0;
  if (neg) {  // magnitude of the two's complement number
    unsigned long long c = 1;
    for (int k = 0; k < kAccWords; ++k) {
      const unsigned long long t = (unsigned long long)(uint32_t)~dg[k] + c;
      dg[k] = (uint32_t)t;
      c = t >> 32;
    }
  }
  int K = kAccWords - 1;
  while (K >= 0 && dg[K] == 0) --K;
  if (K < 0) return 0.0;
  // the 64 bits from the leading one down (left-aligned), and whether anything nonzero lies below them
  int nb = 32;
  while (!((dg[K] >> (nb - 1)) & 1u)) --nb;  // bit length of the leading digit
  const long long msb = 32ll * K + nb - 1;  // position of the leading one (bit 0 weighs 2^-1074)
  // digits K, K-1, K-2 as a 96-bit window [d2 d1 d0], shifted so that the leading one is bit 63 of top
  const unsigned long long d2 = dg[K], d1 = K >= 1 ? dg[K - 1] : 0u, d0 = K >= 2 ? dg[K - 2] : 0u;
  const unsigned long long hi64 = (d2 << 32) | d1;  // bits 32K + 31 .. 32K - 32
  const int sh = 32 - nb;                           // left shift that puts the leading one at bit 63
  const unsigned long long top = sh ? (hi64 << sh) | (d0 >> (32 - sh)) : hi64;
  bool sticky = sh ? ((d0 & ((1ull << (32 - sh)) - 1)) != 0) : (d0 != 0);
  for (int k = 0; k < K - 2 && !sticky; ++k) sticky = dg[k] != 0;
  double r;
  if (msb <= 52) {
    // at most 53 significant bits with lowest weight 2^-1074: exactly representable
    r = ldexp((double)(top >> (63 - msb)), -1074);
  } else {
    unsigned long long mant = top >> 11;          // 53 bits
    const unsigned long long rem = top & 0x7ffull;
    if (rem > 0x400ull || (rem == 0x400ull && (sticky || (mant & 1ull)))) mant += 1;
    long long e2 = msb - 52 - 1074;
    if (mant >> 53) {
      mant >>= 1;
      e2 += 1;
    }
    r = e2 > 1023 - 52 ? INFINITY : ldexp((double)mant, (int)e2);
  }
  return neg ? -r : r;
}

// Error-free sum (Knuth's TwoSum): s + e = a + b exactly, s = fl(a + b).
__host__ __device__ __forceinline__ void two_sum(double a, double b, double* s, double* e) {
  const double t = a + b;
  const double bb = t - a;
  *e = (a - (t - bb)) + (b - bb);
  *s = t;
}

// Compensated (double-double) running sum hi + lo: hi takes the rounded sum, lo the exact rounding errors.
__device__ __forceinline__ void dd_add(double* hi, double* lo, double x) {
  double s, e;
  two_sum(*hi, x, &s, &e);
  *hi = s;
  *lo += e;
}

// Sum of a double-double over the wave by a fixed butterfly.
__device__ __forceinline__ void wave_sum_dd(double* hi, double* lo) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double h2 = __shfl_xor(*hi, off), l2 = __shfl_xor(*lo, off);
    double s, e;
    two_sum(*hi, h2, &s, &e);
    const double l = (*lo + l2) + e;
    two_sum(s, l, hi, lo);
  }
}

// One wave per segment of one point's trees: per bin, the count, the sum of F as a compensated
// (double-double) sum and the sum of F*F (each square rounded to FP64), every lane adding its records in
// index order into its own LDS column, the lanes joined by a fixed butterfly.  Non-finite values
// propagate into the sums (the finalize classifies them).
__global__ __launch_bounds__(kWave) void reduce_kernel(ReduceArgs a) {
  __shared__ double s1h[kRedGroup][kWave], s1l[kRedGroup][kWave], s2[kRedGroup][kWave];
  __shared__ uint16_t lcnt[kRedGroup][kWave];  // a segment holds at most kSegTrees <= 65535 trees

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
      s1h[k][lane] = 0.0;
      s1l[k][lane] = 0.0;
      s2[k][lane] = 0.0;
      lcnt[k][lane] = 0;
    }
    bool above = false;
    // records are loaded kRedBatch at a time so that many loads are in flight per lane; each lane still
    // adds its records in increasing index order
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
        above |= bin >= g0 + kRedGroup;
        if (bin < g0 || bin >= g0 + kRedGroup) continue;
        const uint32_t k = bin - g0;
        const double f = fb[j];
        lcnt[k][lane] += 1;
        dd_add(&s1h[k][lane], &s1l[k][lane], f);
        s2[k][lane] += __dmul_rn(f, f);  // the square rounded on its own, not fused into the sum
      }
    }
    for (int k = 0; k < kRedGroup; ++k) {
      const uint32_t b = g0 + k;
      double h = s1h[k][lane], l = s1l[k][lane];
      wave_sum_dd(&h, &l);
      const double v2 = wave_sum_f64(s2[k][lane]);
      const unsigned long long c = wave_sum_u64((unsigned long long)lcnt[k][lane]);
      if (lane == 0 && b < B) out[b] = Partial{c, h, l, v2};
    }
    if (__ballot(above) == 0) {
      for (uint32_t b = g0 + kRedGroup + lane; b < B; b += kWave) out[b] = Partial{0, 0.0, 0.0, 0.0};
      break;
    }
  }
  nodes = wave_sum_u64(nodes);
  const unsigned long long o = wave_sum_u64(n_ovf), c = wave_sum_u64(n_cap), d = wave_sum_u64(n_dep);
  if (lane == 0) {
    a.seg_nodes[sg.out] = nodes;
    out[B] = Partial{o, 0.0, 0.0, 0.0};
    out[B + 1] = Partial{c, 0.0, 0.0, 0.0};
    out[B + 2] = Partial{d, 0.0, 0.0, 0.0};
  }
}

constexpr int kMaxBins = 128;  // B = max_order + 2 <= 128
constexpr int kMaxPadeM = 16;
// Degree selection of the approximant: a singular value of the denominator's linear conditions counts as
// zero when it is at most kPadeTol times the 2-norm of the coefficients a_0..a_{L+M}.
constexpr double kPadeTol = 1e-12;
// A zero of the denominator within kPoleDist of the segment [0, 1] is reported (BRT_FLAG_POLE), and a value
// whose sensitivity sum_k |du/da_k| |a_k| exceeds kSensitive (BRT_FLAG_SENSITIVE).
constexpr double kPoleDist = 0.5;
constexpr double kSensitive = 100.0;
constexpr int kWindingSamples = 32;  // samples of the pole-test contour per lane (2048 per point)

__host__ __device__ __forceinline__ double coef_at(const double* a, int k) { return k >= 0 ? a[k] : 0.0; }

// Singular values of the n_vec x len matrix whose rows are stored in V (row i at V[i * len]), by one-sided
// Jacobi rotations of those rows (Hestenes): rotate pairs of rows until every pair is orthogonal; the row
// norms are then the singular values (n_vec <= len).  Squared row norms are kept and updated by the
// rotation identities (a' = a - t g, b' = b + t g), recomputed at the start of every sweep.  V is
// overwritten; sv[0..n_vec) comes out descending.
__host__ __device__ void jacobi_singular_values(double* V, int n_vec, int len, double* sv) {
  double nrm[kMaxPadeM + 1];
  for (int sweep = 0; sweep < 64; ++sweep) {
    for (int i = 0; i < n_vec; ++i) {
      double n2 = 0.0;
      for (int k = 0; k < len; ++k) n2 += V[i * len + k] * V[i * len + k];
      nrm[i] = n2;
    }
    bool rotated = false;
    for (int i = 0; i < n_vec - 1; ++i)
      for (int j = i + 1; j < n_vec; ++j) {
        double ga = 0.0;
        for (int k = 0; k < len; ++k) ga += V[i * len + k] * V[j * len + k];
        const double al = nrm[i], be = nrm[j];
        if (ga == 0.0 || ga * ga <= 1e-30 * (al * be)) continue;
        rotated = true;
        // tan of the rotation angle, the smaller root of t^2 + 2 zeta t - 1 = 0 with zeta = (be - al)/(2 ga)
        const double d = be - al;
        const double t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) / (fabs(d) + sqrt(d * d + 4.0 * ga * ga));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int k = 0; k < len; ++k) {
          const double x = V[i * len + k], y = V[j * len + k];
          V[i * len + k] = c * x - s * y;
          V[j * len + k] = s * x + c * y;
        }
        nrm[i] = al - t * ga;
        nrm[j] = be + t * ga;
      }
    if (!rotated) break;
  }
  for (int i = 0; i < n_vec; ++i) {
    double n2 = 0.0;
    for (int k = 0; k < len; ++k) n2 += V[i * len + k] * V[i * len + k];
    sv[i] = sqrt(n2);
  }
  for (int i = 1; i < n_vec; ++i)  // insertion sort, descending
    for (int j = i; j > 0 && sv[j] > sv[j - 1]; --j) {
      const double tmp = sv[j];
      sv[j] = sv[j - 1];
      sv[j - 1] = tmp;
    }
}

// LU factorisation with partial pivoting, in place (row-major M x M, multipliers below the diagonal),
// perm[i] = original row now at position i.  False on a zero or non-finite pivot.
__host__ __device__ bool lu_factor(double* T, int M, int* perm) {
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
    if (!(best == best) || best > 1.7e308 || best == 0.0) return false;
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
    const double inv = 1.0 / T[c * M + c];
    for (int r = c + 1; r < M; ++r) {
      const double l = T[r * M + c] * inv;
      T[r * M + c] = l;
      for (int j = c + 1; j < M; ++j) T[r * M + j] -= l * T[c * M + j];
    }
  }
  return true;
}

struct Order {
  int L, M;
  double margin;  // smallest distance (as a ratio) of a deciding singular value from the threshold
};

// Degrees used for a requested [L/M]: the rows of C (C[i][j] = a_{L+1+i-j}, i < M, j <= M) are the linear
// conditions C q = 0 on the denominator.  With s = ||a_0..a_{L+M}||_2 and rho the singular values of C above
// kPadeTol s: rho < M lowers both degrees by M - rho; a full-rank C whose square block C[:, 1:] has its
// smallest singular value at most kPadeTol s (no denominator with q_0 = 1) moves to [L+1/M-1].  The square
// block is looked at first (by a bound from its LU factors, then by its singular values): when its smallest
// singular value is above the threshold, so are all of C's, and C itself is not decomposed.  V holds
// (M+1)^2 doubles of scratch.
__host__ __device__ Order select_order(const double* a, int L, int M, double* V) {
  Order o{L, M, HUGE_VAL};
  double s2 = 0.0;
  for (int k = 0; k <= L + M; ++k) s2 += a[k] * a[k];
  const double s = sqrt(s2);
  if (!(s > 0.0) || !(s <= 1.7e308)) return Order{0, 0, HUGE_VAL};
  const double thr = kPadeTol * s;
  double sv[kMaxPadeM];
  auto note = [&](double v) {
    if (v > 0.0) {
      const double r = v > thr ? v / thr : thr / v;
      o.margin = r < o.margin ? r : o.margin;
    }
  };
  while (o.M > 0) {
    const int m = o.M, l = o.L;
    // Shortcut for the common case, equivalent to the singular-value rule below: the square block T = C[:, 1:]
    // has sigma_min(T) >= 1 / ||T^-1||_F, and every singular value of C is at least the matching one of T
    // (C C^T = c c^T + T T^T).  A bound well above the threshold settles it: full rank, denominator with
    // q_0 = 1, no change of degrees; the margin reported is then this lower bound.
    {
      int piv[kMaxPadeM];
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) V[i * m + j] = coef_at(a, l + i - j);
      if (lu_factor(V, m, piv)) {
        double fro2 = 0.0;
        for (int c = 0; c < m; ++c) {  // column c of T^-1: L y = P e_c, U x = y
          double x[kMaxPadeM];
          for (int i = 0; i < m; ++i) {
            double v = piv[i] == c ? 1.0 : 0.0;
            for (int j = 0; j < i; ++j) v -= V[i * m + j] * x[j];
            x[i] = v;
          }
          for (int i = m - 1; i >= 0; --i) {
            double v = x[i];
            for (int j = i + 1; j < m; ++j) v -= V[i * m + j] * x[j];
            x[i] = v / V[i * m + i];
            fro2 += x[i] * x[i];
          }
        }
        const double lb = 1.0 / sqrt(fro2);
        if (lb > 64.0 * thr && lb <= 1.7e308) {
          note(lb);
          break;
        }
      }
    }
    // the square block first: sigma_min(C[:, 1:]) above the threshold gives full rank of C as well
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) V[i * m + j] = coef_at(a, l + i - j);  // C[i][j + 1]
    double svT[kMaxPadeM];
    jacobi_singular_values(V, m, m, svT);
    note(svT[m - 1]);
    if (svT[m - 1] > thr) break;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j <= m; ++j) V[i * (m + 1) + j] = coef_at(a, l + 1 + i - j);
    jacobi_singular_values(V, m, m + 1, sv);
    int rho = 0;
    while (rho < m && sv[rho] > thr) ++rho;
    if (rho < m) {
      note(sv[rho]);
      if (rho > 0) note(sv[rho - 1]);
      o.L = l - (m - rho) > 0 ? l - (m - rho) : 0;
      o.M = rho;
      continue;
    }
    note(sv[m - 1]);
    // C has full rank but its square block does not: no denominator with q_0 = 1
    o.L = l + 1;
    o.M = m - 1;
  }
  return o;
}

struct PadeResult {
  double value;
  int L, M;       // degrees used
  double margin;  // of their selection
};

// [L/M] at z = 1 of sum_n a_n z^n with the degrees from select_order.  The denominator q (q_0 = 1) solves
// sum_{j=0}^{M} q_j a_{k-j} = 0 for k = L+1..L+M (a_i = 0 for i < 0); with partial sums
// A_m = a_0 + ... + a_m the value is sum_j q_j A_{L-j} / sum_j q_j.  On return T holds the LU factors
// (M x M), perm the pivoting and q the denominator (for pade_gradient).
__host__ __device__ PadeResult pade(const double* a, int L, int M, double* q, double* T, int* perm, double* V) {
  const Order o = select_order(a, L, M, V);
  PadeResult r{0.0, o.L, o.M, o.margin};
  while (true) {
    q[0] = 1.0;
    const int m = r.M, l = r.L;
    if (m == 0) break;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) T[i * m + j] = coef_at(a, l + i - j);  // T_{ij} = a_{L+i-j}, i, j = 1..M
    if (lu_factor(T, m, perm)) {
      double y[kMaxPadeM];
      for (int i = 0; i < m; ++i) {  // forward: L y = P (-b)
        double s = -a[l + 1 + perm[i]];
        for (int j = 0; j < i; ++j) s -= T[i * m + j] * y[j];
        y[i] = s;
      }
      for (int i = m - 1; i >= 0; --i) {  // backward: U q = y
        double s = y[i];
        for (int j = i + 1; j < m; ++j) s -= T[i * m + j] * q[j + 1];
        q[i + 1] = s / T[i * m + i];
      }
      break;
    }
    r.L = l + 1;  // an exactly singular square system (the rank test keeps these out): next antidiagonal entry
    r.M = m - 1;
  }
  double num = 0.0, den = 0.0;
  for (int j = 0; j <= r.M; ++j) {
    double A = 0.0;
    for (int i = 0; i <= r.L - j; ++i) A += a[i];
    num += q[j] * A;
    den += q[j];
  }
  r.value = num / den;
  return r;
}

// Gradient g_k = d value / d a_k (k = 0..L+M) of the approximant returned by pade().  With
// D = sum_j q_j and c_j = (A_{L-j} - value)/D, solve T^T y = c; then
//   g_k = [k <= L] sum_{j=0}^{min(M, L-k)} q_j / D  -  sum_{i=1}^{M} y_i q_{L+i-k}  (0 <= L+i-k <= M).
__host__ __device__ void pade_gradient(const double* a, const PadeResult& r, const double* q, const double* T,
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

// Point k (0 <= k < n) of the boundary of {z : dist(z, [0, 1]) <= kPoleDist}, counter-clockwise at equal
// arc length: the lower side, the right half circle around 1, the upper side, the left half circle around 0.
// The half circles use single-precision sin/cos: the samples only have to lie on the contour to ~1e-7.
__host__ __device__ void stadium_point(int k, int n, double* re, double* im) {
  const double r = kPoleDist, pi = 3.141592653589793;
  const double per = 2.0 + 2.0 * pi * r;
  double s = per * (double)k / (double)n;
  if (s < 1.0) {
    *re = s;
    *im = -r;
    return;
  }
  s -= 1.0;
  if (s < pi * r) {
    const float ph = (float)(-0.5 * pi + s / r);
    *re = 1.0 + r * (double)cosf(ph);
    *im = r * (double)sinf(ph);
    return;
  }
  s -= pi * r;
  if (s < 1.0) {
    *re = 1.0 - s;
    *im = r;
    return;
  }
  s -= 1.0;
  const float ph = (float)(0.5 * pi + s / r);
  *re = r * (double)cosf(ph);
  *im = r * (double)sinf(ph);
}

// Q(z) = sum_{j<=M} q_j z^j at a complex z (Horner).
__host__ __device__ void q_eval(const double* q, int M, double zr, double zi, double* vr, double* vi) {
  double ar = q[M], ai = 0.0;
  for (int j = M - 1; j >= 0; --j) {
    const double nr = ar * zr - ai * zi + q[j];
    ai = ar * zi + ai * zr;
    ar = nr;
  }
  *vr = ar;
  *vi = ai;
}

// Phase of w1 / w0 (w0, w1 != 0) in (-pi, pi], in single precision after scaling the product w1 conj(w0):
// the winding count only needs each step to an accuracy far below pi.
__host__ __device__ __forceinline__ float phase_step(double r0, double i0, double r1, double i1) {
  const double re = r1 * r0 + i1 * i0, im = i1 * r0 - r1 * i0;
  const double m = fmax(fabs(re), fabs(im));
  if (!(m > 0.0)) return 0.0f;
  return atan2f((float)(im / m), (float)(re / m));
}

// Per-lane scratch of the three Pade evaluations of a point (the value, [L-1/M] and [L/M-1]).
struct PadeScratch {
  double q[kMaxPadeM + 1];
  double T[kMaxPadeM * kMaxPadeM];
  double V[(kMaxPadeM + 1) * (kMaxPadeM + 1)];
  int perm[kMaxPadeM];
};

__global__ __launch_bounds__(64) void finalize_kernel(FinalizeArgs a) {
  __shared__ double coef[kMaxBins];
  __shared__ double m1[kMaxBins];
  __shared__ double m2[kMaxBins];
  __shared__ double grad[kMaxBins];
  __shared__ PadeScratch ps[3];
  __shared__ double res[3];             // values of lanes 0..2
  __shared__ int m_used;
  __shared__ unsigned long long extra[3];
  __shared__ unsigned long long wacc[kAccWords * kWave];  // digit words, one column per lane

  const uint32_t p = blockIdx.x;
  const uint32_t lane = threadIdx.x;
  const PointRec& pr = a.points[p];
  const uint32_t row = pr.out_row;  // output row of this point
  const uint32_t B = a.n_bins;
  const uint32_t NB = B + 3;
  const double N = (double)pr.n_total;
  const double scale = exp(pr.mu * pr.t);

  // Counts and flag counts: integer sums over the point's segments.
  for (uint32_t b = lane; b < NB; b += kWave) {
    unsigned long long cnt = 0;
    for (uint32_t s = 0; s < pr.seg_count; ++s) cnt += a.partials[(size_t)(pr.seg_begin + s) * NB + b].count;
    if (a.hist) a.hist[(size_t)row * NB + b] = cnt;
    if (b >= B) extra[b - B] = cnt;
  }
  // The sums: lane j takes the pair (bin j/2, sum j%2) and adds every segment's value exactly into its own
  // column of digit words, then rounds the total once.  Non-finite segment sums are classified instead.
  for (uint32_t j0 = 0; j0 < 2 * B; j0 += kWave) {
    const uint32_t j = j0 + lane;
    unsigned long long* w = wacc + lane;
    for (int k = 0; k < kAccWords; ++k) w[k * kWave] = 0ull;
    unsigned long long special = 0;
    if (j < 2 * B) {
      const uint32_t b = j >> 1;
      // a window of three words in registers at the last value's word index; a value on another word
      // first moves the window into the lane's LDS column (the segments of a point share a word almost
      // always, and each word takes at most 2^31 digits, far above a point's number of segments)
      uint32_t wk = 0xffffffffu;
      unsigned long long r0 = 0, r1 = 0, r2 = 0;
      for (uint32_t s = 0; s < pr.seg_count; ++s) {
        const Partial& pt = a.partials[(size_t)(pr.seg_begin + s) * NB + b];
        const double parts[2] = {(j & 1) ? pt.s2 : pt.s1_hi, (j & 1) ? 0.0 : pt.s1_lo};
        for (int q = 0; q < 2; ++q) {
          const double x = parts[q];
          if (x == 0.0) continue;
          if (!(fabs(x) <= 1.7976931348623157e308)) {
            special |= x != x ? 4ull : (x > 0 ? 1ull : 2ull);
            continue;
          }
          uint32_t k;
          unsigned long long d[3];
          digits_of(x, &k, d);
          if (k != wk) {
            if (wk != 0xffffffffu) {
              w[(size_t)wk * kWave] += r0;
              w[(size_t)(wk + 1) * kWave] += r1;
              w[(size_t)(wk + 2) * kWave] += r2;
            }
            wk = k;
            r0 = r1 = r2 = 0;
          }
          r0 += d[0];
          r1 += d[1];
          r2 += d[2];
        }
      }
      if (wk != 0xffffffffu) {
        w[(size_t)wk * kWave] += r0;
        w[(size_t)(wk + 1) * kWave] += r1;
        w[(size_t)(wk + 2) * kWave] += r2;
      }
      const double v = acc_round(w, kWave, special);
      const double mm = N > 0 ? v / N : 0.0;
      if (j & 1) {
        m2[b] = mm;
        if (a.s2) a.s2[(size_t)row * B + b] = v;
      } else {
        m1[b] = mm;
        coef[b] = scale * mm;
        if (a.s1) a.s1[(size_t)row * B + b] = v;
        if (a.coef) a.coef[(size_t)row * B + b] = scale * mm;
      }
    }
  }
  __syncthreads();
  for (uint32_t b = lane; b < B; b += kWave) {
    const double var = N > 1 ? scale * scale * (m2[b] - m1[b] * m1[b]) / (N - 1.0) : 0.0;
    if (a.coef_var) a.coef_var[(size_t)row * B + b] = var;
  }
  unsigned long long nodes = 0;
  for (uint32_t s = lane; s < pr.seg_count; s += kWave) nodes += a.seg_nodes[pr.seg_begin + s];
  nodes = wave_sum_u64(nodes);

  // Lanes 0, 1, 2 evaluate [L/M], [L-1/M] and [L/M-1] side by side, each with its own degree selection.
  const int L = (int)a.pade_L, M = (int)a.pade_M;
  PadeResult r{};
  if (lane < 3) {
    const int Lk = lane == 1 ? L - 1 : L, Mk = lane == 2 ? M - 1 : M;
    PadeScratch& w = ps[lane];
    if (Lk >= 0 && Mk >= 0) {
      r = pade(coef, Lk, Mk, w.q, w.T, w.perm, w.V);
      res[lane] = r.value;
    } else {
      res[lane] = NAN;
    }
    if (lane == 0) m_used = r.M;
  }
  __syncthreads();
  // Pole test: the number of zeros of Q inside the contour around [0, 1] is the winding number of Q along
  // it (argument principle), summed from the phase steps between consecutive samples.
  const int mq = m_used;
  const double* qm = ps[0].q;
  float wind = 0.0f;
  bool on_contour = false;
  if (mq > 0) {
    const int n = kWave * kWindingSamples;
    double zr, zi, pr0, pi0;
    stadium_point((int)lane * kWindingSamples, n, &zr, &zi);
    q_eval(qm, mq, zr, zi, &pr0, &pi0);
    for (int k = 1; k <= kWindingSamples; ++k) {
      double pr1, pi1;
      stadium_point(((int)lane * kWindingSamples + k) % n, n, &zr, &zi);
      q_eval(qm, mq, zr, zi, &pr1, &pi1);
      on_contour |= (pr1 == 0.0 && pi1 == 0.0);
      wind += phase_step(pr0, pi0, pr1, pi1);
      pr0 = pr1;
      pi0 = pi1;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) wind += __shfl_xor(wind, off);
  on_contour = __ballot(on_contour) != 0;
  if (lane == 0) {
    uint32_t fl = 0;
    if (extra[0] > 0) fl |= BRT_FLAG_OVERFLOW;
    if (extra[1] > 0) fl |= BRT_FLAG_CAPPED;
    if (extra[2] > 0) fl |= BRT_FLAG_DEPTH;
    if (on_contour || wind > 3.14159265f) fl |= BRT_FLAG_POLE;  // winding number >= 1
    if (r.L != L || r.M != M) fl |= BRT_FLAG_LOWERED;
    double psum = 0.0;
    for (uint32_t b = 0; b < B; ++b) psum += coef[b];
    // delta method: Var(u) = sum_kl g_k g_l Cov(a_k, a_l) with
    // Cov(a_k, a_l) = scale^2 (delta_kl m2_k - m1_k m1_l) / (N - 1); sensitivity kappa = sum_k |g_k| |a_k|
    PadeScratch& w = ps[0];
    pade_gradient(coef, r, w.q, w.T, w.perm, grad);
    double gg = 0.0, gm = 0.0, kappa = 0.0;
    for (int k = 0; k <= r.L + r.M; ++k) {
      gg += grad[k] * grad[k] * m2[k];
      gm += grad[k] * m1[k];
      kappa += fabs(grad[k]) * fabs(coef[k]);
    }
    const double var = N > 1 ? scale * scale * (gg - gm * gm) / (N - 1.0) : 0.0;
    if (kappa > kSensitive) fl |= BRT_FLAG_SENSITIVE;
    if (a.u) a.u[row] = r.value;
    if (a.se) a.se[row] = sqrt(var > 0.0 ? var : 0.0);
    if (a.psum) a.psum[row] = psum;
    if (a.flags) a.flags[row] = fl;
    if (a.nodes) a.nodes[row] = nodes;
    if (a.pade_diag) {
      double* d = a.pade_diag + (size_t)row * BRT_PADE_DIAG;
      d[0] = (double)r.L;
      d[1] = (double)r.M;
      d[2] = res[1];
      d[3] = res[2];
      d[4] = kappa;
      d[5] = r.margin;
    }
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
