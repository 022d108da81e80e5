// Moment reduction and FP64 finalize of the random-tree Monte Carlo (gfx950).
//
//  reduce_kernel    one wave per segment of one point's trees (up to 2^16 of them): per-bin count, compensated
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
#include <cmath>

#include "brt_internal.h"

namespace brt {

constexpr int kRedGroup = 16;   // bins accumulated per pass over a segment (per-lane sums in LDS)
static_assert((kSegTrees + kWave - 1) / kWave <= 65535 && (kPlanSegMax + kWave - 1) / kWave <= 65535,
              "per-lane counts are 16-bit");
constexpr int kRedBatch = 16;   // records loaded per lane per batch (two batches in flight)
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

// The digit words of one sum (kAccWords signed words w[0..kAccWords), word k weighing 2^(32k - 1074)) rounded
// once to the nearest double, ties to even; special = the non-finite values seen (bit 0 +inf, bit 1 -inf,
// bit 2 NaN).  Only the span of nonzero words and the two words above it take part (a word holds a sum of
// fewer than 2^31 digits, so its carry dies out within two words); the span is overwritten by the 32-bit
// digits of the magnitude.
__host__ __device__ double acc_round(unsigned long long* w, unsigned long long special) {
  if (special & 4ull) return NAN;
  if ((special & 3ull) == 3ull) return NAN;
  if (special & 1ull) return INFINITY;
  if (special & 2ull) return -INFINITY;
  int lo = -1, hi = -1;
  for (int k = 0; k < kAccWords; ++k)
    if (w[k] != 0ull) {
      hi = k;
      if (lo < 0) lo = k;
    }
  if (lo < 0) return 0.0;
  const int top = hi + 2 < kAccWords ? hi + 2 : kAccWords - 1;
  // carry-propagate into 32-bit digits; the final carry is the sign (0 or -1)
  long long carry = 0;
  for (int k = lo; k <= top; ++k) {
    const long long t = (long long)w[k] + carry;
    w[k] = (unsigned long long)t & 0xffffffffull;
    carry = t >> 32;
  }
  const bool neg = carry < 0;
  if (neg) {  // magnitude of the two's complement number (the zero digits below lo pass a carry of 1 up)
    unsigned long long c = 1;
    for (int k = lo; k <= top; ++k) {
      const unsigned long long t = (unsigned long long)(uint32_t)~(uint32_t)w[k] + c;
      w[k] = t & 0xffffffffull;
      c = t >> 32;
    }
  }
  int K = top;
  while (K >= lo && w[K] == 0ull) --K;
  if (K < lo) return 0.0;
  // the 64 bits from the leading one down (left-aligned), and whether anything nonzero lies below them
  const uint32_t dK = (uint32_t)w[K];
  int nb = 32;
  while (!((dK >> (nb - 1)) & 1u)) --nb;  // bit length of the leading digit
  const long long msb = 32ll * K + nb - 1;  // position of the leading one (bit 0 weighs 2^-1074)
  // digits K, K-1, K-2 as a 96-bit window [d2 d1 d0], shifted so that the leading one is bit 63 of top
  const unsigned long long d2 = dK, d1 = K >= 1 ? (uint32_t)w[K - 1] : 0u, d0 = K >= 2 ? (uint32_t)w[K - 2] : 0u;
  const unsigned long long hi64 = (d2 << 32) | d1;  // bits 32K + 31 .. 32K - 32
  const int sh = 32 - nb;                           // left shift that puts the leading one at bit 63
  const unsigned long long topb = sh ? (hi64 << sh) | (d0 >> (32 - sh)) : hi64;
  bool sticky = sh ? ((d0 & ((1ull << (32 - sh)) - 1)) != 0) : (d0 != 0);
  for (int k = lo; k < K - 2 && !sticky; ++k) sticky = w[k] != 0ull;
  double r;
  if (msb <= 52) {
    // at most 53 significant bits with lowest weight 2^-1074: exactly representable
    r = ldexp((double)(topb >> (63 - msb)), -1074);
  } else {
    unsigned long long mant = topb >> 11;          // 53 bits
    const unsigned long long rem = topb & 0x7ffull;
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
  __shared__ uint16_t lcnt[kRedGroup][kWave];  // a lane takes at most 65535 of a segment's trees

  const uint32_t seg = blockIdx.x;
  const uint32_t lane = threadIdx.x;
  const Segment sg = a.segs[seg];
  const PointRec& pr = a.points[sg.point];
  // the segment's records, indexed from its first tree (a segment holds at most 2^16 trees, so these
  // 32-bit indices cannot wrap even where the point's own tree indices approach 2^32)
  const double* F = a.tree_f + pr.tree_base + sg.begin;
  const uint32_t* M = a.tree_meta + pr.tree_base + sg.begin;
  const uint32_t n_seg = sg.end - sg.begin;
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
    // records are loaded kRedBatch at a time, and the next batch is requested before the current one
    // is added (two batches in registers), so the loads' latency overlaps the accumulation; each lane
    // still adds its records in increasing index order
    uint32_t mb[kRedBatch], mn[kRedBatch];
    double fb[kRedBatch], fn[kRedBatch];
    auto load_batch = [&](uint32_t i0, uint32_t* m, double* f) {
#pragma unroll
      for (int j = 0; j < kRedBatch; ++j) {
        const uint32_t i = i0 + j * kWave;
        m[j] = i < n_seg ? M[i] : kAbsent;
        f[j] = i < n_seg ? F[i] : 0.0;
      }
    };
    load_batch(lane, mb, fb);
    // complete the first batch here: the loop then waits for its prefetch only where it copies it
#pragma unroll
    for (int j = 0; j < kRedBatch; ++j) asm volatile("" ::"v"(mb[j]), "v"(fb[j]));
    for (uint32_t i0 = lane; i0 < n_seg; i0 += kWave * kRedBatch) {
      load_batch(i0 + kWave * kRedBatch, mn, fn);
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
#pragma unroll
      for (int j = 0; j < kRedBatch; ++j) {
        mb[j] = mn[j];
        fb[j] = fn[j];
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
// Degree selection of the approximant: a singular value of the denominator's linear conditions counts as
// zero when it is at most kPadeTol times the 2-norm of the coefficients a_0..a_{L+M}.
constexpr double kPadeTol = 1e-12;
// A zero of the denominator within kPoleDist of the segment [0, 1] is reported (BRT_FLAG_POLE), and a value
// whose sensitivity sum_k |du/da_k| |a_k| exceeds kSensitive (BRT_FLAG_SENSITIVE).
constexpr double kPoleDist = 0.5;
constexpr double kSensitive = 100.0;
constexpr int kWindingSamples = 32;  // samples of the pole-test contour per lane (2048 per point)
constexpr int kJoinGroup = 16;       // bins joined per pass of the finalize (its LDS columns bound the blocks per CU)
constexpr int kJoinBatch = 16;       // a segment's bins loaded per batch
static_assert(2 * kJoinGroup <= kWave, "one lane rounds each column of a pass");
constexpr int kAccStride = kAccWords + 1;  // LDS column of one exact sum (padded against bank conflicts)

__host__ __device__ __forceinline__ double coef_at(const double* a, int k) { return k >= 0 ? a[k] : 0.0; }

struct Order {
  int L, M;
  double margin;  // smallest distance (as a ratio) of a deciding singular value from the threshold
};

struct PadeResult {
  double value;
  int L, M;       // degrees used
  double margin;  // of their selection
};

// The small dense linear algebra of the Pade step for denominators of degree M <= MM.  Every array has a
// compile-time size and every loop runs to MM with the runtime size as a guard, so that after unrolling
// all indices are constants and the arrays live in registers (the coefficients a_n are read from LDS).
template <int MM>
struct SmallPade {
  // Singular values of the nv x len matrix with rows V[0..nv) (nv <= len <= MM + 1), by one-sided Jacobi
  // rotations of those rows (Hestenes): rotate pairs of rows, in cyclic order, until every pair is
  // orthogonal; the row norms are then the singular values.  Squared row norms are kept and updated by
  // the rotation identities (a' = a - t g, b' = b + t g), recomputed at the start of every sweep.  V is
  // overwritten; sv[0..nv) comes out descending.
  __host__ __device__ static void singular_values(double (&V)[MM][MM + 1], int nv, int len, double (&sv)[MM]) {
    double nrm[MM];
    for (int sweep = 0; sweep < 64; ++sweep) {
#pragma unroll
      for (int i = 0; i < MM; ++i) {
        double n2 = 0.0;
#pragma unroll
        for (int k = 0; k <= MM; ++k)
          if (k < len) n2 += V[i][k] * V[i][k];
        nrm[i] = n2;
      }
      bool rotated = false;
#pragma unroll
      for (int i = 0; i < MM - 1; ++i) {
#pragma unroll
        for (int j = i + 1; j < MM; ++j) {
          if (j >= nv) continue;
          double ga = 0.0;
#pragma unroll
          for (int k = 0; k <= MM; ++k)
            if (k < len) ga += V[i][k] * V[j][k];
          const double al = nrm[i], be = nrm[j];
          if (ga == 0.0 || ga * ga <= 1e-30 * (al * be)) continue;
          rotated = true;
          // tan of the rotation angle, the smaller root of t^2 + 2 zeta t - 1 = 0 with zeta = (be - al)/(2 ga)
          const double d = be - al;
          const double t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) / (fabs(d) + sqrt(d * d + 4.0 * ga * ga));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll
          for (int k = 0; k <= MM; ++k) {
            if (k >= len) continue;
            const double x = V[i][k], y = V[j][k];
            V[i][k] = c * x - s * y;
            V[j][k] = s * x + c * y;
          }
          nrm[i] = al - t * ga;
          nrm[j] = be + t * ga;
        }
      }
      if (!rotated) break;
    }
#pragma unroll
    for (int i = 0; i < MM; ++i) {
      double n2 = 0.0;
#pragma unroll
      for (int k = 0; k <= MM; ++k)
        if (k < len) n2 += V[i][k] * V[i][k];
      sv[i] = i < nv ? sqrt(n2) : 0.0;
    }
    // descending order (the unused entries are zeros and stay behind the used ones)
#pragma unroll
    for (int pass = 0; pass < MM - 1; ++pass)
#pragma unroll
      for (int i = 0; i < MM - 1 - pass; ++i)
        if (sv[i + 1] > sv[i]) {
          const double tmp = sv[i];
          sv[i] = sv[i + 1];
          sv[i + 1] = tmp;
        }
  }

  // LU factorisation with partial pivoting of the m x m block T, in place (multipliers below the
  // diagonal); perm[i] = original row now at position i.  False on a zero or non-finite pivot.
  __host__ __device__ static bool lu(double (&T)[MM][MM], int m, int (&perm)[MM]) {
#pragma unroll
    for (int i = 0; i < MM; ++i) perm[i] = i;
#pragma unroll
    for (int c = 0; c < MM; ++c) {
      if (c >= m) break;
      int piv = c;
      double best = fabs(T[c][c]);
#pragma unroll
      for (int r = c + 1; r < MM; ++r) {
        if (r >= m) continue;
        const double v = fabs(T[r][c]);
        if (v > best || !(v == v)) {
          best = v;
          piv = r;
        }
      }
      if (!(best == best) || best > 1.7e308 || best == 0.0) return false;
#pragma unroll
      for (int r = c + 1; r < MM; ++r) {
        if (r != piv) continue;
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          const double tmp = T[c][j];
          T[c][j] = T[r][j];
          T[r][j] = tmp;
        }
        const int tp = perm[c];
        perm[c] = perm[r];
        perm[r] = tp;
      }
      const double inv = 1.0 / T[c][c];
#pragma unroll
      for (int r = c + 1; r < MM; ++r) {
        if (r >= m) continue;
        const double l = T[r][c] * inv;
        T[r][c] = l;
#pragma unroll
        for (int j = c + 1; j < MM; ++j)
          if (j < m) T[r][j] -= l * T[c][j];
      }
    }
    return true;
  }

  // T_{ij} = a_{l+i-j}, i, j < m: the square block of the denominator's conditions.
  __host__ __device__ static void toeplitz(const double* a, int l, int m, double (&T)[MM][MM]) {
#pragma unroll
    for (int i = 0; i < MM; ++i)
#pragma unroll
      for (int j = 0; j < MM; ++j) T[i][j] = (i < m && j < m) ? coef_at(a, l + i - j) : 0.0;
  }

  // Degrees used for a requested [L/M]: the rows of C (C[i][j] = a_{L+1+i-j}, i < M, j <= M) are the linear
  // conditions C q = 0 on the denominator.  With s = ||a_0..a_{L+M}||_2 and rho the singular values of C
  // above kPadeTol s: rho < M lowers both degrees by M - rho; a full-rank C whose square block C[:, 1:] has
  // its smallest singular value at most kPadeTol s (no denominator with q_0 = 1) moves to [L+1/M-1].  The
  // square block is looked at first (by a bound from its LU factors, then by its singular values): when its
  // smallest singular value is above the threshold, so are all of C's, and C itself is not decomposed.
  __host__ __device__ static Order select_order(const double* a, int L, int M) {
    Order o{L, M, HUGE_VAL};
    double s2 = 0.0;
    for (int k = 0; k <= L + M; ++k) s2 += a[k] * a[k];
    const double s = sqrt(s2);
    if (!(s > 0.0) || !(s <= 1.7e308)) return Order{0, 0, HUGE_VAL};
    const double thr = kPadeTol * s;
    auto note = [&](double v) {
      if (v > 0.0) {
        const double r = v > thr ? v / thr : thr / v;
        o.margin = r < o.margin ? r : o.margin;
      }
    };
    while (o.M > 0) {
      const int m = o.M, l = o.L;
      // Shortcut for the common case, equivalent to the singular-value rule below: the square block
      // T = C[:, 1:] has sigma_min(T) >= 1 / ||T^-1||_F, and every singular value of C is at least the
      // matching one of T (C C^T = c c^T + T T^T).  A bound well above the threshold settles it: full rank,
      // denominator with q_0 = 1, no change of degrees; the margin reported is then this lower bound.
      {
        double T[MM][MM];
        int piv[MM];
        toeplitz(a, l, m, T);
        if (lu(T, m, piv)) {
          double fro2 = 0.0;
#pragma unroll
          for (int c = 0; c < MM; ++c) {  // column c of T^-1: L y = P e_c, U x = y
            if (c >= m) continue;
            double x[MM];
#pragma unroll
            for (int i = 0; i < MM; ++i) {
              double v = piv[i] == c ? 1.0 : 0.0;
#pragma unroll
              for (int j = 0; j < i; ++j) v -= T[i][j] * x[j];
              x[i] = v;
            }
#pragma unroll
            for (int i = MM - 1; i >= 0; --i) {
              if (i >= m) continue;
              double v = x[i];
#pragma unroll
              for (int j = i + 1; j < MM; ++j)
                if (j < m) v -= T[i][j] * x[j];
              x[i] = v / T[i][i];
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
      double V[MM][MM + 1];
      double sv[MM];
      // the square block first: sigma_min(C[:, 1:]) above the threshold gives full rank of C as well
#pragma unroll
      for (int i = 0; i < MM; ++i)
#pragma unroll
        for (int j = 0; j <= MM; ++j) V[i][j] = (i < m && j < m) ? coef_at(a, l + i - j) : 0.0;  // C[i][j + 1]
      singular_values(V, m, m, sv);
      double last = 0.0;
#pragma unroll
      for (int i = 0; i < MM; ++i)
        if (i == m - 1) last = sv[i];
      note(last);
      if (last > thr) break;
#pragma unroll
      for (int i = 0; i < MM; ++i)
#pragma unroll
        for (int j = 0; j <= MM; ++j) V[i][j] = (i < m && j <= m) ? coef_at(a, l + 1 + i - j) : 0.0;
      singular_values(V, m, m + 1, sv);
      int rho = 0;
#pragma unroll
      for (int i = 0; i < MM; ++i)
        if (i < m && rho == i && sv[i] > thr) rho = i + 1;
      if (rho < m) {
        double at = 0.0, below = 0.0;
#pragma unroll
        for (int i = 0; i < MM; ++i) {
          if (i == rho) at = sv[i];
          if (i == rho - 1) below = sv[i];
        }
        note(at);
        if (rho > 0) note(below);
        o.L = l - (m - rho) > 0 ? l - (m - rho) : 0;
        o.M = rho;
        continue;
      }
      double lastc = 0.0;
#pragma unroll
      for (int i = 0; i < MM; ++i)
        if (i == m - 1) lastc = sv[i];
      note(lastc);
      // C has full rank but its square block does not: no denominator with q_0 = 1
      o.L = l + 1;
      o.M = m - 1;
    }
    return o;
  }

  // [L/M] at z = 1 of sum_n a_n z^n with the degrees from select_order.  The denominator q (q_0 = 1) solves
  // sum_{j=0}^{M} q_j a_{k-j} = 0 for k = L+1..L+M (a_i = 0 for i < 0); with partial sums
  // A_m = a_0 + ... + a_m the value is sum_j q_j A_{L-j} / sum_j q_j.  On return T holds the LU factors,
  // perm the pivoting and q the denominator (for gradient), q_j = 0 for j > M.
  __host__ __device__ static PadeResult pade(const double* a, int L, int M, double (&q)[MM + 1],
                                             double (&T)[MM][MM], int (&perm)[MM]) {
    const Order o = select_order(a, L, M);
    PadeResult r{0.0, o.L, o.M, o.margin};
#pragma unroll
    for (int j = 0; j <= MM; ++j) q[j] = j == 0 ? 1.0 : 0.0;
    while (r.M > 0) {
      const int m = r.M, l = r.L;
      toeplitz(a, l, m, T);
      if (lu(T, m, perm)) {
        double y[MM];
#pragma unroll
        for (int i = 0; i < MM; ++i) {  // forward: L y = P (-b)
          if (i >= m) continue;
          double v = -a[l + 1 + perm[i]];
#pragma unroll
          for (int j = 0; j < i; ++j) v -= T[i][j] * y[j];
          y[i] = v;
        }
#pragma unroll
        for (int i = MM - 1; i >= 0; --i) {  // backward: U q = y
          if (i >= m) continue;
          double v = y[i];
#pragma unroll
          for (int j = i + 1; j < MM; ++j)
            if (j < m) v -= T[i][j] * q[j + 1];
          q[i + 1] = v / T[i][i];
        }
        break;
      }
      r.L = l + 1;  // an exactly singular square system (the rank test keeps these out): next antidiagonal entry
      r.M = m - 1;
    }
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int j = 0; j <= MM; ++j) {
      if (j > r.M) continue;
      double A = 0.0;
      for (int i = 0; i <= r.L - j; ++i) A += a[i];
      num += q[j] * A;
      den += q[j];
    }
    r.value = num / den;
    return r;
  }

  // Gradient g_k = d value / d a_k (k = 0..L+M) of the approximant returned by pade(); qs is q in LDS (for
  // the index L + i - k).  With D = sum_j q_j and c_j = (A_{L-j} - value)/D, solve T^T y = c; then
  //   g_k = [k <= L] sum_{j=0}^{min(M, L-k)} q_j / D  -  sum_{i=1}^{M} y_i q_{L+i-k}  (0 <= L+i-k <= M).
  __host__ __device__ static void gradient(const double* a, const PadeResult& r, const double (&q)[MM + 1],
                                           const double* qs, const double (&T)[MM][MM], const int (&perm)[MM],
                                           double* g) {
    const int L = r.L, M = r.M;
    double D = 0.0;
#pragma unroll
    for (int j = 0; j <= MM; ++j)
      if (j <= M) D += q[j];
    double y[MM];
#pragma unroll
    for (int i = 0; i < MM; ++i) y[i] = 0.0;
    if (M > 0) {
      double v[MM];
#pragma unroll
      for (int i = 0; i < MM; ++i) {  // U^T v = c
        if (i >= M) continue;
        double A = 0.0;
        for (int m = 0; m <= L - (i + 1); ++m) A += a[m];
        double s = (A - r.value) / D;
#pragma unroll
        for (int j = 0; j < i; ++j) s -= T[j][i] * v[j];
        v[i] = s / T[i][i];
      }
      double w[MM];
#pragma unroll
      for (int i = MM - 1; i >= 0; --i) {  // L^T w = v
        if (i >= M) continue;
        double s = v[i];
#pragma unroll
        for (int j = i + 1; j < MM; ++j)
          if (j < M) s -= T[j][i] * w[j];
        w[i] = s;
      }
#pragma unroll
      for (int i = 0; i < MM; ++i) {  // P y = w
        if (i >= M) continue;
#pragma unroll
        for (int k = 0; k < MM; ++k)
          if (perm[i] == k) y[k] = w[i];
      }
    }
    for (int k = 0; k <= L + M; ++k) {
      double gk = 0.0;
      if (k <= L) {
        const int jm = (L - k) < M ? (L - k) : M;
#pragma unroll
        for (int j = 0; j <= MM; ++j)
          if (j <= jm) gk += q[j];
        gk /= D;
      }
#pragma unroll
      for (int i = 1; i <= MM; ++i) {
        if (i > M) continue;
        const int j = L + i - k;
        if (j >= 0 && j <= M) gk -= y[i - 1] * qs[j];
      }
      g[k] = gk;
    }
  }
};

// Samples of the pole test's contour, the boundary of {z : dist(z, [0, 1]) <= kPoleDist}, counter-clockwise
// at equal arc length: the lower side, the right half circle around 1, the upper side, the left half
// circle around 0.  The same for every point: computed once on the host and copied to each device.
constexpr int kContourSamples = kWave * kWindingSamples;
__device__ double2 g_contour[kContourSamples];

static void stadium_point(int k, double* re, double* im) {
  const double r = kPoleDist, pi = 3.141592653589793;
  double s = (2.0 + 2.0 * pi * r) * (double)k / (double)kContourSamples;
  if (s < 1.0) {
    *re = s;
    *im = -r;
    return;
  }
  s -= 1.0;
  if (s < pi * r) {
    *re = 1.0 + r * std::cos(-0.5 * pi + s / r);
    *im = r * std::sin(-0.5 * pi + s / r);
    return;
  }
  s -= pi * r;
  if (s < 1.0) {
    *re = 1.0 - s;
    *im = r;
    return;
  }
  s -= 1.0;
  *re = r * std::cos(0.5 * pi + s / r);
  *im = r * std::sin(0.5 * pi + s / r);
}

int contour_init_device(int device) {
  static bool done[64] = {};
  if (device < 0 || device >= 64) return set_error(BRT_E_DEVICE, "device %d: no contour slot", device);
  if (done[device]) return BRT_OK;
  double2 h[kContourSamples];
  for (int k = 0; k < kContourSamples; ++k) stadium_point(k, &h[k].x, &h[k].y);
  const hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_contour), h, sizeof(h));
  if (e != hipSuccess) return set_error(BRT_E_DEVICE, "contour table on device %d: %s", device, hipGetErrorString(e));
  done[device] = true;
  return BRT_OK;
}

// Phase of w1 / w0 (w0, w1 != 0) in (-pi, pi], in single precision after scaling the product w1 conj(w0) by
// a power of two: the winding count only needs each step to an accuracy far below pi.
__host__ __device__ __forceinline__ float phase_step(double r0, double i0, double r1, double i1) {
  const double re = r1 * r0 + i1 * i0, im = i1 * r0 - r1 * i0;
  const double m = fmax(fabs(re), fabs(im));
  if (!(m > 0.0) || !(m <= 1.7e308)) return 0.0f;
  int e;
  frexp(m, &e);
  const double sc = ldexp(1.0, -e);
  return atan2f((float)(im * sc), (float)(re * sc));
}

// Adds a finite or non-finite double exactly into an LDS column of digit words (atomically, so that any
// number of lanes may add into one column); non-finite values are recorded in *special instead.
__device__ __forceinline__ void lds_add_exact(unsigned long long* col, unsigned int* special, double x) {
  if (x == 0.0) return;
  if (!(fabs(x) <= 1.7976931348623157e308)) {
    atomicOr(special, x != x ? 4u : (x > 0 ? 1u : 2u));
    return;
  }
  uint32_t k;
  unsigned long long d[3];
  digits_of(x, &k, d);
  if (d[0]) atomicAdd(col + k, d[0]);
  if (d[1]) atomicAdd(col + k + 1, d[1]);
  if (d[2]) atomicAdd(col + k + 2, d[2]);
}

template <int MM>
__global__ __launch_bounds__(64) void finalize_kernel(FinalizeArgs a) {
  __shared__ double coef[kMaxBins];
  __shared__ double m1[kMaxBins];
  __shared__ double m2[kMaxBins];
  __shared__ double grad[kMaxBins];
  __shared__ double qs[MM + 1];         // lane 0's denominator, for the pole test and the gradient
  __shared__ double res[3];             // values of lanes 0..2
  __shared__ int m_used;
  __shared__ unsigned long long cnt[kJoinGroup + 3];
  __shared__ unsigned int special[2 * kJoinGroup];
  __shared__ unsigned long long wacc[2 * kJoinGroup * kAccStride];  // digit words of the sums being joined

  const uint32_t p = blockIdx.x;
  const uint32_t lane = threadIdx.x;
  const PointRec& pr = a.points[p];
  const uint32_t row = pr.out_row;  // output row of this point
  const uint32_t B = a.n_bins;
  const uint32_t NB = B + 3;
  const double N = (double)pr.n_total;
  const double scale = exp(pr.mu * pr.t);
  const Partial* parts = a.partials + (size_t)pr.seg_begin * NB;

  // The point's segments joined exactly, kJoinGroup bins at a time: lanes take segments, add each
  // segment's count and sums into shared columns of digit words (integer atomics: the result does not
  // depend on the order), and lane j then rounds the column of (bin j/2, sum j%2) once.
  unsigned long long extra[3] = {0, 0, 0};
  for (uint32_t g0 = 0; g0 < B; g0 += kJoinGroup) {
    const uint32_t nb = B - g0 < (uint32_t)kJoinGroup ? B - g0 : (uint32_t)kJoinGroup;
    for (uint32_t i = lane; i < 2 * nb * kAccStride; i += kWave) wacc[i] = 0ull;
    if (lane < kJoinGroup + 3) cnt[lane] = 0ull;
    if (lane < 2 * kJoinGroup) special[lane] = 0u;
    __syncthreads();
    for (uint32_t sg = lane; sg < pr.seg_count; sg += kWave) {
      const Partial* prow = parts + (size_t)sg * NB + g0;
      for (uint32_t b0 = 0; b0 < nb; b0 += kJoinBatch) {
        Partial v[kJoinBatch];
#pragma unroll
        for (int k = 0; k < kJoinBatch; ++k)
          v[k] = b0 + k < nb ? prow[b0 + k] : Partial{0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kJoinBatch; ++k) {
          const uint32_t b = b0 + k;
          if (b >= nb) continue;
          if (v[k].count) atomicAdd(&cnt[b], (unsigned long long)v[k].count);
          unsigned long long* c1 = wacc + (2 * b) * kAccStride;
          lds_add_exact(c1, &special[2 * b], v[k].s1_hi);
          lds_add_exact(c1, &special[2 * b], v[k].s1_lo);
          lds_add_exact(c1 + kAccStride, &special[2 * b + 1], v[k].s2);
        }
      }
      if (g0 == 0) {
        const Partial* ext = parts + (size_t)sg * NB + B;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const unsigned long long c = ext[e].count;
          if (c) atomicAdd(&cnt[kJoinGroup + e], c);
        }
      }
    }
    __syncthreads();
    if (lane < nb && a.hist) a.hist[(size_t)row * NB + g0 + lane] = cnt[lane];
    if (g0 == 0) {
#pragma unroll
      for (int e = 0; e < 3; ++e) extra[e] = cnt[kJoinGroup + e];
      if (lane < 3 && a.hist) a.hist[(size_t)row * NB + B + lane] = cnt[kJoinGroup + lane];
    }
    if (lane < 2 * nb) {
      const uint32_t b = g0 + (lane >> 1);
      const double v = acc_round(wacc + lane * kAccStride, special[lane]);
      const double mm = N > 0 ? v / N : 0.0;
      if (lane & 1) {
        m2[b] = mm;
        if (a.s2) a.s2[(size_t)row * B + b] = v;
      } else {
        m1[b] = mm;
        coef[b] = scale * mm;
        if (a.s1) a.s1[(size_t)row * B + b] = v;
        if (a.coef) a.coef[(size_t)row * B + b] = scale * mm;
      }
    }
    __syncthreads();
  }
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
  double q[MM + 1];
  double T[MM][MM];
  int perm[MM];
  if (lane < 3) {
    const int Lk = lane == 1 ? L - 1 : L, Mk = lane == 2 ? M - 1 : M;
    if (Lk >= 0 && Mk >= 0) {
      r = SmallPade<MM>::pade(coef, Lk, Mk, q, T, perm);
      res[lane] = r.value;
    } else {
      res[lane] = NAN;
    }
    if (lane == 0) {
      m_used = r.M;
#pragma unroll
      for (int j = 0; j <= MM; ++j) qs[j] = q[j];
    }
  }
  __syncthreads();
  // Pole test: the number of zeros of Q inside the contour around [0, 1] is the winding number of Q along
  // it (argument principle), summed from the phase steps between consecutive samples.
  const int mq = m_used;
  float wind = 0.0f;
  bool on_contour = false;
  if (mq > 0) {
    double qr[MM + 1];
#pragma unroll
    for (int j = 0; j <= MM; ++j) qr[j] = qs[j];
    auto q_at = [&](double zr, double zi, double* vr, double* vi) {  // Horner; q_j = 0 above the degree
      double ar = qr[MM], ai = 0.0;
#pragma unroll
      for (int j = MM - 1; j >= 0; --j) {
        const double nr = ar * zr - ai * zi + qr[j];
        ai = ar * zi + ai * zr;
        ar = nr;
      }
      *vr = ar;
      *vi = ai;
    };
    double pr0, pi0;
    const double2 z0 = g_contour[lane * kWindingSamples];
    q_at(z0.x, z0.y, &pr0, &pi0);
    for (int k = 1; k <= kWindingSamples; ++k) {
      double pr1, pi1;
      const double2 z = g_contour[(lane * kWindingSamples + k) % kContourSamples];
      q_at(z.x, z.y, &pr1, &pi1);
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
    SmallPade<MM>::gradient(coef, r, q, qs, T, perm, grad);
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
  if (a.pade_M <= 6)
    hipLaunchKernelGGL(finalize_kernel<6>, dim3(a.n_points), dim3(kWave), 0, s, a);
  else if (a.pade_M <= 8)
    hipLaunchKernelGGL(finalize_kernel<8>, dim3(a.n_points), dim3(kWave), 0, s, a);
  else
    hipLaunchKernelGGL(finalize_kernel<16>, dim3(a.n_points), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

}  // namespace brt
