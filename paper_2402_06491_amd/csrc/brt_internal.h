// Internal layouts shared by the HIP kernels and the host runtime of libbrt.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "brt.h"

namespace brt {

constexpr int kWave = 64;
constexpr int kMaxProblems = 64;
// How a walker launch holds its problems: one problem (constants in scalar registers), a table of
// several (each lane reads its problem's record), or a family of several that differ only in their
// initial data (shared constants in scalar registers, each lane reads its problem's initial data).
constexpr int kOneProblem = 0, kProblemTable = 1, kFamily = 2;
constexpr int kMaxU0Params = 32;
constexpr int kMaxWalkThreads = 256;  // walker block size limit (4 waves): lets FP64 walkers keep state in VGPRs

// tree_meta bit layout
constexpr uint32_t kMetaNeMask = 0xffu;
constexpr uint32_t kMetaOverflow = 1u << 8;
constexpr uint32_t kMetaCapped = 1u << 9;
constexpr uint32_t kMetaDepth = 1u << 10;
constexpr int kMetaNodesShift = 11;
constexpr uint32_t kMaxNodeCap = (1u << 21) - 1;  // nodes field is 21 bits
constexpr uint32_t kMaxEulerSteps = 1u << 20;     // Euler-Maruyama steps per edge at most

// Per-problem constants after the Strategy A normalisation, in the walker's precision.
template <typename Real>
struct PdeT {
  Real sigma;        // sqrt(2a)
  Real inv_lambda;   // Strategy A: 1/lambda (unused when K == 0)
  Real mu;           // Strategy A: c_1 + lambda; Strategy B: c_1
  Real inv_q;        // Strategy B: 1/q (leaf values are g/q)
  Real s_scale;      // Strategy B: 1/(2^32 - Q), maps a vertex's w0 to its split fraction
  uint32_t K;        // number of non-linear terms
  uint32_t jpack;    // their powers, 4 bits each, ascending
  uint32_t u0_nterms;
  uint32_t q_lo;     // Strategy B: Q - 1 with Q = floor(q 2^32); a node is a leaf iff w0 <= q_lo
  uint32_t cmod;     // 0: constant coefficients; 1: c_j exp(-bx x^2 - by y^2) (tau + t0)^(-cm_pow)
  uint32_t cm_pow;   // 0 or 1
  uint32_t drift_on; // 1: constant drift b, an edge of duration s moves by b s + sigma W_s
  Real cm_bx, cm_by, cm_t0;
  Real drift[2];
  uint32_t sde;      // 1: Euler-Maruyama steps for b(x) = drift + dlin x, sigma(x) = sigma (1 + sig_amp e^{-sig_k |x|^2})
  uint32_t pad3;
  Real dlin[2], sig_amp, sig_k, inv_h;
  Real omega[8];     // Strategy A: K c_j / lambda; Strategy B: K c_j / (1 - q)
  Real u0[kMaxU0Params];
};

// Per-point record (device).
struct PointRec {
  double x[2];
  double t;
  double theta;      // exp(-lambda t) from the host (1 when K == 0)
  double mu;         // for the finalize
  uint64_t tree_base;
  uint32_t n_trees;
  uint32_t point_id; // Philox counter word 2
  uint32_t pde;
  uint32_t seg_begin;  // first reduction partial of this point (finalize)
  uint32_t seg_count;  // number of partials of this point (finalize)
  uint32_t tree_first; // Philox tree counter of the point's first tree in this launch
  uint64_t n_total;    // trees behind the point's partials (the N of the sample mean)
  uint32_t out_row;    // row of the per-point outputs written by the finalize
  uint32_t pad;
};

// A walker work chunk: trees [begin, end) of one point.
struct Chunk {
  uint32_t point;
  uint32_t begin;
  uint32_t end;
  uint32_t pad;
};

// A reduction segment: trees [begin, end) of one point.
struct Segment {
  uint32_t point;
  uint32_t begin;
  uint32_t end;
  uint32_t out;  // index of the partial this segment writes
};

// Per (segment, bin) partial moments: the count, the compensated sum of F as an unevaluated pair
// s1_hi + s1_lo, and the sum of F*F (each F*F rounded to FP64).  The finalize joins a point's segments
// exactly (kAccWords digit words) and rounds once, so the result does not depend on the order of the
// segments.  Entries B, B+1, B+2 of a segment count trees pruned (overflow), capped and over the stack
// depth in `count`.
struct Partial {
  uint64_t count;
  double s1_hi;
  double s1_lo;
  double s2;
};
// Digit words of an exact sum: word k holds a signed sum of 32-bit digits weighing 2^(32k - 1074), which
// covers every finite double (k <= 65) with headroom for carries.
constexpr int kAccWords = 68;

struct WalkArgs {
  const PointRec* points;
  const Chunk* chunks;
  uint32_t n_chunks;
  uint32_t n_problems;
  const void* pdes;          // PdeT<Real>[n_problems]
  uint32_t* chunk_counter;   // reset before each launch
  unsigned long long* depth_counter;
  double* tree_f;
  uint32_t* tree_meta;
  void* spill;               // global stack levels beyond the LDS part: [spill_depth][entry fields][n_threads]
  uint32_t key0, key1;
  uint32_t max_order;
  uint32_t prune;
  uint32_t node_cap;
  uint32_t strategy;         // 0: Strategy A, 1: Strategy B
  uint32_t cmod;             // 1: some problem of the launch has variable coefficients or a drift
  uint32_t stack_depth;      // LDS levels per lane
  uint32_t spill_depth;      // global levels per lane
  uint32_t n_threads;        // grid size in threads (spill stride)
  uint32_t u0_stride;        // > 0: the n_problems > 1 problems form a family; initial-data parameters kept per problem
};

struct ReduceArgs {
  const PointRec* points;
  const Segment* segs;
  uint32_t n_segs;
  const double* tree_f;
  const uint32_t* tree_meta;
  Partial* partials;         // [n_segs][n_bins + 3]
  unsigned long long* seg_nodes;  // [n_segs]
  uint32_t n_bins;           // B = max_order + 2
};

struct FinalizeArgs {
  const PointRec* points;
  uint32_t n_points;
  const Partial* partials;
  const unsigned long long* seg_nodes;
  uint32_t n_bins;
  uint32_t pade_L, pade_M;
  double* u;
  double* se;
  double* psum;
  double* coef;
  double* coef_var;
  unsigned long long* hist;
  double* s1;
  double* s2;
  unsigned long long* nodes;
  uint32_t* flags;
  double* pade_diag;  // [n][BRT_PADE_DIAG] (nullable)
};

}  // namespace brt

// A context: one HIP device and its launch settings (brt_runtime.hip).
struct brt_ctx {
  int device = 0;
  int n_cu = 0;
  brt_launch launch{};
};

namespace brt {

// Look up the address of the allocation-free entry point's scratch array on `device` (current) once per
// device (brt_noalloc.hip); BRT_E_DEVICE if the lookup fails.
int noalloc_init_device(int device);
// Copy the pole test's contour samples to `device` (current) once (brt_moments.hip); BRT_E_DEVICE on failure.
int contour_init_device(int device);

// Strategy A normalisation of one problem (brt_runtime.hip).
struct Norm {
  double sigma = 0, lambda = 0, inv_lambda = 0, mu = 0;
  double q = 1.0;       // Strategy B: probability of a leaf (1 when K == 0)
  uint64_t Q = 0;       // Strategy B: floor(q 2^32)
  uint32_t K = 0;
  uint32_t J[8] = {0};
  double omega[8] = {0};
};
Norm normalize(const brt_problem& p, const brt_mc& mc);
// A problem the walker's general-coefficients variant takes: variable coefficients or a drift.
inline bool general_coefficients(const brt_problem& p) {
  return p.coef_mod != BRT_COEF_MOD_NONE || p.drift[0] != 0.0 || p.drift[1] != 0.0 || p.sde != BRT_SDE_EXACT;
}
size_t pde_bytes(int precision);
void pde_to_device(const brt_problem& p, const Norm& n, int precision, void* dst);
double est_nodes(const Norm& n, const brt_mc& mc, double t);
int set_error(int code, const char* fmt, ...);  // records the thread's error message, returns code
constexpr uint32_t kSegTrees = 1u << 13;          // trees per reduction segment of a serving round
constexpr uint32_t kPlanSegMin = 1u << 10, kPlanSegMax = 1u << 16;  // trees per reduction segment of a plan
// A plan's segment size: the power of two in [kPlanSegMin, kPlanSegMax] nearest above total / 4096, so
// that a large workload has few partials per point to join and a small one still spreads its
// reduction over many waves.
inline uint32_t plan_seg_trees(uint64_t total) {
  uint32_t s = kPlanSegMin;
  while (s < kPlanSegMax && (uint64_t)s * 4096u < total) s <<= 1;
  return s;
}
constexpr uint32_t kMaxDepthUnpruned = 64;        // stack levels per lane when trees are not pruned
constexpr uint32_t kDefaultLdsLevels = 8;         // stack levels per lane kept in LDS by default

// Launchers (brt_kernels.hip).
hipError_t launch_reset(uint32_t* chunk_counter, unsigned long long* depth_counter, hipStream_t s);
hipError_t launch_walk(int precision, int dim, int u0_kind, const WalkArgs& a, int grid, int waves_per_block,
                       hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
// Initial-data parameters a problem's leaves read (BRT_U0_* kind; nterms for Gaussian sums).
uint32_t u0_param_count(uint32_t u0_kind, uint32_t nterms);
// The initial-data stride of a launch of n problem records (device layout, back to back) if they form a
// family (equal but for their initial-data parameters and term counts), else 0.
uint32_t family_u0_stride(int precision, uint32_t u0_kind, const void* recs, size_t n);
// u0_stride > 0: a family launch (WalkArgs::u0_stride)
size_t walk_lds_bytes(int precision, int dim, int stack_depth, int waves_per_block, int n_problems, int strategy,
                      int u0_stride = 0);
size_t stack_entry_size(int precision, int dim);  // bytes of one spill level (full layout)
int walk_max_blocks_per_cu(int precision, int dim, int u0_kind, int n_problems, int stack_depth, int waves_per_block,
                           int strategy, int u0_stride = 0);

}  // namespace brt
