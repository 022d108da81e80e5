/*
 * ORACLE — test infrastructure, not product code.
 *
 * A plain, slow, FP64 CPU walker for the random-tree Monte Carlo of
 * Strategy A (Sec. 2.1 of Acebron & Rodriguez-Rozas, "A new parallel solver
 * suited for arbitrary semilinear parabolic PDEs based on generalized random
 * trees").  Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of
 * bench.py may load this library.  It shares no code with the HIP path; the
 * only thing both sides agree on is the published definition of
 * Philox4x32-10 and the documented assignment of its output words (below).
 *
 * What one tree computes (Strategy A with a clock of rate lambda):
 *   - the PDE  u_t = a*Lap(u) + sum_j c_j u^j  (problem statement, Sec. 1)
 *     is rewritten with u = v*exp(mu*t), mu = c_1 + lambda (the change of
 *     variables of Strategy A, generalised so that the linear coefficient is
 *     absorbed and the artificial potential has rate lambda; lambda = 1 and
 *     c_1 = 0 give the paper's u = v*e^t);
 *   - the Green's function is sampled with the SDE d(beta) = sigma dW,
 *     sigma = sqrt(2a) (Feynman-Kac form, eqs. green/SDE);
 *   - each node draws an Exp(lambda) time S; if S is shorter than the time
 *     left, the node is a vertex (a split), otherwise a leaf (eq. probexp1);
 *   - a vertex picks its arity alpha uniformly among the K non-zero
 *     non-linear terms and carries the weight K*c_alpha/lambda *
 *     exp((alpha-1)*mu*tau') where tau' is the PDE time left after the split
 *     (eq. probexp2 and the recursion, with c' = (m-1)c);
 *   - a leaf carries g evaluated where its path ends;
 *   - the tree's value is the product of all vertex weights and leaf values
 *     (the multiplicative functional of eq. rep_strategyB), and the tree is
 *     binned by its number of splits Ne (series coefficient index).
 *
 * Randomness (one Philox4x32-10 block per node):
 *   key     = (seed & 0xffffffff, seed >> 32)
 *   counter = (node preorder index, tree index, point id, 0)
 *   word 0  -> clock uniform U = (w0 + 0.5) 2^-32
 *   word 1  -> arity index floor(w1 * K / 2^32)
 *   words 2,3 -> Box-Muller: u1 = (w2 + 0.5) 2^-32, u2 = w3 2^-32,
 *                z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = sqrt(-2 ln u1) sin(2 pi u2)
 * The node is a vertex iff the product of the clock uniforms along its
 * lineage (itself included) is > theta = exp(-lambda t); this is the event
 * "sum of the exponential times < t" written with exact FP64 products.
 * Preorder: a vertex's children are visited in order 0..alpha-1, each
 * subtree completely before the next.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_FLAG_OVERFLOW 1u /* pruned: more than max_order splits */
#define OR_FLAG_CAPPED 2u   /* node cap reached */

#define OR_U0_CONST 0
#define OR_U0_LOGISTIC 1
#define OR_U0_GAUSS_SUM 2
#define OR_U0_COS2_BUMP 3

/* Mirror of the ctypes structure in oracle/__init__.py. */
typedef struct {
  int32_t dim;
  int32_t u0_kind;
  int32_t u0_nterms;
  int32_t K;          /* number of non-linear terms */
  int32_t J[8];       /* their powers, ascending */
  double omega[8];    /* K c_j / lambda for each entry of J */
  double sigma;       /* sqrt(2 a) */
  double lambda;      /* clock rate */
  double mu;          /* c_1 + lambda */
  double u0p[40];
  uint32_t key[2];
  int32_t max_order;
  int32_t prune;
  uint32_t node_cap;
  int32_t strategy;   /* 0: Strategy A (exponential clock), 1: Strategy B (coin + uniform time) */
  uint64_t Q;         /* Strategy B: a node is a leaf iff w0 < Q = floor(q 2^32) */
  double q;           /* Strategy B: probability of a leaf */
  int32_t cmod;       /* 1: c_j(x, t) = c_j exp(-bx x^2 - by y^2) (t + t0)^(-pow) */
  int32_t cmod_pow;
  double cmod_bx, cmod_by, cmod_t0;
  double drift[2];    /* constant drift b of L = a Lap + b.grad: an edge of duration s moves by b s + sigma W_s */
  int32_t sde;        /* 1: Euler-Maruyama edges for b(x) = drift + dlin x, sigma(x) = sigma (1 + sig_amp e^{-sig_k |x|^2}) */
  int32_t sde_pad;
  double dlin[2];
  double sig_amp, sig_k;
  double inv_h;       /* 1 / (largest Euler step) */
} or_problem;

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += 0x9E3779B9u; /* golden ratio */
      k1 += 0xBB67AE85u; /* sqrt(3) - 1 */
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ---- initial data g (the u(x,0) families used by the examples) ---------- */
static double or_g(const or_problem* pb, const double* x) {
  const double* p = pb->u0p;
  switch (pb->u0_kind) {
    case OR_U0_CONST:
      return p[0];
    case OR_U0_LOGISTIC: {
      /* A * (1 + exp(s * (n.x - x0)))^(-pow) */
      double nx = x[0] * p[4];
      if (pb->dim == 2) nx += x[1] * p[5];
      double e = exp(p[1] * (nx - p[2]));
      double base = 1.0 / (1.0 + e);
      double r = 1.0;
      int pw = (int)p[3];
      for (int i = 0; i < pw; i++) r *= base;
      return p[0] * r;
    }
    case OR_U0_GAUSS_SUM: {
      /* sum_k A_k exp(-|x - c_k|^2 / (2 s_k^2)), term k = (A, cx, cy, s) */
      double acc = 0.0;
      for (int k = 0; k < pb->u0_nterms; k++) {
        const double* q = p + 4 * k;
        double r2 = (x[0] - q[1]) * (x[0] - q[1]);
        if (pb->dim == 2) r2 += (x[1] - q[2]) * (x[1] - q[2]);
        acc += q[0] * exp(-r2 / (2.0 * q[3] * q[3]));
      }
      return acc;
    }
    case OR_U0_COS2_BUMP: {
      /* A cos^2(pi x / (2 Ax)) cos^2(pi y / (2 Ay)) inside the box, else 0 */
      if (fabs(x[0]) > p[1]) return 0.0;
      double cx = cos(M_PI * x[0] / (2.0 * p[1]));
      double v = p[0] * cx * cx;
      if (pb->dim == 2) {
        if (fabs(x[1]) > p[2]) return 0.0;
        double cy = cos(M_PI * x[1] / (2.0 * p[2]));
        v *= cy * cy;
      }
      return v;
    }
  }
  return NAN;
}

typedef struct {
  uint32_t node;   /* next preorder index */
  uint32_t ne;     /* splits so far */
  uint32_t flags;
  uint32_t tree;
  uint32_t pid;
  double theta;
} or_tree;

/* Factor by which a split at position x with PDE time tau left scales its constant coefficient
 * (variable coefficients c_j(x, t), evaluated where and when the tree splits). */
static double or_cmod(const or_problem* pb, const double* x, double tau) {
  if (!pb->cmod) return 1.0;
  double e = pb->cmod_bx * x[0] * x[0];
  if (pb->dim == 2) e += pb->cmod_by * x[1] * x[1];
  double v = exp(-e);
  if (pb->cmod_pow == 1) v /= tau + pb->cmod_t0;
  return v;
}

/* End of one edge of duration dt that starts at x, for the node with Philox counter node (z: the normals
 * of its own block).  Constant coefficients: one exact Gaussian increment, b dt + sigma sqrt(dt) z.  A
 * general L: n = ceil(dt / h) equal Euler-Maruyama steps (they end at the edge's end, the branching
 * time), y += b(y) dt/n + sigma(y) sqrt(dt/n) z_k, with z_0 = z and z_k from the block (node, tree,
 * point, k). */
static void or_move(const or_problem* pb, const or_tree* st, uint32_t node, const double* x, double dt,
                    const double* z, double* out) {
  if (!pb->sde) {
    for (int d = 0; d < pb->dim; d++) out[d] = x[d] + pb->drift[d] * dt + pb->sigma * sqrt(dt) * z[d];
    return;
  }
  const double nf = ceil(dt * pb->inv_h);
  const uint32_t n = nf < 1.0 ? 1u : nf > 1048576.0 ? 1048576u : (uint32_t)nf;  /* at most 2^20 steps */
  const double h = dt / (double)n, sh = sqrt(h);
  double y[2] = {x[0], pb->dim == 2 ? x[1] : 0.0};
  double zz[2] = {z[0], z[1]};
  for (uint32_t k = 0; k < n; k++) {
    if (k > 0) {
      uint32_t ctr[4] = {node, st->tree, st->pid, k};
      uint32_t w[4];
      or_philox4x32_10(ctr, pb->key, w);
      const double u1 = ((double)w[2] + 0.5) / 4294967296.0, u2 = (double)w[3] / 4294967296.0;
      const double r = sqrt(-2.0 * log(u1));
      zz[0] = r * cos(2.0 * M_PI * u2);
      zz[1] = r * sin(2.0 * M_PI * u2);
    }
    double r2 = y[0] * y[0];
    if (pb->dim == 2) r2 += y[1] * y[1];
    const double sg = pb->sigma * (1.0 + pb->sig_amp * exp(-pb->sig_k * r2));
    double inc[2];
    for (int d = 0; d < pb->dim; d++) inc[d] = (pb->drift[d] + pb->dlin[d] * y[d]) * h + sg * sh * zz[d];
    for (int d = 0; d < pb->dim; d++) y[d] += inc[d];
  }
  for (int d = 0; d < pb->dim; d++) out[d] = y[d];
}

/* Value of the subtree whose root starts at position x with lineage clock
 * product P and remaining PDE time tau. */
static double or_visit(const or_problem* pb, or_tree* st, const double* x, double P, double tau) {
  if (st->node >= pb->node_cap) {
    st->flags |= OR_FLAG_CAPPED;
    return 0.0;
  }
  const uint32_t node = st->node;
  uint32_t ctr[4] = {node, st->tree, st->pid, 0u};
  uint32_t w[4];
  or_philox4x32_10(ctr, pb->key, w);
  st->node += 1;

  const double two32 = 4294967296.0;
  double U = ((double)w[0] + 0.5) / two32;
  double Pn = P * U;
  double u1 = ((double)w[2] + 0.5) / two32;
  double u2 = (double)w[3] / two32;
  double r = sqrt(-2.0 * log(u1));
  double z[2] = {r * cos(2.0 * M_PI * u2), r * sin(2.0 * M_PI * u2)};

  if (Pn > st->theta) {
    /* vertex: the exponential time is shorter than the time left */
    double S = -log(U) / pb->lambda;
    double tau2 = tau - S;
    if (tau2 < 0.0) tau2 = 0.0;
    double xs[2];
    or_move(pb, st, node, x, S, z, xs);
    st->ne += 1;
    if (pb->prune && st->ne > (uint32_t)pb->max_order) {
      st->flags |= OR_FLAG_OVERFLOW;
      return 0.0;
    }
    uint32_t idx = (uint32_t)(((uint64_t)w[1] * (uint64_t)pb->K) >> 32);
    int alpha = pb->J[idx];
    double val = pb->omega[idx] * exp((double)(alpha - 1) * pb->mu * tau2) * or_cmod(pb, xs, tau2);
    for (int c = 0; c < alpha; c++) {
      double child = or_visit(pb, st, xs, Pn, tau2);
      if (st->flags) return 0.0;
      val *= child;
    }
    return val;
  }
  /* leaf: the path runs to the final time; evaluate g where it ends */
  double xl[2];
  or_move(pb, st, node, x, tau, z, xl);
  return or_g(pb, xl);
}

/* Strategy B (Sec. 2.2): the integral equation is sampled with a coin xi, P(leaf) = q.  A leaf
 * evaluates g where its path ends, divided by q.  A vertex splits after the uniform fraction S of the
 * time left tau (the path moves for tau S, its children have tau' = tau (1 - S) left) and carries
 * tau * K c_alpha / (1 - q) * e^{(alpha-1) mu tau'} (eta(t) = t, c~ = c/(1-q), c' = (m-1)c~, with the
 * linear coefficient absorbed as u = v e^{mu t}, mu = c_1).  Randomness: the coin is w0 < Q; for a
 * vertex S = (w0 - Q + 1/2) / (2^32 - Q) (w0 is uniform on [Q, 2^32) given the coin); w1 picks the
 * arity; w2, w3 the normals. */
static double or_visit_b(const or_problem* pb, or_tree* st, const double* x, double tau) {
  if (st->node >= pb->node_cap) {
    st->flags |= OR_FLAG_CAPPED;
    return 0.0;
  }
  const uint32_t node = st->node;
  uint32_t ctr[4] = {node, st->tree, st->pid, 0u};
  uint32_t w[4];
  or_philox4x32_10(ctr, pb->key, w);
  st->node += 1;

  const double two32 = 4294967296.0;
  double u1 = ((double)w[2] + 0.5) / two32;
  double u2 = (double)w[3] / two32;
  double r = sqrt(-2.0 * log(u1));
  double z[2] = {r * cos(2.0 * M_PI * u2), r * sin(2.0 * M_PI * u2)};

  if ((uint64_t)w[0] >= pb->Q) {
    /* vertex */
    /* split after the fraction V = (w0 - Q + 1/2)/(2^32 - Q) of tau; the time left after it,
       tau (1 - V), is formed from the complementary count 2^32 - w0 - 1/2 so that it carries no
       cancellation when V is close to 1 (the vertex weight is proportional to it) */
    const double span = two32 - (double)pb->Q;
    double s = tau * (((double)((uint64_t)w[0] - pb->Q) + 0.5) / span);
    double tau2 = tau * (((double)(0xFFFFFFFFu - w[0]) + 0.5) / span);
    double xs[2];
    or_move(pb, st, node, x, s, z, xs);
    st->ne += 1;
    if (pb->prune && st->ne > (uint32_t)pb->max_order) {
      st->flags |= OR_FLAG_OVERFLOW;
      return 0.0;
    }
    uint32_t idx = (uint32_t)(((uint64_t)w[1] * (uint64_t)pb->K) >> 32);
    int alpha = pb->J[idx];
    double val = tau * pb->omega[idx] * exp((double)(alpha - 1) * pb->mu * tau2) * or_cmod(pb, xs, tau2);
    for (int c = 0; c < alpha; c++) {
      double child = or_visit_b(pb, st, xs, tau2);
      if (st->flags) return 0.0;
      val *= child;
    }
    return val;
  }
  double xl[2];
  or_move(pb, st, node, x, tau, z, xl);
  return or_g(pb, xl) / pb->q;
}

/*
 * Walk n independent trees.  Item i is tree tree_idx[i] of the point with
 * position x[i*dim..], time t[i] and id point_id[i].  Outputs per item: the
 * tree value F (0 when abandoned), its number of splits, its number of nodes
 * and its flags.  theta_out (nullable) receives exp(-lambda t) per item.
 * Returns 0.
 */
int or_walk(const or_problem* pb, int64_t n, const double* x, const double* t,
            const uint32_t* point_id, const uint32_t* tree_idx, double* F,
            uint32_t* ne, uint32_t* nodes, uint32_t* flags, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#else
  (void)nthreads;
#endif
  for (int64_t i = 0; i < n; i++) {
    or_tree st;
    st.node = 0;
    st.ne = 0;
    st.flags = 0;
    st.tree = tree_idx[i];
    st.pid = point_id[i];
    /* K = 0 (no non-linear term): no clock, the root is always a leaf */
    st.theta = (pb->K > 0) ? exp(-pb->lambda * t[i]) : 1.0;
    double x0[2] = {x[i * pb->dim], pb->dim == 2 ? x[i * pb->dim + 1] : 0.0};
    double v = pb->strategy == 1 ? or_visit_b(pb, &st, x0, t[i]) : or_visit(pb, &st, x0, 1.0, t[i]);
    F[i] = st.flags ? 0.0 : v;
    ne[i] = st.ne;
    nodes[i] = st.node;
    flags[i] = st.flags;
  }
  return 0;
}
