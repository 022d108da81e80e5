// Continuous-batching server for point queries (brt_server_* in include/brt.h).
//
// An engine thread runs ticks.  A tick gives every unfinished point of the requests it covers one more
// round of `round_trees` trees: the rounds of those requests are packed into launch groups of up to
// kGroupPoints points and kMaxProblems requests (problems), so requests of different sizes and horizons
// share launches; a group whose problems differ only in their initial data runs the walker's family
// mode (shared constants in scalar registers).  Each point owns a device slot holding the reduction
// partials of all its rounds; the finalize recomputes the point's coefficients, Pade value and SE from
// the slot after every round.  A point finishes when its SE reaches the target or its trees reach the cap; a request completes
// when all its points have finished.  New requests are admitted at tick
// boundaries while free slots remain (memory admission); a point's slot is freed as soon as the point
// finishes and its results are read; the submission queue is bounded.
//
// Admitted requests are split between two lanes, each with its own stream, staging and device buffers
// (the slots and their partials are shared).  The engine alternates: it waits for one lane's tick, reads
// its results (copied back by the tick itself), admits requests and enqueues that lane's next tick,
// while the other lane's tick runs on the GPU.  So the host's packing and bookkeeping overlap the
// device's work, and the two lanes' kernels may overlap on the device.
//
// A point's trees are addressed by (seed, point id, tree counter), its partials are combined in round
// order, and the number of rounds depends only on its own SE: its results are bit-identical whether it
// is served alone or among other requests, in either lane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "brt.h"
#include "brt_api.h"
#include "brt_internal.h"

using namespace brt;
using Clock = std::chrono::steady_clock;

namespace {

constexpr uint32_t kMaxRequestPoints = 1024;
constexpr uint32_t kChunkTrees = 1024;
constexpr int kLanes = 2;
// Launch groups: consecutive requests of a lane until the group holds kGroupPoints unfinished points or
// kMaxProblems requests.  The walker keeps the group's problem table in LDS beside its stack levels (at 64
// full FP32 records, 16 KB, it costs a third of the walker's resident waves; a family of problems that
// differ only in their initial data keeps just those, 8.4 KB at most), so large requests go in small
// groups and only small requests share a launch with many others.
constexpr uint32_t kGroupPoints = 4096;
// Walker blocks per CU left free by a launch group's persistent walker (when it would hold three or
// more): the other lane's reduction and finalize then run beside it instead of waiting for its end.
constexpr int kSpareBlocks = 1;
constexpr uint32_t kCounterStride = 16;  // 64 bytes between the chunk counters of a lane's launch groups

struct Request {
  uint64_t ticket = 0;
  brt_problem prob{};
  Norm norm;
  uint32_t stream_id = 0;
  uint32_t n = 0;
  int lane = 0;
  std::vector<double> x, t;
  Clock::time_point arrival, finished_at;
  std::vector<uint32_t> slot, rounds;
  std::vector<uint8_t> done;
  uint32_t n_done = 0;
  bool complete = false;
  std::vector<double> u, se, coef;
  std::vector<uint32_t> flags;
};

// One lane: a stream, its launch staging (pinned) and device buffers, and the read-back of its ticks.
struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_done = nullptr;
  void* d_pdes = nullptr;                 // problem tables of the tick's launch groups, back to back
  PointRec* d_points = nullptr;           // [max_points]
  Chunk* d_chunks = nullptr;              // [max_points * chunks_per_round]
  Segment* d_segs = nullptr;              // [max_points * segs_per_round]
  uint32_t* d_counter = nullptr;          // [max_groups * kCounterStride]
  unsigned long long* d_depth = nullptr;  // [max_groups]
  double* d_tree_f = nullptr;             // [max_points * round_trees]
  uint32_t* d_tree_meta = nullptr;
  void* d_spill = nullptr;
  PointRec* h_points = nullptr;
  Chunk* h_chunks = nullptr;
  Segment* h_segs = nullptr;
  unsigned char* h_pdes = nullptr;
  double *h_u = nullptr, *h_se = nullptr, *h_coef = nullptr;  // read-back, indexed by slot
  unsigned long long* h_nodes = nullptr;
  uint32_t* h_flags = nullptr;
  std::vector<Request*> reqs;      // admitted, unfinished requests of this lane
  std::vector<Request*> inflight;  // the requests of the tick in flight
  bool busy = false;
  uint32_t slot_lo = 0, slot_hi = 0;  // slots read back by the tick in flight
};

}  // namespace

struct brt_server {
  int device = 0;
  int n_cu = 0;
  brt_server_opts opts{};
  uint32_t B = 0, NB = 0, seg_trees = 0, segs_per_round = 0, max_segs = 0, chunks_per_round = 0, max_groups = 0;
  int wpb = 4, lds_depth = 0, spill_depth = 0;
  int grid_k[kMaxProblems + 1] = {};  // resident walker blocks for a launch group of k problems
  int wpb_k[kMaxProblems + 1] = {};   // and their waves per block
  // the same for a launch group whose problems form a family, by its initial-data stride (found at
  // creation for the strides the served initial-data kind has; -1: no block size fits, the group takes
  // the full table)
  int fam_grid[kMaxProblems + 1][kMaxU0Params + 1] = {};
  int fam_wpb[kMaxProblems + 1][kMaxU0Params + 1] = {};
  size_t spill_threads = 0;           // the spill area's stride: the most threads of any group's launch
  Lane lanes[kLanes];
  // per-slot device state shared by the lanes (each slot belongs to one point of one lane at a time)
  Partial* d_partials = nullptr;
  unsigned long long* d_seg_nodes = nullptr;
  double *d_u = nullptr, *d_se = nullptr, *d_coef = nullptr;
  unsigned long long* d_nodes = nullptr;
  uint32_t* d_flags = nullptr;
  // state
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> requests;
  std::vector<uint32_t> free_slots;
  uint32_t n_active = 0;  // admitted, incomplete requests
  uint64_t next_ticket = 1;
  bool stop = false;     // finish the admitted requests, then exit
  bool abandon = false;  // exit at the next tick boundary
  int engine_rc = BRT_OK;
  char engine_msg[512] = {};  // the engine's error (a fixed buffer: recording it never allocates)
  std::thread engine;
  // statistics
  std::vector<double> latencies;
  uint64_t submitted = 0, completed = 0, rejected = 0, ticks = 0, trees = 0, nodes = 0;
  double busy_s = 0.0;
  bool any_submit = false;
  Clock::time_point first_submit, last_complete;
};

namespace {

#define SRV_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return set_error(BRT_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

void server_free(brt_server* s) {
  if (!s) return;
  for (Lane& L : s->lanes) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    void* dev[] = {L.d_pdes, L.d_points, L.d_chunks, L.d_segs, L.d_counter, L.d_depth, L.d_tree_f, L.d_tree_meta,
                   L.d_spill};
    for (void* p : dev) (void)hipFree(p);
    void* host[] = {L.h_points, L.h_chunks, L.h_segs, L.h_pdes, L.h_u, L.h_se, L.h_coef, L.h_nodes, L.h_flags};
    for (void* p : host) (void)hipHostFree(p);
    if (L.ev_start) (void)hipEventDestroy(L.ev_start);
    if (L.ev_done) (void)hipEventDestroy(L.ev_done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  void* dev[] = {s->d_partials, s->d_seg_nodes, s->d_u, s->d_se, s->d_coef, s->d_nodes, s->d_flags};
  for (void* p : dev) (void)hipFree(p);
  for (auto& kv : s->requests) delete kv.second;
  for (Request* r : s->queue)
    if (!s->requests.count(r->ticket)) delete r;
  delete s;
}

// The resident grid and block size of a family launch of k problems at initial-data stride `stride`
// (the block size with the most resident waves, the larger on a tie), found once.
void family_launch(brt_server* s, int k, int stride) {
  int& fg = s->fam_grid[k][stride];
  if (fg != 0) return;
  const brt_mc& mc = s->opts.mc;
  int maxb = 0, wb = 0;
  for (int c = kMaxWalkThreads / kWave; c >= 1; --c) {
    const int b = walk_max_blocks_per_cu((int)mc.precision, (int)s->opts.dim, (int)s->opts.u0_kind, k, s->lds_depth, c,
                                         (int)mc.strategy, stride);
    if (b * c > maxb * wb) maxb = b, wb = c;
  }
  // the spill area holds spill_threads threads' levels
  if (maxb > 0 && s->spill_depth > 0)
    maxb = std::min<int>(maxb, (int)(s->spill_threads / ((size_t)wb * kWave * s->n_cu)));
  if (maxb >= 2 + kSpareBlocks) maxb -= kSpareBlocks;
  fg = maxb > 0 ? maxb * s->n_cu : -1;
  s->fam_wpb[k][stride] = wb;
}

template <typename T>
int dev_alloc(T** p, size_t n) {
  if (hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(1, n) * sizeof(T)) != hipSuccess)
    return set_error(BRT_E_NOMEM, "server: device allocation of %zu bytes failed", n * sizeof(T));
  return BRT_OK;
}

template <typename T>
int host_alloc(T** p, size_t n) {
  if (hipHostMalloc(reinterpret_cast<void**>(p), std::max<size_t>(1, n) * sizeof(T)) != hipSuccess)
    return set_error(BRT_E_NOMEM, "server: pinned allocation of %zu bytes failed", n * sizeof(T));
  return BRT_OK;
}

// Enqueue one tick of a lane on its stream: one round for every unfinished point of the lane's requests,
// in launch groups (kGroupPoints, kMaxProblems), then the copies of every slot's results back to the
// lane's pinned buffers and the completion event.  Nothing here waits for the device.
int issue_tick(brt_server* s, Lane& L) {
  const brt_mc& mc = s->opts.mc;
  const uint32_t R = s->opts.round_trees;
  const size_t pb = pde_bytes((int)mc.precision);
  struct Item {
    Request* r;
    uint32_t i, k;
    double cost;
  };
  std::vector<Item> items;
  uint32_t np = 0, nc = 0, ns = 0, slot_lo = ~0u, slot_hi = 0;
  L.inflight = L.reqs;
  SRV_TRY(hipEventRecord(L.ev_start, L.stream));
  for (size_t g0 = 0, grp = 0, prob_off = 0; g0 < L.reqs.size(); ++grp) {
    size_t g1 = g0;
    for (uint32_t pts = 0; g1 < L.reqs.size() && g1 - g0 < (size_t)kMaxProblems && pts < kGroupPoints; ++g1)
      pts += L.reqs[g1]->n - L.reqs[g1]->n_done;
    const size_t gprob = prob_off, kprob = g1 - g0;
    prob_off += kprob;
    // the group's points, most expensive first (longest-processing-time order of the chunks)
    items.clear();
    uint32_t cmod = 0;
    unsigned char* pdes = L.h_pdes + gprob * pb;
    for (size_t k = g0; k < g1; ++k) {
      Request* r = L.reqs[k];
      pde_to_device(r->prob, r->norm, (int)mc.precision, pdes + (k - g0) * pb);
      cmod |= general_coefficients(r->prob) ? 1u : 0u;
      for (uint32_t i = 0; i < r->n; ++i)
        if (!r->done[i]) items.push_back(Item{r, i, (uint32_t)(k - g0), est_nodes(r->norm, mc, r->t[i])});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    const uint32_t p0 = np, c0 = nc, s0 = ns;
    for (const Item& it : items) {
      Request* r = it.r;
      const uint32_t slot = r->slot[it.i];
      const uint32_t round = r->rounds[it.i];
      slot_lo = std::min(slot_lo, slot);
      slot_hi = std::max(slot_hi, slot + 1);
      PointRec& pr = L.h_points[np];
      std::memset(&pr, 0, sizeof(pr));
      pr.x[0] = r->x[(size_t)it.i * s->opts.dim];
      pr.x[1] = s->opts.dim == 2 ? r->x[(size_t)it.i * 2 + 1] : 0.0;
      pr.t = r->t[it.i];
      pr.theta = r->norm.K > 0 ? std::exp(-r->norm.lambda * pr.t) : 1.0;
      pr.mu = r->norm.mu;
      pr.tree_base = (uint64_t)np * R;
      pr.n_trees = R;
      pr.point_id = r->stream_id * kMaxRequestPoints + it.i;
      pr.pde = it.k;
      pr.tree_first = round * R;
      pr.n_total = (uint64_t)(round + 1) * R;
      pr.seg_begin = slot * s->max_segs;
      pr.seg_count = (round + 1) * s->segs_per_round;
      pr.out_row = slot;
      for (uint32_t g = 0; g < s->segs_per_round; ++g)
        L.h_segs[ns++] = Segment{np, g * s->seg_trees, (g + 1) * s->seg_trees, slot * s->max_segs + round * s->segs_per_round + g};
      ++np;
    }
    // chunks interleaved in cost order: all points' first chunks, then their second chunks, ...
    for (uint32_t c = 0; c < s->chunks_per_round; ++c)
      for (uint32_t p = p0; p < np; ++p) L.h_chunks[nc++] = Chunk{p, c * kChunkTrees, (c + 1) * kChunkTrees, 0u};
    g0 = g1;  // the next group starts after this one
    if (np == p0) continue;
    void* d_pdes = static_cast<unsigned char*>(L.d_pdes) + gprob * pb;
    SRV_TRY(hipMemcpyAsync(d_pdes, pdes, kprob * pb, hipMemcpyHostToDevice, L.stream));
    SRV_TRY(hipMemcpyAsync(L.d_points + p0, L.h_points + p0, (np - p0) * sizeof(PointRec), hipMemcpyHostToDevice,
                           L.stream));
    SRV_TRY(hipMemcpyAsync(L.d_chunks + c0, L.h_chunks + c0, (nc - c0) * sizeof(Chunk), hipMemcpyHostToDevice, L.stream));
    SRV_TRY(hipMemcpyAsync(L.d_segs + s0, L.h_segs + s0, (ns - s0) * sizeof(Segment), hipMemcpyHostToDevice, L.stream));
    uint32_t* counter = L.d_counter + grp * kCounterStride;
    unsigned long long* depth = L.d_depth + grp;
    SRV_TRY(launch_reset(counter, depth, L.stream));
    WalkArgs w{};
    w.points = L.d_points;
    w.chunks = L.d_chunks + c0;
    w.n_chunks = nc - c0;
    w.n_problems = (uint32_t)kprob;
    w.pdes = d_pdes;
    w.chunk_counter = counter;
    w.depth_counter = depth;
    w.tree_f = L.d_tree_f;
    w.tree_meta = L.d_tree_meta;
    w.spill = L.d_spill;
    w.key0 = (uint32_t)(mc.seed & 0xffffffffull);
    w.key1 = (uint32_t)(mc.seed >> 32);
    w.max_order = mc.max_order;
    w.prune = mc.prune;
    w.node_cap = mc.node_cap;
    w.strategy = mc.strategy;
    w.cmod = cmod;
    w.stack_depth = (uint32_t)s->lds_depth;
    w.spill_depth = (uint32_t)s->spill_depth;
    w.n_threads = (uint32_t)s->spill_threads;
    // a family (requests that differ only in their initial data) keeps only the initial data per problem
    // in the block's table: more resident blocks, and the node step's constants stay in scalar registers
    int kgrid = s->grid_k[kprob], kwpb = s->wpb_k[kprob];
    w.u0_stride = family_u0_stride((int)mc.precision, s->opts.u0_kind, pdes, kprob);
    if (w.u0_stride) {
      family_launch(s, (int)kprob, (int)w.u0_stride);
      if (s->fam_grid[kprob][w.u0_stride] > 0) {
        kgrid = s->fam_grid[kprob][w.u0_stride];
        kwpb = s->fam_wpb[kprob][w.u0_stride];
      } else {
        w.u0_stride = 0;
      }
    }
    const int grid = std::max(1, std::min<int>(kgrid, (int)(nc - c0)));
    SRV_TRY(launch_walk((int)mc.precision, (int)s->opts.dim, (int)s->opts.u0_kind, w, grid, kwpb, L.stream));
    ReduceArgs ra{};
    ra.points = L.d_points;
    ra.segs = L.d_segs + s0;
    ra.n_segs = ns - s0;
    ra.tree_f = L.d_tree_f;
    ra.tree_meta = L.d_tree_meta;
    ra.partials = s->d_partials;
    ra.seg_nodes = s->d_seg_nodes;
    ra.n_bins = s->B;
    SRV_TRY(launch_reduce(ra, L.stream));
    FinalizeArgs f{};
    f.points = L.d_points + p0;
    f.n_points = np - p0;
    f.partials = s->d_partials;
    f.seg_nodes = s->d_seg_nodes;
    f.n_bins = s->B;
    f.pade_L = mc.pade_L;
    f.pade_M = mc.pade_M;
    f.u = s->d_u;
    f.se = s->d_se;
    f.coef = s->d_coef;
    f.nodes = s->d_nodes;
    f.flags = s->d_flags;
    SRV_TRY(launch_finalize(f, L.stream));
  }
  // the lane's results back to its pinned buffers (the span of slots its points occupy)
  if (np > 0) {
    const size_t n = slot_hi - slot_lo;
    SRV_TRY(hipMemcpyAsync(L.h_u + slot_lo, s->d_u + slot_lo, n * sizeof(double), hipMemcpyDeviceToHost, L.stream));
    SRV_TRY(hipMemcpyAsync(L.h_se + slot_lo, s->d_se + slot_lo, n * sizeof(double), hipMemcpyDeviceToHost, L.stream));
    SRV_TRY(hipMemcpyAsync(L.h_flags + slot_lo, s->d_flags + slot_lo, n * sizeof(uint32_t), hipMemcpyDeviceToHost,
                           L.stream));
    SRV_TRY(hipMemcpyAsync(L.h_nodes + slot_lo, s->d_nodes + slot_lo, n * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, L.stream));
    SRV_TRY(hipMemcpyAsync(L.h_coef + (size_t)slot_lo * s->B, s->d_coef + (size_t)slot_lo * s->B,
                           n * s->B * sizeof(double), hipMemcpyDeviceToHost, L.stream));
  }
  SRV_TRY(hipEventRecord(L.ev_done, L.stream));
  L.slot_lo = np ? slot_lo : 0;
  L.slot_hi = np ? slot_hi : 0;
  L.busy = true;
  return BRT_OK;
}

// Wait for a lane's tick and fold its results into its requests (called without the lock; takes it).
int finish_tick(brt_server* s, Lane& L) {
  SRV_TRY(hipEventSynchronize(L.ev_done));
  float ms = 0.f;
  SRV_TRY(hipEventElapsedTime(&ms, L.ev_start, L.ev_done));
  L.busy = false;
  const uint32_t R = s->opts.round_trees;
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  s->busy_s += ms * 1e-3;
  s->ticks += 1;
  std::vector<Request*> still;
  for (Request* r : L.inflight) {
    for (uint32_t i = 0; i < r->n; ++i) {
      if (r->done[i]) continue;
      const uint32_t slot = r->slot[i];
      r->rounds[i] += 1;
      s->trees += R;
      const uint64_t n_trees = (uint64_t)r->rounds[i] * R;
      const double se = L.h_se[slot];
      const bool reached = s->opts.target_se > 0.0 && se <= s->opts.target_se;
      if (reached || n_trees >= s->opts.max_trees) {
        r->done[i] = 1;
        r->n_done += 1;
        r->u[i] = L.h_u[slot];
        r->se[i] = se;
        r->flags[i] = L.h_flags[slot];
        s->nodes += L.h_nodes[slot];
        std::memcpy(r->coef.data() + (size_t)i * s->B, L.h_coef + (size_t)slot * s->B, s->B * sizeof(double));
        s->free_slots.push_back(slot);  // the point's results are on the host: its slot takes the next point
      }
    }
    if (r->n_done == r->n) {
      r->complete = true;
      r->finished_at = now;
      s->latencies.push_back(std::chrono::duration<double>(now - r->arrival).count());
      s->completed += 1;
      s->n_active -= 1;
      s->last_complete = now;
    } else {
      still.push_back(r);
    }
  }
  // requests admitted into this lane while its tick ran are already in L.reqs after the in-flight ones
  std::vector<Request*> added(L.reqs.begin() + (ptrdiff_t)L.inflight.size(), L.reqs.end());
  L.reqs.swap(still);
  L.reqs.insert(L.reqs.end(), added.begin(), added.end());
  L.inflight.clear();
  s->done_cv.notify_all();
  return BRT_OK;
}

// Admission (under the lock): queued requests in arrival order while their points fit the free slots and
// the cap on requests in flight allows; each goes to the lane with fewer unfinished points.
void admit(brt_server* s) {
  while (!s->queue.empty()) {
    Request* r = s->queue.front();
    if (r->n > s->free_slots.size()) break;
    if (s->opts.max_active_requests && s->n_active >= s->opts.max_active_requests) break;
    s->queue.pop_front();
    for (uint32_t i = 0; i < r->n; ++i) {
      r->slot[i] = s->free_slots.back();
      s->free_slots.pop_back();
    }
    size_t load[kLanes] = {0, 0};
    for (int l = 0; l < kLanes; ++l)
      for (Request* q : s->lanes[l].reqs) load[l] += q->n - q->n_done;
    r->lane = load[1] < load[0] ? 1 : 0;
    s->lanes[r->lane].reqs.push_back(r);
    s->n_active += 1;
  }
}

void engine_fail(brt_server* s, int rc) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->engine_rc = rc;
  std::snprintf(s->engine_msg, sizeof(s->engine_msg), "%s", brt_last_error());
  s->stop = true;
  s->done_cv.notify_all();
}

void engine_loop(brt_server* s) {
  if (hipSetDevice(s->device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->engine_rc = BRT_E_DEVICE;
    std::snprintf(s->engine_msg, sizeof(s->engine_msg), "%s", "server engine: hipSetDevice failed");
    s->done_cv.notify_all();
    return;
  }
  int turn = 0;
  while (true) {
    Lane& L = s->lanes[turn];
    if (L.busy) {
      const int rc = finish_tick(s, L);
      if (rc) return engine_fail(s, rc);
    }
    bool issue = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->abandon) return;
      admit(s);
      issue = !L.reqs.empty();
      if (!issue && !s->lanes[turn ^ 1].busy && s->lanes[turn ^ 1].reqs.empty()) {
        // nothing in flight and nothing admitted
        if (s->stop && s->queue.empty()) return;
        s->cv.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
    }
    if (issue) {
      const int rc = issue_tick(s, L);
      if (rc) return engine_fail(s, rc);
    }
    turn ^= 1;
  }
}

// The engine thread: a C++ exception (a failed host allocation in the bookkeeping) stops the server
// with an error that submit and poll then report, instead of terminating the process.
void engine_main(brt_server* s) {
  try {
    engine_loop(s);
  } catch (const std::bad_alloc&) {
    engine_fail(s, set_error(BRT_E_NOMEM, "server engine: host allocation failed"));
  } catch (...) {
    engine_fail(s, set_error(BRT_E_ARG, "server engine: internal error"));
  }
}

}  // namespace

extern "C" {

int brt_server_create(brt_ctx* ctx, const brt_server_opts* o, brt_server** out) {
  return brt::api_guard("brt_server_create", [&]() -> int {
    if (!ctx || !o || !out) return set_error(BRT_E_ARG, "brt_server_create: NULL argument");
    *out = nullptr;
    if (o->struct_size != sizeof(brt_server_opts)) return set_error(BRT_E_ARG, "brt_server_opts.struct_size mismatch");
    if (o->dim != 1 && o->dim != 2) return set_error(BRT_E_ARG, "server: dim must be 1 or 2");
    if (o->u0_kind > BRT_U0_COS2_BUMP) return set_error(BRT_E_ARG, "server: unknown u0_kind");
    const brt_mc& mc = o->mc;
    if (mc.struct_size != sizeof(brt_mc) || (mc.precision != 32 && mc.precision != 64) || !(mc.lambda > 0.0) ||
        mc.max_order > 126 || mc.node_cap < 1 || mc.node_cap > kMaxNodeCap || mc.pade_L + mc.pade_M > mc.max_order ||
        mc.pade_M > 16 || mc.strategy > BRT_STRATEGY_B)
      return set_error(BRT_E_ARG, "server: invalid Monte Carlo parameters");
    if (o->max_points < 1 || o->max_points > (1u << 20)) return set_error(BRT_E_ARG, "server: max_points must be 1..2^20");
    if (o->round_trees < kSegTrees || o->round_trees % kSegTrees || o->round_trees > (1u << 22))
      return set_error(BRT_E_ARG, "server: round_trees must be a multiple of %u, at most 2^22", kSegTrees);
    if (o->max_trees < o->round_trees || o->max_trees % o->round_trees || o->max_trees > (1u << 26))
      return set_error(BRT_E_ARG, "server: max_trees must be a multiple of round_trees, at most 2^26");
    if (!(o->target_se >= 0.0)) return set_error(BRT_E_ARG, "server: target_se must be >= 0");
    if (o->queue_cap < 1) return set_error(BRT_E_ARG, "server: queue_cap must be >= 1");

    brt_server* s = new (std::nothrow) brt_server;
    if (!s) return set_error(BRT_E_NOMEM, "server: host allocation");
    s->opts = *o;
    brt_launch lc{};
    lc.struct_size = sizeof(lc);
    brt_get_launch(ctx, &lc);
    s->wpb = (int)lc.waves_per_block;
    hipDeviceProp_t prop;
    if (hipGetDevice(&s->device) != hipSuccess || hipGetDeviceProperties(&prop, s->device) != hipSuccess) {
      server_free(s);
      return set_error(BRT_E_DEVICE, "server: device query failed");
    }
    s->n_cu = prop.multiProcessorCount;
    s->B = mc.max_order + 2;
    s->NB = s->B + 3;
    // reduction segments: the largest power of two up to the plan's largest segment that divides a
    // round (one segment per point and round at the default 32768 trees): fewer, longer segments make
    // both the reduction (fewer per-bin butterflies) and every tick's exact join in the finalize cheaper
    s->seg_trees = kSegTrees;
    while (s->seg_trees < kPlanSegMax && o->round_trees % (2 * s->seg_trees) == 0) s->seg_trees *= 2;
    s->segs_per_round = o->round_trees / s->seg_trees;
    s->max_segs = o->max_trees / s->seg_trees;
    s->chunks_per_round = o->round_trees / kChunkTrees;
    const uint32_t needed = mc.prune ? std::max(1u, mc.max_order) : kMaxDepthUnpruned;
    s->lds_depth = (int)std::min(needed, lc.stack_depth ? lc.stack_depth : kDefaultLdsLevels);
    s->spill_depth = (int)(needed - (uint32_t)s->lds_depth);
    // resident blocks per CU and waves per block for every launch-group size.  One problem takes the
    // context's block size (reduced if one problem's table does not fit); a group of several takes the
    // block size with the most resident waves, the larger one on a tie: every block holds its own copy of
    // the group's problem table in LDS, so larger blocks share a copy among more waves
    auto fit = [&](int k, int w) {
      return walk_max_blocks_per_cu((int)mc.precision, (int)o->dim, (int)o->u0_kind, k, s->lds_depth, w,
                                    (int)mc.strategy);
    };
    for (int k = 1; k <= kMaxProblems; ++k) {
      int maxb = 0, w = 0;
      if (k == 1) {
        for (w = s->wpb; w >= 1 && (maxb = fit(k, w)) <= 0;) --w;
      } else {
        for (int c = kMaxWalkThreads / kWave; c >= 1; --c) {
          const int b = fit(k, c);
          if (b * c > maxb * w) maxb = b, w = c;
        }
      }
      if (maxb <= 0 || w <= 0) {
        server_free(s);
        return set_error(BRT_E_ARG, "server: walker launch for %d problems does not fit the device", k);
      }
      s->grid_k[k] = (maxb >= 2 + kSpareBlocks ? maxb - kSpareBlocks : maxb) * s->n_cu;
      s->wpb_k[k] = w;
      s->spill_threads = std::max(s->spill_threads, (size_t)s->grid_k[k] * w * kWave);
    }
    // family launches at every stride the served initial-data kind can give (Gaussian sums: 4 per term)
    for (int k = 2; k <= kMaxProblems; ++k) {
      if (o->u0_kind == BRT_U0_GAUSS_SUM) {
        for (int st = 4; st <= kMaxU0Params; st += 4) family_launch(s, k, st);
      } else {
        family_launch(s, k, (int)u0_param_count(o->u0_kind, 0));
      }
    }
    const size_t P = o->max_points;
    const size_t R = o->round_trees;
    int rc = BRT_OK;
    s->max_groups = (uint32_t)P;  // at most one group per request
    const size_t pb = pde_bytes((int)mc.precision);
    const size_t spill = s->spill_depth > 0 ? s->spill_threads * s->spill_depth *
                                                  stack_entry_size((int)mc.precision, (int)o->dim)
                                            : 0;
    for (Lane& L : s->lanes) {
      rc = rc ? rc : (hipStreamCreate(&L.stream) == hipSuccess ? BRT_OK : set_error(BRT_E_DEVICE, "server: stream"));
      rc = rc ? rc : (hipEventCreate(&L.ev_start) == hipSuccess ? BRT_OK : set_error(BRT_E_DEVICE, "server: event"));
      rc = rc ? rc : (hipEventCreate(&L.ev_done) == hipSuccess ? BRT_OK : set_error(BRT_E_DEVICE, "server: event"));
      rc = rc ? rc : dev_alloc(reinterpret_cast<unsigned char**>(&L.d_pdes), P * pb);  // one problem per request
      rc = rc ? rc : dev_alloc(&L.d_points, P);
      rc = rc ? rc : dev_alloc(&L.d_chunks, P * s->chunks_per_round);
      rc = rc ? rc : dev_alloc(&L.d_segs, P * s->segs_per_round);
      rc = rc ? rc : dev_alloc(&L.d_counter, (size_t)s->max_groups * kCounterStride);
      rc = rc ? rc : dev_alloc(&L.d_depth, s->max_groups);
      rc = rc ? rc : dev_alloc(&L.d_tree_f, P * R);
      rc = rc ? rc : dev_alloc(&L.d_tree_meta, P * R);
      if (!rc && spill) rc = dev_alloc(reinterpret_cast<unsigned char**>(&L.d_spill), spill);
      rc = rc ? rc : host_alloc(&L.h_points, P);
      rc = rc ? rc : host_alloc(&L.h_chunks, P * s->chunks_per_round);
      rc = rc ? rc : host_alloc(&L.h_segs, P * s->segs_per_round);
      rc = rc ? rc : host_alloc(&L.h_pdes, P * pb);
      rc = rc ? rc : host_alloc(&L.h_u, P);
      rc = rc ? rc : host_alloc(&L.h_se, P);
      rc = rc ? rc : host_alloc(&L.h_coef, P * s->B);
      rc = rc ? rc : host_alloc(&L.h_nodes, P);
      rc = rc ? rc : host_alloc(&L.h_flags, P);
    }
    rc = rc ? rc : dev_alloc(&s->d_partials, P * s->max_segs * s->NB);
    rc = rc ? rc : dev_alloc(&s->d_seg_nodes, P * s->max_segs);
    rc = rc ? rc : dev_alloc(&s->d_u, P);
    rc = rc ? rc : dev_alloc(&s->d_se, P);
    rc = rc ? rc : dev_alloc(&s->d_coef, P * s->B);
    rc = rc ? rc : dev_alloc(&s->d_nodes, P);
    rc = rc ? rc : dev_alloc(&s->d_flags, P);
    if (rc) {
      server_free(s);
      return rc;
    }
    s->free_slots.resize(P);
    for (size_t i = 0; i < P; ++i) s->free_slots[i] = (uint32_t)(P - 1 - i);
    s->engine = std::thread(engine_main, s);
    *out = s;
    return BRT_OK;
  });
}

int brt_server_submit(brt_server* s, const brt_request* q, uint64_t* ticket) {
  return brt::api_guard("brt_server_submit", [&]() -> int {
    if (!s || !q || !ticket) return set_error(BRT_E_ARG, "brt_server_submit: NULL argument");
    if (q->struct_size != sizeof(brt_request)) return set_error(BRT_E_ARG, "brt_request.struct_size mismatch");
    if (!q->problem || !q->x || !q->t) return set_error(BRT_E_ARG, "brt_server_submit: NULL array");
    if (q->n < 1 || q->n > kMaxRequestPoints || q->n > s->opts.max_points)
      return set_error(BRT_E_ARG, "brt_server_submit: 1..%u points per request", std::min(kMaxRequestPoints, s->opts.max_points));
    if (q->stream_id >= (1u << 22)) return set_error(BRT_E_ARG, "brt_server_submit: stream_id must be < 2^22");
    int rc = brt_problem_check(q->problem, &s->opts.mc);
    if (rc) return rc;
    if (q->problem->dim != s->opts.dim || q->problem->u0_kind != s->opts.u0_kind)
      return set_error(BRT_E_ARG, "brt_server_submit: problem dim/u0_kind differ from the server's");
    for (uint32_t i = 0; i < q->n; ++i)
      if (!(q->t[i] >= 0.0) || !std::isfinite(q->t[i])) return set_error(BRT_E_ARG, "brt_server_submit: bad t");
    Request* r = new (std::nothrow) Request;
    if (!r) return set_error(BRT_E_NOMEM, "brt_server_submit: host allocation");
    r->prob = *q->problem;
    r->norm = normalize(r->prob, s->opts.mc);
    r->stream_id = q->stream_id;
    r->n = q->n;
    r->x.assign(q->x, q->x + (size_t)q->n * s->opts.dim);
    r->t.assign(q->t, q->t + q->n);
    r->slot.assign(q->n, 0u);
    r->rounds.assign(q->n, 0u);
    r->done.assign(q->n, 0u);
    r->u.assign(q->n, 0.0);
    r->se.assign(q->n, 0.0);
    r->flags.assign(q->n, 0u);
    r->coef.assign((size_t)q->n * s->B, 0.0);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->engine_rc) {
      delete r;
      return set_error(s->engine_rc, "server stopped: %s", s->engine_msg);
    }
    if (s->queue.size() >= s->opts.queue_cap) {
      delete r;
      s->rejected += 1;
      return set_error(BRT_E_BUSY, "server: admission queue full (%u requests)", s->opts.queue_cap);
    }
    r->ticket = s->next_ticket++;
    r->arrival = Clock::now();
    if (!s->any_submit) {
      s->any_submit = true;
      s->first_submit = r->arrival;
    }
    s->submitted += 1;
    s->queue.push_back(r);
    s->requests[r->ticket] = r;
    *ticket = r->ticket;
    s->cv.notify_all();
    return BRT_OK;
  });
}

int brt_server_poll(brt_server* s, uint64_t ticket, brt_result* out, int* done) {
  return brt::api_guard("brt_server_poll", [&]() -> int {
    if (!s || !done) return set_error(BRT_E_ARG, "brt_server_poll: NULL argument");
    if (out && out->struct_size != sizeof(brt_result)) return set_error(BRT_E_ARG, "brt_result.struct_size mismatch");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return set_error(BRT_E_STATE, "brt_server_poll: unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second;
    *done = r->complete ? 1 : 0;
    if (!r->complete) {
      if (s->engine_rc) return set_error(s->engine_rc, "server stopped: %s", s->engine_msg);
      return BRT_OK;
    }
    if (out) {
      const uint32_t R = s->opts.round_trees;
      for (uint32_t i = 0; i < r->n; ++i) {
        if (out->u) out->u[i] = r->u[i];
        if (out->se) out->se[i] = r->se[i];
        if (out->flags) out->flags[i] = r->flags[i];
        if (out->trees) out->trees[i] = (uint64_t)r->rounds[i] * R;
      }
      if (out->coef) std::memcpy(out->coef, r->coef.data(), r->coef.size() * sizeof(double));
      out->latency_s = std::chrono::duration<double>(r->finished_at - r->arrival).count();
    }
    s->requests.erase(it);
    delete r;
    return BRT_OK;
  });
}

int brt_server_drain(brt_server* s, double timeout_s) {
  return brt::api_guard("brt_server_drain", [&]() -> int {
    if (!s) return set_error(BRT_E_ARG, "brt_server_drain: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = Clock::now() + std::chrono::duration<double>(timeout_s);
    while (!s->queue.empty() || s->n_active > 0) {
      if (s->engine_rc) return set_error(s->engine_rc, "server stopped: %s", s->engine_msg);
      if (s->done_cv.wait_until(lk, deadline) == std::cv_status::timeout && (!s->queue.empty() || s->n_active > 0))
        return set_error(BRT_E_BUSY, "brt_server_drain: timed out");
    }
    return s->engine_rc;
  });
}

int brt_server_stats_get(brt_server* s, brt_server_stats* o) {
  return brt::api_guard("brt_server_stats_get", [&]() -> int {
    if (!s || !o || o->struct_size != sizeof(brt_server_stats)) return set_error(BRT_E_ARG, "brt_server_stats_get: bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
      if (l.empty()) return 0.0;
      const double pos = q * (double)(l.size() - 1);
      const size_t i = (size_t)pos;
      const double f = pos - (double)i;
      return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
    };
    o->submitted = s->submitted;
    o->completed = s->completed;
    o->rejected = s->rejected;
    o->ticks = s->ticks;
    o->trees = s->trees;
    o->nodes = s->nodes;
    o->p50_latency_s = pct(0.50);
    o->p99_latency_s = pct(0.99);
    o->mean_latency_s = l.empty() ? 0.0 : std::accumulate(l.begin(), l.end(), 0.0) / (double)l.size();
    o->busy_s = s->busy_s;
    o->span_s = (s->any_submit && s->completed) ? std::chrono::duration<double>(s->last_complete - s->first_submit).count() : 0.0;
    o->trees_per_s = o->span_s > 0 ? (double)s->trees / o->span_s : 0.0;
    return BRT_OK;
  });
}

void brt_server_destroy(brt_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->abandon = true;  // requests in flight are abandoned at the next tick boundary
    // requests never admitted are dropped
    for (Request* r : s->queue) {
      s->requests.erase(r->ticket);
      delete r;
    }
    s->queue.clear();
    s->cv.notify_all();
  }
  if (s->engine.joinable()) s->engine.join();
  s->queue.clear();
  server_free(s);
}

}  // extern "C"
