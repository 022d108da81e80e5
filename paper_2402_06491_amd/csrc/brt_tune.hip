// Launch-setting autotuner (brt_autotune in include/brt.h).
//
// Times the tree walker for every candidate (waves per block x LDS stack levels x chunk size) on a
// subsample of the caller's points, with HIP events around the walk kernel, keeps the fastest in the
// context and records it in a JSON-lines cache keyed by the GPU architecture and the workload shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "brt.h"
#include "brt_api.h"
#include "brt_internal.h"

using namespace brt;

namespace {

std::string tune_key(const char* arch, const brt_problem& p, const brt_mc& mc, uint32_t n_problems) {
  uint32_t K = 0, amax = 0;
  for (uint32_t j = 0; j < 8; ++j)
    if (j != 1 && p.coef[j] != 0.0) {
      K += 1;
      amax = j;
    }
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|p%u|d%u|g%u|m%u|K%u|a%u|o%u|r%u", arch, mc.precision, p.dim, p.u0_kind,
           n_problems > 1 ? 1u : 0u, K, amax, mc.max_order, mc.prune);
  return buf;
}

bool cache_lookup(const char* path, const std::string& key, brt_launch* out) {
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char k[512];
    unsigned w = 0, d = 0, c = 0;
    // {"key": "<key>", "waves_per_block": W, "stack_depth": D, "chunk_trees": C, ...}
    if (sscanf(line, " {\"key\": \"%511[^\"]\", \"waves_per_block\": %u, \"stack_depth\": %u, \"chunk_trees\": %u", k, &w,
               &d, &c) == 4 &&
        key == k) {
      out->waves_per_block = w;
      out->stack_depth = d;
      out->chunk_trees = c;
      found = true;  // the last entry for a key wins
    }
  }
  fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const brt_launch& l, double ms) {
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"waves_per_block\": %u, \"stack_depth\": %u, \"chunk_trees\": %u, \"walk_ms\": %.6f}\n",
          key.c_str(), l.waves_per_block, l.stack_depth, l.chunk_trees, ms);
  fclose(f);
}

}  // namespace

extern "C" int brt_autotune(brt_ctx* ctx, uint32_t n_problems, const brt_problem* problems, const brt_mc* mc,
                            const brt_points* pts, const char* cache_path, brt_launch* best) {
  return brt::api_guard("brt_autotune", [&]() -> int {
    if (!ctx || !problems || !mc || !pts || n_problems < 1) return set_error(BRT_E_ARG, "brt_autotune: NULL argument");
    if (pts->struct_size != sizeof(brt_points)) return set_error(BRT_E_ARG, "brt_points.struct_size mismatch");
    int rc = brt_problem_check(&problems[0], mc);
    if (rc) return rc;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
      return set_error(BRT_E_DEVICE, "brt_autotune: device query failed");
    const std::string key = tune_key(prop.gcnArchName, problems[0], *mc, n_problems);
    brt_launch cur{};
    cur.struct_size = sizeof(cur);
    brt_get_launch(ctx, &cur);
    brt_launch found = cur;
    if (cache_lookup(cache_path, key, &found)) {
      rc = brt_set_launch(ctx, &found);
      if (rc) return rc;
      if (best) *best = found;
      return BRT_OK;
    }

    // subsample: every point keeps its share, at most about 2^28 trees in total (workloads below that are
    // timed whole), at least 1024 each; shorter samples let the drain of the persistent grid at the end of
    // a launch decide the ranking
    uint64_t total = 0;
    for (uint32_t i = 0; i < pts->n; ++i) total += pts->n_trees[i];
    if (total == 0) return set_error(BRT_E_ARG, "brt_autotune: no trees to time");
    const double frac = std::min(1.0, (double)(1u << 28) / (double)total);
    std::vector<uint64_t> sub(pts->n);
    for (uint32_t i = 0; i < pts->n; ++i)
      sub[i] = pts->n_trees[i] ? std::max<uint64_t>(std::min<uint64_t>(1024, pts->n_trees[i]),
                                                    (uint64_t)((double)pts->n_trees[i] * frac))
                               : 0;
    brt_points sp = *pts;
    sp.n_trees = sub.data();
    sp.tree_first = nullptr;

    const uint32_t needed = mc->prune ? std::max(1u, mc->max_order) : 64u;
    const uint32_t waves[] = {1, 2, 4};
    const uint32_t depths[] = {4, 6, 8, 12, 16};
    const uint32_t chunks[] = {256, 1024, 4096};
    double best_ms = 1e30;
    brt_launch best_l = cur;
    for (uint32_t w : waves)
      for (uint32_t d : depths) {
        if (d > needed && d != depths[0]) continue;
        for (uint32_t c : chunks) {
          brt_launch l{};
          l.struct_size = sizeof(l);
          l.waves_per_block = w;
          l.blocks_per_cu = 0;
          l.chunk_trees = c;
          l.stack_depth = std::min(d, needed);
          if (brt_set_launch(ctx, &l)) continue;
          brt_plan* plan = nullptr;
          if (brt_plan_create(ctx, n_problems, problems, mc, &sp, &plan)) continue;  // does not fit: skip
          brt_out o{};
          o.struct_size = sizeof(o);
          int erc = brt_plan_set_timing(plan, 1);
          erc = erc ? erc : brt_plan_execute(plan, &o, nullptr);  // warm-up
          double ms[3] = {0, 0, 0};
          uint64_t runs = 0;
          erc = erc ? erc : brt_plan_get_timing(plan, ms, &runs);
          double walk = 1e30;  // fastest of three runs
          for (int k = 0; !erc && k < 3; ++k) {
            erc = brt_plan_execute(plan, &o, nullptr);
            erc = erc ? erc : brt_plan_get_timing(plan, ms, &runs);
            if (!erc && runs) walk = std::min(walk, ms[0] / (double)runs);
          }
          brt_plan_destroy(plan);
          if (erc) {
            brt_set_launch(ctx, &cur);
            return erc;
          }
          if (walk < best_ms) {
            best_ms = walk;
            best_l = l;
          }
        }
      }
    if (best_ms >= 1e30) {
      brt_set_launch(ctx, &cur);
      return set_error(BRT_E_ARG, "brt_autotune: no candidate launch fits the device");
    }
    rc = brt_set_launch(ctx, &best_l);
    if (rc) return rc;
    cache_store(cache_path, key, best_l, best_ms);
    if (best) *best = best_l;
    return BRT_OK;
  });
}
