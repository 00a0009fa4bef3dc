// Host side of the persistent tile schedule (device side: sched.hpp): how
// many of a launch's tiles are computed whole and how the rest are split
// along K, chosen by simulating the per-XCD work queues.
//
// Cost model, in units of one interior tile's time: the MFMA work of a tile
// sits on the 4 SIMDs of a CU, waves w and w + 4 of the workgroup on one
// SIMD (measured on gfx950), so a tile takes as long as its busiest SIMD.
// Waves whose sub-tile lies outside the output do no MFMA work, so e.g. a
// last column tile with at most 64 live columns costs half a tile.  A K
// segment costs its share of the K range, plus a little for storing and
// summing partial tiles.  The queues are simulated as each XCD's workgroups
// taking its items in order, each item going to the workgroup that frees
// first.
#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <queue>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "sched.hpp"

namespace chase {

namespace {

constexpr double kSegmentOverhead = 3e-3;  // partial-tile store and sum, per segment
constexpr double kTileFixed = 0.13;

double tile_cost(const TileGeom& g, int64_t tile) {
  int64_t tm, tn;
  tile_rc(tile_order(g.M, g.N, g.bm, g.bn), tile, &tm, &tn);
  const int64_t rm = std::min<int64_t>(g.bm, g.M - tm * g.bm), rn = std::min<int64_t>(g.bn, g.N - tn * g.bn);
  const int waves = g.wgm * g.wgn;
  int wgm = g.wgm;  // edge layouts of a ragged last column
  if (g.narrow_cols > 0 && rn <= g.narrow_cols) wgm = waves;
  else if (g.narrow_cols > 0 && rn <= 2 * g.narrow_cols) wgm = waves / 2;
  const int sub_m = g.bm / wgm, sub_n = g.bn / g.wgn;
  // work of one wave relative to a wave of the main layout
  const double work = (double)sub_m / (g.bm / g.wgm);
  int load[4] = {0, 0, 0, 0};
  for (int w = 0; w < waves; ++w)
    if ((w % wgm) * sub_m < rm && (w / wgm) * sub_n < rn) ++load[w % 4];
  const int busiest = *std::max_element(load, load + 4);
  const int full = (waves + 3) / 4;
  // a fixed share of a tile's time does not shrink with its MFMA work
  // (prologue, epilogue, barriers): fitted to step times measured at
  // N = 20000 with 16 to 1300 columns
  return kTileFixed + (1.0 - kTileFixed) * busiest * work / full;
}


// Makespan of the per-XCD queues for `full` whole tiles and the rest split
// into ks segments each, with `grid` workgroups (the device's queue_share).
double simulate(const TileGeom& g, int64_t tiles, int64_t full, int64_t ks, int64_t grid,
                const std::vector<double>& cost) {
  const TileOrder o = tile_order(g.M, g.N, g.bm, g.bn);
  TailSplit t;
  t.full = full;
  t.ksplit = ks;
  const int64_t wgs = std::max<int64_t>(1, grid / 8);
  double makespan = 0.0;
  for (int x = 0; x < 8; ++x) {
    const QueueShare q = queue_share_for(t, o, x);
    std::priority_queue<double, std::vector<double>, std::greater<double>> freeq;
    for (int64_t i = 0; i < wgs; ++i) freeq.push(0.0);
    for (int64_t it = 0; it < q.n_items; ++it) {
      const int64_t i = share_item(q, it);
      const double c = i < full ? cost[(size_t)i] : cost[(size_t)(full + (i - full) / ks)] / (double)ks + kSegmentOverhead;
      const double t_end = freeq.top() + c;
      freeq.pop();
      freeq.push(t_end);
      makespan = std::max(makespan, t_end);
    }
  }
  (void)tiles;
  return makespan;
}

int64_t grid_for(int64_t resident, int64_t full, int64_t nseg) {
  const int64_t wave = 8 * cdiv(resident, 8);
  const int64_t need = 8 * (cdiv(full, 8) + cdiv(nseg, 8));
  return std::min(wave, need);
}

struct PlanCache {
  std::mutex mu;
  std::map<std::tuple<int64_t, int64_t, int64_t, int, int, int, int, int64_t, int, bool, int>,
           std::pair<int64_t, int64_t>>
      plans;
};
PlanCache& plan_cache() {
  static PlanCache c;
  return c;
}

}  // namespace

int64_t plan_schedule(const TileGeom& g, int64_t nkt, int64_t resident, int min_kt_per_seg, bool allow_split,
                      void* ws, int* counters, TailSplit* t, int max_segments) {
  max_segments = std::max(0, std::min(max_segments, kTailMaxSegments));
  const int64_t tiles_n = cdiv(g.N, g.bn);
  const int64_t tiles = cdiv(g.M, g.bm) * tiles_n;
  t->full = tiles;
  t->ksplit = 1;
  t->ws = ws;
  t->counters = counters;
  t->queue = counters + kTailMaxSegments;
  if (allow_split && ws && tiles > 0) {
    const auto key = std::make_tuple(g.M, g.N, nkt, g.bm, g.bn, g.wgm, g.wgn * 1000 + g.narrow_cols, resident,
                                     min_kt_per_seg, allow_split, max_segments);
    PlanCache& pc = plan_cache();
    std::lock_guard<std::mutex> lock(pc.mu);
    auto it = pc.plans.find(key);
    if (it == pc.plans.end()) {
      std::vector<double> cost((size_t)tiles);
      for (int64_t i = 0; i < tiles; ++i) cost[(size_t)i] = tile_cost(g, i);
      int64_t best_full = tiles, best_ks = 1;
      double best = simulate(g, tiles, tiles, 1, grid_for(resident, tiles, 0), cost);
      // split the last r tiles: the last partial round, plus up to all the
      // rest in steps of an eighth of a round (cheap edge tiles can leave
      // whole tiles as the critical path)
      const int64_t rem = tiles % resident;
      std::vector<int64_t> cands;
      for (int64_t r = rem; r < tiles; r += std::max<int64_t>(1, resident / 8)) cands.push_back(r);
      cands.push_back(tiles);
      for (int64_t r : cands) {
        if (r <= 0 || r > tiles) continue;
        for (int64_t ks = 2; ks <= 8; ++ks) {
          if (nkt < (int64_t)min_kt_per_seg * ks || r * ks > max_segments) break;
          const int64_t full = tiles - r;
          const double m = simulate(g, tiles, full, ks, grid_for(resident, full, r * ks), cost);
          if (m < best - 1e-6) {
            best = m;
            best_full = full;
            best_ks = ks;
          }
        }
      }
      it = pc.plans.emplace(key, std::make_pair(best_full, best_ks)).first;
    }
    t->full = it->second.first;
    t->ksplit = it->second.second;
  }
  return grid_for(resident, t->full, (tiles - t->full) * t->ksplit);
}

}  // namespace chase
