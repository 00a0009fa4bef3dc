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

namespace chase {

namespace {

double tile_cost(const TileGeom& g, int64_t tiles_n, int64_t tile) {
  const int64_t tm = tile / tiles_n, tn = tile % tiles_n;
  const int64_t rm = std::min<int64_t>(g.bm, g.M - tm * g.bm), rn = std::min<int64_t>(g.bn, g.N - tn * g.bn);
  const int waves = g.wgm * g.wgn;
  const int sub_m = g.bm / g.wgm, sub_n = g.bn / g.wgn;
  int load[4] = {0, 0, 0, 0};
  for (int w = 0; w < waves; ++w)
    if ((w % g.wgm) * sub_m < rm && (w / g.wgm) * sub_n < rn) ++load[w % 4];
  const int busiest = *std::max_element(load, load + 4);
  const int full = (waves + 3) / 4;
  return (double)busiest / full;
}

constexpr double kSegmentOverhead = 3e-3;  // partial-tile store and sum, per segment

// Makespan of the per-XCD queues for `full` whole tiles and the rest split
// into ks segments each, with `grid` workgroups.
double simulate(const TileGeom& g, int64_t tiles_n, int64_t tiles, int64_t full, int64_t ks, int64_t grid,
                const std::vector<double>& cost) {
  const int64_t nseg = (tiles - full) * ks;
  const int64_t per_m = cdiv(full, 8), per_t = cdiv(nseg, 8);
  const int64_t wgs = std::max<int64_t>(1, grid / 8);
  double makespan = 0.0;
  for (int x = 0; x < 8; ++x) {
    std::priority_queue<double, std::vector<double>, std::greater<double>> freeq;
    for (int64_t i = 0; i < wgs; ++i) freeq.push(0.0);
    auto take = [&](double c) {
      const double t = freeq.top() + c;
      freeq.pop();
      freeq.push(t);
      makespan = std::max(makespan, t);
    };
    const int64_t m_lo = std::min(x * per_m, full), m_hi = std::min(m_lo + per_m, full);
    for (int64_t i = m_lo; i < m_hi; ++i) take(cost[i]);
    const int64_t t_lo = std::min(x * per_t, nseg), t_hi = std::min(t_lo + per_t, nseg);
    for (int64_t j = t_lo; j < t_hi; ++j) take(cost[full + j / ks] / (double)ks + kSegmentOverhead);
  }
  return makespan;
}

int64_t grid_for(int64_t resident, int64_t full, int64_t nseg) {
  const int64_t wave = 8 * cdiv(resident, 8);
  const int64_t need = 8 * (cdiv(full, 8) + cdiv(nseg, 8));
  return std::min(wave, need);
}

struct PlanCache {
  std::mutex mu;
  std::map<std::tuple<int64_t, int64_t, int64_t, int, int, int, int, int64_t, int, bool>, std::pair<int64_t, int64_t>>
      plans;
};
PlanCache& plan_cache() {
  static PlanCache c;
  return c;
}

}  // namespace

int64_t plan_schedule(const TileGeom& g, int64_t nkt, int64_t resident, int min_kt_per_seg, bool allow_split,
                      void* ws, int* counters, TailSplit* t) {
  const int64_t tiles_n = cdiv(g.N, g.bn);
  const int64_t tiles = cdiv(g.M, g.bm) * tiles_n;
  t->full = tiles;
  t->ksplit = 1;
  t->ws = ws;
  t->counters = counters;
  t->queue = counters + kTailMaxSegments;
  if (allow_split && ws && tiles > 0) {
    const auto key = std::make_tuple(g.M, g.N, nkt, g.bm, g.bn, g.wgm, g.wgn, resident, min_kt_per_seg, allow_split);
    PlanCache& pc = plan_cache();
    std::lock_guard<std::mutex> lock(pc.mu);
    auto it = pc.plans.find(key);
    if (it == pc.plans.end()) {
      std::vector<double> cost((size_t)tiles);
      for (int64_t i = 0; i < tiles; ++i) cost[(size_t)i] = tile_cost(g, tiles_n, i);
      int64_t best_full = tiles, best_ks = 1;
      double best = simulate(g, tiles_n, tiles, tiles, 1, grid_for(resident, tiles, 0), cost);
      // split the tiles of the last round, or of the last round and a half
      const int64_t rem = tiles % resident;
      for (int64_t r : {rem, rem + resident / 2}) {
        if (r <= 0 || r > tiles) continue;
        for (int64_t ks = 2; ks <= 8; ++ks) {
          if (nkt < (int64_t)min_kt_per_seg * ks || r * ks > kTailMaxSegments) break;
          const int64_t full = tiles - r;
          const double m = simulate(g, tiles_n, tiles, full, ks, grid_for(resident, full, r * ks), cost);
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
