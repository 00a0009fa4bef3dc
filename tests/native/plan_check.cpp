// Host check of the split-K planner (schedule.cpp) together with the work
// queue it drives (sched.hpp): over launch shapes of the filter (128 x 128
// tiles, 8 waves, the narrow edge layouts) and of the 128 x 64 tile, every
// plan keeps within the segment cap and splits only tiles it does not
// compute whole; the grid is a multiple of 8 no larger than one resident
// wave of workgroups; and the items the 8 per-XCD shares hand out cover
// every tile's K range exactly once.
#include <cstdio>
#include <vector>
#include "kernels.hpp"
#include "sched.hpp"
using namespace chase;
int main() {
  long cases = 0, bad = 0, split = 0;
  static char ws_dummy[16];
  std::vector<int> counters(kTailCounterInts, 0);
  for (long M : {1L, 100L, 128L, 517L, 2000L, 7001L, 20000L, 50000L})
    for (long N : {1L, 20L, 32L, 33L, 64L, 65L, 128L, 192L, 300L, 1024L, 1300L, 2400L})
      for (int cfg = 0; cfg < 2; ++cfg)
        for (long K : {16L, 517L, 2000L, 20000L})
          for (long resident : {256L, 512L, 80L})
            for (int maxseg : {kTailMaxSegments, 64}) {
              TileGeom g;
              g.M = M; g.N = N;
              g.bm = 128; g.bn = cfg == 0 ? 128 : 64; g.wgm = 2; g.wgn = cfg == 0 ? 4 : 2;
              g.narrow_cols = cfg == 0 ? 32 : 0;
              const int bk = cfg == 0 ? 16 : 8;
              const long nkt = (K + bk - 1) / bk;
              TailSplit t;
              const long grid = plan_schedule(g, nkt, resident, 16, true, ws_dummy, counters.data(), &t, maxseg);
              const TileOrder o = tile_order(M, N, g.bm, g.bn);
              const long tiles = o.tiles_m * o.tiles_n;
              if (t.full < 0 || t.full > tiles || t.ksplit < 1 || t.ksplit > 8) ++bad;
              if (t.full == tiles && t.ksplit != 1) ++bad;
              if ((tiles - t.full) * t.ksplit > maxseg) ++bad;
              if (grid < 8 || grid % 8 || grid > 8 * ((resident + 7) / 8)) ++bad;
              if (t.ws != ws_dummy || t.counters != counters.data() || t.queue != counters.data() + kTailMaxSegments) ++bad;
              if (t.ksplit > 1) ++split;
              const long items = t.full + (tiles - t.full) * t.ksplit;
              std::vector<int> hits(items, 0);
              std::vector<long> covered(tiles, 0);
              for (int x = 0; x < 8; ++x) {
                const QueueShare q = queue_share_for(t, o, x);
                for (long it = 0; it < q.n_items; ++it) {
                  const long i = share_item(q, it);
                  if (i < 0 || i >= items) { ++bad; continue; }
                  hits[i]++;
                  const WorkItem w = work_item(t, o, i, K, bk);
                  if (w.tile < 0 || w.tile >= tiles || w.kbeg < 0 || w.kend > K || w.kbeg > w.kend) { ++bad; continue; }
                  covered[w.tile] += w.kend - w.kbeg;
                }
              }
              for (long i = 0; i < items; ++i) if (hits[i] != 1) ++bad;
              for (long tile = 0; tile < tiles; ++tile) if (covered[tile] != K) ++bad;
              ++cases;
            }
  printf("%ld plans checked (%ld split along K), %ld violations\n", cases, split, bad);
  return bad != 0;
}
