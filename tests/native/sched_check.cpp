// Host check of the work-queue arithmetic the tiled kernels run on the GPU
// (sched.hpp, compiled here for the host): over many launch shapes and K
// splits, the 8 per-XCD shares hand out every item exactly once, the tile
// order is a bijection onto the tile grid, and the K segments of each split
// tile cover [0, K) without gap or overlap.
#include <cstdio>
#include <vector>
#include <set>
#include "kernels.hpp"
#include "sched.hpp"
using namespace chase;
int main() {
  long cases = 0, bad = 0;
  for (long M : {1L, 17L, 128L, 129L, 300L, 517L, 2000L, 20000L})
    for (long N : {1L, 2L, 31L, 32L, 33L, 64L, 100L, 127L, 128L, 129L, 144L, 160L, 300L, 1300L})
      for (int bn : {128, 64}) {
        const int bm = 128;
        TileOrder o = tile_order(M, N, bm, bn);
        const long tiles = o.tiles_m * o.tiles_n;
        std::set<std::pair<long, long>> seen;
        for (long t = 0; t < tiles; ++t) {
          int64_t tm, tn;
          tile_rc(o, t, &tm, &tn);
          if (tm < 0 || tm >= o.tiles_m || tn < 0 || tn >= o.tiles_n) ++bad;
          seen.insert({tm, tn});
        }
        if ((long)seen.size() != tiles) ++bad;
        for (long full = 0; full <= tiles; full += (tiles > 16 ? tiles / 7 + 1 : 1))
          for (long ks : {1L, 2L, 3L, 5L, 8L}) {
            if (full == tiles && ks != 1) continue;
            TailSplit t;
            t.full = full;
            t.ksplit = ks;
            const long items = full + (tiles - full) * ks;
            std::vector<int> hits(items, 0);
            for (int x = 0; x < 8; ++x) {
              QueueShare q = queue_share_for(t, o, x);
              for (long it = 0; it < q.n_items; ++it) {
                long i = share_item(q, it);
                if (i < 0 || i >= items) { ++bad; continue; }
                hits[i]++;
              }
            }
            for (long i = 0; i < items; ++i) if (hits[i] != 1) ++bad;
            // segments of every split tile, in order, tile [0, K)
            for (long K : {1L, 7L, 8L, 16L, 517L, 20000L})
              for (int bk : {8, 16, 32}) {
                const long kext = (K + bk - 1) / bk * bk;  // the padded extent a kernel may pass
                for (long kx : {K, kext}) {
                  std::vector<long> pos(tiles, 0);
                  for (long i = full; i < items; ++i) {
                    const WorkItem w = work_item(t, o, i, kx, bk);
                    if (w.seg != i - full || w.tile != full + (i - full) / ks) ++bad;
                    if (w.kbeg % bk) ++bad;
                    if (w.kbeg < w.kend && w.kbeg != pos[w.tile]) ++bad;
                    if (w.kend > pos[w.tile]) pos[w.tile] = w.kend;
                  }
                  for (long tile = full; tile < tiles; ++tile)
                    if (pos[tile] != kx) ++bad;
                }
              }
            ++cases;
          }
      }
  printf("%ld schedules checked, %ld violations\n", cases, bad);
  return bad != 0;
}
