// Device side of the persistent schedule shared by the large tiled products
// (filter steps in FP64 / FP32 / BF16x3, the Rayleigh-Ritz H C product).
//
// A launch covers `tiles` output tiles: tail.full of them are computed whole,
// the rest are split along K into tail.ksplit segments each (the last,
// partial round of tiles, see plan_schedule).  The grid is one resident wave
// of workgroups; workgroup b runs on XCD b % 8 (the dispatcher deals
// workgroups to the XCDs in rotation).  XCD x owns a contiguous eighth of the
// whole tiles and of the segments (whole tiles that share a row panel of H
// stay on one L2) and its workgroups take items from the XCD's own counter
// one at a time, so a workgroup that finishes early (an edge tile, a short
// segment) starts the next item at once.  With one workgroup per item
// instead, the dispatcher binds each workgroup to a shader engine in a fixed
// rotation and holds it until that engine has room, however many CUs
// elsewhere are idle; measured on gfx950 this left half the chip idle for
// up to half a tile whenever tiles of unequal cost shared a launch.
//
// No workgroup ever waits on another: the counters only hand out work.  The
// last workgroup to leave (counted in queue[8]) clears the counters for the
// next launch on the stream.
#pragma once
#include "kernels.hpp"

namespace chase {

// Order of the tiles of an M x N output in bm x bn tiles.  Row panels of H
// come one after the other (tiles sharing a panel are neighbours); when the
// last column of tiles is ragged, its tiles (cheaper: fewer live columns)
// are all placed after the full-width ones, so the queues hand out the
// longest items first.  plan_schedule numbers tiles the same way.
struct TileOrder {
  int64_t tiles_m, tiles_n;
  bool edge_last;
};

__host__ __device__ __forceinline__ TileOrder tile_order(int64_t M, int64_t N, int bm, int bn) {
  TileOrder o;
  o.tiles_m = (M + bm - 1) / bm;
  o.tiles_n = (N + bn - 1) / bn;
  o.edge_last = o.tiles_n > 1 && N % bn != 0;
  return o;
}

__host__ __device__ __forceinline__ void tile_rc(const TileOrder& o, int64_t tile, int64_t* tm, int64_t* tn) {
  const int64_t wide = o.edge_last ? o.tiles_n - 1 : o.tiles_n;
  const int64_t head = o.tiles_m * wide;
  if (tile < head) {
    *tm = tile / wide;
    *tn = tile % wide;
  } else {
    *tm = tile - head;
    *tn = o.tiles_n - 1;
  }
}

// One item of a launch: a whole tile, or K range [kbeg, kend) of a tile
// whose partial product goes to segment slot `seg` of the tail workspace.
struct WorkItem {
  int64_t tile;  // index in the tile order
  int64_t tm, tn;
  int64_t seg;  // -1: whole tile
  int64_t kbeg, kend;
};

// Item i of the launch in global order (whole tiles first, then segments);
// K ranges are in units of bk-wide K-tiles over kext (K rounded as the
// kernel's loads expect).
__host__ __device__ __forceinline__ WorkItem work_item(const TailSplit& tail, const TileOrder& o, int64_t i,
                                                       int64_t kext, int bk) {
  WorkItem w;
  if (i < tail.full) {
    w.tile = i;
    w.seg = -1;
    w.kbeg = 0;
    w.kend = kext;
  } else {
    const int64_t j = i - tail.full;
    const int64_t tl = j / tail.ksplit, sp = j % tail.ksplit;
    const int64_t nkt = (kext + bk - 1) / bk;
    const int64_t per = (nkt + tail.ksplit - 1) / tail.ksplit;
    w.tile = tail.full + tl;
    w.seg = j;
    w.kbeg = sp * per * bk;
    w.kend = (sp + 1) * per * bk < kext ? (sp + 1) * per * bk : kext;
  }
  tile_rc(o, w.tile, &w.tm, &w.tn);
  return w;
}

// This workgroup's share of the queue.  The launch's items fall in four
// classes, taken in this order: whole full-width tiles, whole tiles of the
// ragged last column, K segments of full-width tiles, K segments of
// last-column tiles.  XCD x owns a contiguous eighth of each class
// (neighbouring tiles share a row panel of H on one L2, and every XCD gets
// the same mix of long and short items).
constexpr int kQueueClasses = 4;
struct QueueShare {
  int xcd;
  int64_t base[kQueueClasses], lo[kQueueClasses], cnt[kQueueClasses];
  int64_t n_items;
};

__host__ __device__ __forceinline__ QueueShare queue_share_for(const TailSplit& tail, const TileOrder& o, int xcd) {
  QueueShare q;
  q.xcd = xcd;
  const int64_t tiles = o.tiles_m * o.tiles_n;
  const int64_t head = o.edge_last ? o.tiles_m * (o.tiles_n - 1) : tiles;  // full-width tiles
  const int64_t f = tail.full, ks = tail.ksplit;
  const int64_t whole_wide = f < head ? f : head;
  const int64_t split_wide = f < head ? head - f : 0;  // split tiles that are full-width
  const int64_t len[kQueueClasses] = {whole_wide, f - whole_wide, split_wide * ks, (tiles - f - split_wide) * ks};
  const int64_t base[kQueueClasses] = {0, whole_wide, f, f + split_wide * ks};
  q.n_items = 0;
  for (int c = 0; c < kQueueClasses; ++c) {
    const int64_t per = (len[c] + 7) / 8;
    const int64_t lo = xcd * per < len[c] ? xcd * per : len[c];
    const int64_t hi = lo + per < len[c] ? lo + per : len[c];
    q.base[c] = base[c];
    q.lo[c] = lo;
    q.cnt[c] = hi - lo;
    q.n_items += hi - lo;
  }
  return q;
}

__device__ __forceinline__ QueueShare queue_share(const TailSplit& tail, const TileOrder& o) {
  return queue_share_for(tail, o, (int)(blockIdx.x % 8));
}

// Global item index of the it-th item of a share (it < n_items): whole tile
// indices below tail.full, segment indices from tail.full on.
__host__ __device__ __forceinline__ int64_t share_item(const QueueShare& q, int64_t it) {
  for (int c = 0; c < kQueueClasses - 1; ++c) {
    if (it < q.cnt[c]) return q.base[c] + q.lo[c] + it;
    it -= q.cnt[c];
  }
  return q.base[kQueueClasses - 1] + q.lo[kQueueClasses - 1] + it;
}

// Fetch-and-add of `add` on *counter by the workgroup, without a divergent
// branch: wave 0 (a uniform, scalar test) issues the atomic from all its
// lanes, lane 0 adding `add` and the others 0, and every thread gets lane
// 0's old value through LDS.  A branch on threadIdx.x == 0 here would, inside
// the item loop, become the divergent latch of that loop after rotation: the
// compiler then splits the loop by lane and lets the waves of a workgroup
// reach its barriers different numbers of times (a deadlock).  Values read
// back from LDS go through readfirstlane for the same reason: a plain LDS
// load counts as divergent.
__device__ __forceinline__ int wg_fetch_add(int* counter, int add, int* sh) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __syncthreads();  // the previous value in *sh has been read by every thread
  if (wave == 0) {
    const int old = atomicAdd(counter, (threadIdx.x & 63) == 0 ? add : 0);
    *sh = __builtin_amdgcn_readfirstlane(old);
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*sh);
}

// Next item of the workgroup's XCD as a global item index, or -1 once the
// XCD's share is exhausted.  Called by every thread; item_sh is LDS.
__device__ __forceinline__ int64_t queue_next(const TailSplit& tail, const QueueShare& q, int* item_sh) {
  const int64_t it = wg_fetch_add(tail.queue + q.xcd, 1, item_sh);
  const int64_t i = it >= q.n_items ? -1 : share_item(q, it);
  // uniform in fact; made uniform for the compiler too, so the item loop's
  // exit is a scalar branch in every instantiation (see wg_fetch_add)
  const uint64_t u = (uint64_t)i;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The workgroup is done with the launch; the last one clears the queue.
__device__ __forceinline__ void queue_leave(const TailSplit& tail) {
  if (threadIdx.x == 0 && atomicAdd(tail.queue + 8, 1) == (int)gridDim.x - 1)
    for (int i = 0; i < 9; ++i) atomicExch(tail.queue + i, 0);
}

}  // namespace chase
