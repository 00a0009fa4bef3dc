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

// One item of a launch: a whole tile, or K range [kbeg, kend) of a tile
// whose partial product goes to segment slot `seg` of the tail workspace.
struct WorkItem {
  int64_t tile;
  int64_t seg;  // -1: whole tile
  int64_t kbeg, kend;
};

// Item i of the launch in global order (whole tiles first, then segments);
// K ranges are in units of bk-wide K-tiles over kext (K rounded as the
// kernel's loads expect).
__device__ __forceinline__ WorkItem work_item(const TailSplit& tail, int64_t i, int64_t kext, int bk) {
  WorkItem w;
  if (i < tail.full) {
    w.tile = i;
    w.seg = -1;
    w.kbeg = 0;
    w.kend = kext;
    return w;
  }
  const int64_t j = i - tail.full;
  const int64_t tl = j / tail.ksplit, sp = j % tail.ksplit;
  const int64_t nkt = (kext + bk - 1) / bk;
  const int64_t per = (nkt + tail.ksplit - 1) / tail.ksplit;
  w.tile = tail.full + tl;
  w.seg = j;
  w.kbeg = sp * per * bk;
  w.kend = (sp + 1) * per * bk < kext ? (sp + 1) * per * bk : kext;
  return w;
}

// This workgroup's share of the queue: its XCD's whole tiles [m_lo, m_lo +
// n_main) and segments [t_lo, t_lo + n_items - n_main).
struct QueueShare {
  int xcd;
  int64_t m_lo, n_main, t_lo, n_items;
};

__device__ __forceinline__ QueueShare queue_share(const TailSplit& tail, int64_t tiles) {
  QueueShare q;
  q.xcd = (int)(blockIdx.x % 8);
  const int64_t per_m = (tail.full + 7) / 8;
  q.m_lo = q.xcd * per_m < tail.full ? q.xcd * per_m : tail.full;
  const int64_t m_hi = q.m_lo + per_m < tail.full ? q.m_lo + per_m : tail.full;
  const int64_t nseg = (tiles - tail.full) * tail.ksplit;
  const int64_t per_t = (nseg + 7) / 8;
  q.t_lo = q.xcd * per_t < nseg ? q.xcd * per_t : nseg;
  const int64_t t_hi = q.t_lo + per_t < nseg ? q.t_lo + per_t : nseg;
  q.n_main = m_hi - q.m_lo;
  q.n_items = q.n_main + (t_hi - q.t_lo);
  return q;
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
  if (it >= q.n_items) return -1;
  return it < q.n_main ? q.m_lo + it : tail.full + q.t_lo + (it - q.n_main);
}

// The workgroup is done with the launch; the last one clears the queue.
__device__ __forceinline__ void queue_leave(const TailSplit& tail) {
  if (threadIdx.x == 0 && atomicAdd(tail.queue + 8, 1) == (int)gridDim.x - 1)
    for (int i = 0; i < 9; ++i) atomicExch(tail.queue + i, 0);
}

}  // namespace chase
