// BF16x3 split-precision filter step (mixed-precision solve, lowest rung):
//
//   Y = alpha H X + beta Y + gamma X        (X, Y, Z complex64; FP32 accumulate)
//
// H and X are each split into two bfloat16 parts, x = x_hi + x_lo with
// x_hi = bf16(x) and x_lo = bf16(x - x_hi), which keeps ~16 significant bits.
// Every real product is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi (the
// a_lo b_lo term is below that precision) on V_MFMA_F32_16X16X32_BF16 with
// FP32 accumulation, so one complex multiply-add costs 12 bf16 MFMA products.
// The real part's negative term Im(X) Im(H) is accumulated on its own and
// subtracted in the epilogue, so no negated planes are stored.
//
// H is stored once per solve as four bfloat16 planes (Re hi, Re lo, Im hi,
// Im lo) of conj(H) in H's own memory order: H is Hermitian, so column m of
// the stored matrix, conjugated, is row m of H, and each output row then
// reads K-contiguous runs.  Rows are padded to a multiple of 32 with zeros.
// The block X comes as the same four planes, column by column: each step's
// epilogue writes the planes of its output beside the FP32 result, so the
// split happens once per element and step.  (Splitting in the consumer
// repeats it for every 128-row panel of H, and measured as the larger part
// of the step's time.)
//
// Tiling: 128 (m) x 128 (n) complex tile, 8 waves of 64 x 32, K tile 32 (one
// MFMA K step).  Both operands go from memory straight to LDS
// (global_load_lds_dwordx4, 16 bytes per lane: 8 k of one plane of one row),
// two K tiles of the four H planes and the four X planes (bf16, 64-byte rows,
// 16-byte chunks XOR-swizzled by row so that the 16 lanes of a fragment read
// hit distinct banks): 128 KB.  The last partial round of tiles is split
// along K as in the FP64 kernel.  The MFMA row index
// is the output column n and the column index the output row m; the f32
// accumulator layout (lane l, element r: row 4 (l/16) + r, column l % 16)
// was measured on gfx950.
#include "common.hpp"
#include "kernels.hpp"
#include "sched.hpp"

namespace chase {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128, BK = 32, NT = 512;
constexpr int TM = 4, TN = 2;  // 16-blocks per wave along m and n

struct alignas(8) cv {
  float re, im;
};

__device__ __forceinline__ uint32_t bf16_bits(float x) {  // round to nearest even
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

struct BSmem {
  uint4 h[2][4][BM][BK / 8];  // [buffer][plane][m][chunk of 8 k]
  uint4 x[2][4][BN][BK / 8];  // [buffer][plane][n][chunk]
};

__device__ __forceinline__ int swz(int row, int chunk) { return chunk ^ ((row >> 2) & 3); }


// The four bfloat16 planes of an output value, for the next step's X.
__device__ __forceinline__ void store_planes(const BGemmArgs& g, int64_t m, int64_t n, cv v) {
  const uint32_t a = bf16_bits(v.re), b = bf16_bits(v.im);
  uint16_t* q = g.Yp + n * g.ldyp + m;
  q[0] = (uint16_t)a;
  q[g.yps] = (uint16_t)bf16_bits(v.re - bf16_value(a));
  q[2 * g.yps] = (uint16_t)b;
  q[3 * g.yps] = (uint16_t)bf16_bits(v.im - bf16_value(b));
}

// One 128 x 128 output tile over K range [kbeg, kend) (multiples of BK, kend
// may exceed K: both operands' planes are zero-padded in k).
template <bool EDGE>
__device__ __forceinline__ void btile(const BGemmArgs& g, int64_t tm, int64_t tn, int64_t kbeg, int64_t kend,
                                      cv* part, BSmem& s) {
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, kq = lane >> 4;
  // EDGE tiles: a wave whose 64 x 32 sub-tile lies wholly outside the output
  // skips its fragment reads and MFMAs; one that touches it computes the
  // whole sub-tile on the zero-padded operands.  The test is a single
  // wave-uniform branch per K-tile, so the MFMA stream is never split.
  const bool active = !EDGE || (m0 + wm * 64 < g.M && n0 + wn * 32 < g.N);
  f32x4 rp[TN][TM], rn_[TN][TM], im[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      rp[a][b] = f32x4{0, 0, 0, 0};
      rn_[a][b] = f32x4{0, 0, 0, 0};
      im[a][b] = f32x4{0, 0, 0, 0};
    }

  // Loads of K tile [k0, k0 + 32) into buffer `buf`: 64 instructions, 8 per
  // wave.  Instruction i moves 16 rows (H, i < 32) or 16 columns (X) of plane
  // (i / 8) % 4; lane l takes row (column) 16 (i mod 8) + l / 4 and stores the
  // chunk that belongs at position l % 4 of its swizzled row.  Rows past M and
  // columns past N are not loaded (they only reach discarded outputs); k past
  // K reads the planes' zero padding.
  auto issue = [&](int64_t k0, int buf) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int i = wave * 8 + r;
      const bool is_h = i < 32;
      const int p = (i >> 3) & 3, r0 = (i & 7) << 4;
      const int row = r0 + (lane >> 2);
      const int c = (lane & 3) ^ ((row >> 2) & 3);  // chunk stored at position lane & 3
      if (is_h) {
        const int64_t m = m0 + row;
        if (!EDGE || m < g.M)
          __builtin_amdgcn_global_load_lds(g.P + p * g.plane_stride + m * g.ldp + k0 + 8 * c, &s.h[buf][p][r0][0],
                                           16, 0, 0);
      } else {
        const int64_t n = n0 + row;
        if (!EDGE || n < g.N)
          __builtin_amdgcn_global_load_lds(g.Xp + p * g.xps + n * g.ldxp + k0 + 8 * c, &s.x[buf][p][r0][0], 16, 0,
                                           0);
      }
    }
  };

  const int64_t nkt = (kend - kbeg) / BK;
  if (nkt > 0) issue(kbeg, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // Every wave issues the next K tile's loads after its X fragment reads,
  // before its first row block of MFMAs: the loads get the whole K tile to
  // land.  (Staggering waves w and w + 4, which share a SIMD, as the FP64
  // step does, measured 3 % slower here: 11.50 against 11.11 ms at N =
  // 20000, 1300 columns; issuing before the fragment reads, 13.58 ms.)
  const int issue_at = 0;
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int buf = (int)(kt & 1);
    {
      bf16x8 xf[TN][4];
      if (active) {
#pragma unroll
        for (int nb = 0; nb < TN; ++nb) {
          const int n = wn * 32 + nb * 16 + l16;
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const uint4 w = s.x[buf][p][n][swz(n, kq)];
            xf[nb][p] = __builtin_bit_cast(bf16x8, w);
          }
        }
      }
#pragma unroll
      for (int mb = 0; mb < TM; ++mb) {
        // buffer buf ^ 1 was last read before the previous barrier
        if (mb == issue_at && kt + 1 < nkt) issue(kbeg + (kt + 1) * BK, buf ^ 1);
        if (!active) continue;
        const int m = wm * 64 + mb * 16 + l16;
        bf16x8 hf[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) hf[p] = __builtin_bit_cast(bf16x8, s.h[buf][p][m][swz(m, kq)]);
        // planes: 0 Re hi, 1 Re lo, 2 Im hi, 3 Im lo
#define BMMA(acc, xp, hp)                                                                   \
  _Pragma("unroll") for (int nb = 0; nb < TN; ++nb)                                        \
      acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xf[nb][xp], hf[hp], acc[nb][mb], 0, 0, 0);
        BMMA(rp, 0, 0) BMMA(rn_, 2, 2) BMMA(im, 0, 2) BMMA(im, 2, 0)
        BMMA(rp, 0, 1) BMMA(rn_, 2, 3) BMMA(im, 0, 3) BMMA(im, 2, 1)
        BMMA(rp, 1, 0) BMMA(rn_, 3, 2) BMMA(im, 1, 2) BMMA(im, 3, 0)
#undef BMMA
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next K tile have landed
    __syncthreads();
  }

  if (part != nullptr) {
#pragma unroll
    for (int nb = 0; nb < TN; ++nb)
#pragma unroll
      for (int mb = 0; mb < TM; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int nl = wn * 32 + nb * 16 + 4 * kq + r;
          const int ml = wm * 64 + mb * 16 + l16;
          part[ml + nl * BM] = cv{rp[nb][mb][r] - rn_[nb][mb][r], im[nb][mb][r]};
        }
    return;
  }
  cv* Y = reinterpret_cast<cv*>(g.Y);
  const cv* Z = reinterpret_cast<const cv*>(g.Z);
#pragma unroll
  for (int nb = 0; nb < TN; ++nb)
#pragma unroll
    for (int mb = 0; mb < TM; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * 32 + nb * 16 + 4 * kq + r;
        const int64_t m = m0 + wm * 64 + mb * 16 + l16;
        if (m >= g.M || n >= g.N) continue;
        cv out{g.alpha * (rp[nb][mb][r] - rn_[nb][mb][r]), g.alpha * im[nb][mb][r]};
        if (g.beta != 0.f) {
          const cv y = Y[m + n * g.ldy];
          out.re += g.beta * y.re;
          out.im += g.beta * y.im;
        }
        if (g.gamma != 0.f) {
          const cv z = Z[m + n * g.ldz];
          out.re += g.gamma * z.re;
          out.im += g.gamma * z.im;
        }
        Y[m + n * g.ldy] = out;
        store_planes(g, m, n, out);
      }
}

__device__ __forceinline__ void btile_any(const BGemmArgs& g, int64_t tm, int64_t tn, int64_t kbeg, int64_t kend,
                                          cv* part, BSmem& s) {
  if ((tm + 1) * BM <= g.M && (tn + 1) * BN <= g.N)
    btile<false>(g, tm, tn, kbeg, kend, part, s);
  else
    btile<true>(g, tm, tn, kbeg, kend, part, s);
}

// A segment has stored its partial tile: count it in; the last segment of a
// tile to arrive sums the partials in segment order and applies the epilogue.
__device__ __forceinline__ void barrive(const BGemmArgs& g, const TailSplit& tail, const WorkItem& w, int* last) {
  const int64_t tl = w.seg / tail.ksplit;
  const int64_t tm = w.tm, tn = w.tn;
  __threadfence();
  if (wg_fetch_add(tail.counters + tl, 1, last) != tail.ksplit - 1) return;
  __threadfence();
  const cv* parts = reinterpret_cast<const cv*>(tail.ws) + tl * tail.ksplit * (int64_t)(BM * BN);
  cv* Y = reinterpret_cast<cv*>(g.Y);
  const cv* Z = reinterpret_cast<const cv*>(g.Z);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  for (int e = threadIdx.x; e < BM * BN; e += NT) {
    const int64_t m = m0 + e % BM, n = n0 + e / BM;
    if (m >= g.M || n >= g.N) continue;
    float sr = 0.f, si = 0.f;
    for (int q = 0; q < tail.ksplit; ++q) {
      const cv v = parts[q * (int64_t)(BM * BN) + e];
      sr += v.re;
      si += v.im;
    }
    cv out{g.alpha * sr, g.alpha * si};
    if (g.beta != 0.f) {
      const cv y = Y[m + n * g.ldy];
      out.re += g.beta * y.re;
      out.im += g.beta * y.im;
    }
    if (g.gamma != 0.f) {
      const cv z = Z[m + n * g.ldz];
      out.re += g.gamma * z.re;
      out.im += g.gamma * z.im;
    }
    Y[m + n * g.ldy] = out;
    store_planes(g, m, n, out);
  }
  if (threadIdx.x == 0) tail.counters[tl] = 0;
}

// Persistent grid on the per-XCD work queue (sched.hpp).
__global__ __launch_bounds__(NT, 1) void bfilter_step(BGemmArgs g, TailSplit tail) {
  __shared__ BSmem s;
  __shared__ int last, item;
  const int64_t kpad = (g.K + BK - 1) / BK * BK;
  const TileOrder o = tile_order(g.M, g.N, BM, BN);
  const QueueShare q = queue_share(tail, o);
  for (int64_t i; (i = queue_next(tail, q, &item)) >= 0;) {
    const WorkItem w = work_item(tail, o, i, kpad, BK);
    cv* part = w.seg < 0 ? nullptr : reinterpret_cast<cv*>(tail.ws) + w.seg * (int64_t)(BM * BN);
    btile_any(g, w.tm, w.tn, w.kbeg, w.kend, part, s);
    if (w.seg >= 0) barrive(g, tail, w, &last);
  }
  queue_leave(tail);
}

// conj(H) split into Re hi/lo and Im hi/lo bfloat16 planes, rows padded.
__global__ void bsplit_kernel(const double* H, int64_t lda, int64_t N, uint16_t* P, int64_t ldp,
                              int64_t plane_stride) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = blockIdx.y;
  if (k >= ldp) return;
  float re = 0.f, im = 0.f;
  double dre = 0.0, dim = 0.0;
  if (k < N) {
    dre = H[2 * (k + m * lda)];
    dim = -H[2 * (k + m * lda) + 1];
    re = (float)dre;
    im = (float)dim;
  }
  const uint32_t rh = bf16_bits(re), ih = bf16_bits(im);
  const uint32_t rl = bf16_bits((float)(dre - (double)bf16_value(rh)));
  const uint32_t il = bf16_bits((float)(dim - (double)bf16_value(ih)));
  const int64_t o = m * ldp + k;
  P[o] = (uint16_t)rh;
  P[plane_stride + o] = (uint16_t)rl;
  P[2 * plane_stride + o] = (uint16_t)ih;
  P[3 * plane_stride + o] = (uint16_t)il;
}

// The four planes of a complex64 block (rows padded with zeros to ldxp).
__global__ void bsplit_x_kernel(const cv* X, int64_t ldx, int64_t rows, uint16_t* Xp, int64_t ldxp, int64_t xps) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = blockIdx.y;
  if (k >= ldxp) return;
  const cv v = k < rows ? X[k + n * ldx] : cv{0.f, 0.f};
  const uint32_t a = bf16_bits(v.re), b = bf16_bits(v.im);
  uint16_t* q = Xp + n * ldxp + k;
  q[0] = (uint16_t)a;
  q[xps] = (uint16_t)bf16_bits(v.re - bf16_value(a));
  q[2 * xps] = (uint16_t)b;
  q[3 * xps] = (uint16_t)bf16_bits(v.im - bf16_value(b));
}

static int cu_count_b() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

}  // namespace

int64_t bsplit_ld(int64_t N) { return cdiv(N, BK) * BK; }

int bsplit_planes(const z64* H, int64_t lda, int64_t N, uint16_t* P, hipStream_t s) {
  const int64_t ldp = bsplit_ld(N);
  hipLaunchKernelGGL(bsplit_kernel, dim3((unsigned)cdiv(ldp, 256), (unsigned)N), dim3(256), 0, s,
                     reinterpret_cast<const double*>(H), lda, N, P, ldp, ldp * N);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int bsplit_block(const c32* X, int64_t ldx, int64_t rows, int64_t ncols, uint16_t* Xp, int64_t ldxp, int64_t xps,
                 hipStream_t s) {
  if (ncols <= 0) return kOk;
  if (ldxp < rows || ldxp % BK) return -1;
  hipLaunchKernelGGL(bsplit_x_kernel, dim3((unsigned)cdiv(ldxp, 256), (unsigned)ncols), dim3(256), 0, s,
                     reinterpret_cast<const cv*>(X), ldx, rows, Xp, ldxp, xps);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int bfilter_launch(const BGemmArgs& g, hipStream_t s, void* tail_ws, int* tail_counters) {
  if (g.M <= 0 || g.N <= 0) return kOk;
  if (!tail_ws || !tail_counters) return -1;
  // 16-byte DMA lanes: plane rows / columns padded to whole K tiles, aligned
  if (!g.Xp || !g.Yp || g.ldp % BK || g.ldxp % BK || g.ldxp < g.K || g.ldp < g.K ||
      reinterpret_cast<uintptr_t>(g.P) % 16 || reinterpret_cast<uintptr_t>(g.Xp) % 16 || g.plane_stride % 8 ||
      g.xps % 8)
    return -1;
  TileGeom geo;  // 8 waves of 64 x 32: wave w at (w & 1, w >> 1)
  geo.M = g.M; geo.N = g.N; geo.bm = BM; geo.bn = BN; geo.wgm = 2; geo.wgn = 4;
  TailSplit t;
  const int64_t grid = plan_schedule(geo, cdiv(g.K, BK), cu_count_b(), 8, true, tail_ws, tail_counters, &t);
  hipLaunchKernelGGL(bfilter_step, dim3((unsigned)grid), dim3(NT), 0, s, g, t);
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
