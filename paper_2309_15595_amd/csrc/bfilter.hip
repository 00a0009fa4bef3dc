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
//
// Tiling: 128 (m) x 128 (n) complex tile, 8 waves of 64 x 32, K tile 32 (one
// MFMA K step).  LDS holds two K tiles of the four H planes and the four X
// planes (bf16, 64-byte rows, 16-byte chunks XOR-swizzled by row so that the
// 16 lanes of a fragment read hit distinct banks): 128 KB.  The last partial
// round of tiles is split along K as in the FP64 kernel.  The MFMA row index
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


// One 128 x 128 output tile over K range [kbeg, kend) (multiples of BK, kend
// may exceed K: the planes are zero-padded and X loads are guarded).
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

  // staging registers: one 8-k chunk of each H plane for row hx_m, and 8
  // complex of X (column xn, chunk xkc); 4 consecutive threads cover a row
  uint4 rh[4];
  cv rx[8];
  const int hx_m = t / 4, hx_c = t % 4;
  const int xn = t / 4, xkc = t % 4;
  auto gload = [&](int64_t k0) {
    const int64_t m = m0 + hx_m;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const uint4* row = reinterpret_cast<const uint4*>(g.P + (int64_t)p * g.plane_stride + m * g.ldp + k0);
      rh[p] = (m < g.M) ? row[hx_c] : uint4{0, 0, 0, 0};
    }
    const int64_t n = n0 + xn;
    const cv* col = reinterpret_cast<const cv*>(g.X) + n * g.ldx + k0 + 8 * xkc;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int64_t k = k0 + 8 * xkc + v;
      rx[v] = (n < g.N && k < g.K) ? col[v] : cv{0.f, 0.f};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 4; ++p) s.h[buf][p][hx_m][swz(hx_m, hx_c)] = rh[p];
    uint32_t rh_[8], rl_[8], ih_[8], il_[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const uint32_t a = bf16_bits(rx[v].re), b = bf16_bits(rx[v].im);
      rh_[v] = a;
      rl_[v] = bf16_bits(rx[v].re - bf16_value(a));
      ih_[v] = b;
      il_[v] = bf16_bits(rx[v].im - bf16_value(b));
    }
    auto pack = [](const uint32_t* w) {
      return uint4{w[0] | (w[1] << 16), w[2] | (w[3] << 16), w[4] | (w[5] << 16), w[6] | (w[7] << 16)};
    };
    const int c = swz(xn, xkc);
    s.x[buf][0][xn][c] = pack(rh_);
    s.x[buf][1][xn][c] = pack(rl_);
    s.x[buf][2][xn][c] = pack(ih_);
    s.x[buf][3][xn][c] = pack(il_);
  };

  const int64_t nkt = (kend - kbeg) / BK;
  if (nkt > 0) {
    gload(kbeg);
    sstore(0);
    if (nkt > 1) gload(kbeg + BK);
  }
  __syncthreads();
  // Row block at which the wave stores the next K-tile and loads the one
  // after: waves w and w + 4 share a SIMD; staggering them keeps one wave's
  // store / load issue under the other's MFMAs.
  const int stage_at = wave >= 4 ? TM / 2 : 0;
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
        if (mb == stage_at && kt + 1 < nkt) {
          sstore(buf ^ 1);
          if (kt + 2 < nkt) gload(kbeg + (kt + 2) * BK);
        }
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

int bfilter_launch(const BGemmArgs& g, hipStream_t s, void* tail_ws, int* tail_counters) {
  if (g.M <= 0 || g.N <= 0) return kOk;
  if (!tail_ws || !tail_counters) return -1;
  TileGeom geo;  // 8 waves of 64 x 32: wave w at (w & 1, w >> 1)
  geo.M = g.M; geo.N = g.N; geo.bm = BM; geo.bn = BN; geo.wgm = 2; geo.wgn = 4;
  TailSplit t;
  const int64_t grid = plan_schedule(geo, cdiv(g.K, BK), cu_count_b(), 8, true, tail_ws, tail_counters, &t);
  hipLaunchKernelGGL(bfilter_step, dim3((unsigned)grid), dim3(NT), 0, s, g, t);
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
