// The Chebyshev filter step, Eq. (1): one complex FP64 GEMM of the N x N
// Hermitian H with the active block, the recurrence fused into the epilogue:
//
//   Y = alpha H X + beta Y + gamma X         (gamma = -alpha c; Y holds X_{k-1})
//
// This is the hot kernel of the solve (about 90 % of the flops), so it gets a
// schedule of its own on gfx950:
//   * a workgroup of WGM x WGN waves computes a (WGM*TM*16) x (WGN*TN*16)
//     complex tile, each wave TM x TN blocks of 16 x 16; per K-substep of 4 a
//     wave issues 4*TM*TN V_MFMA_F64_16X16X4_F64 (four real products per
//     complex one) against 2*(TM+TN) LDS fragment reads;
//   * LDS holds two K-tiles (Re/Im planes of H and X): global loads of tile
//     t+2 are in flight while tile t is multiplied and tile t+1 is stored,
//     with one barrier per K-tile;
//   * accumulators live in AGPRs;
//   * tiles are handed out XCD-major, n fastest, so the workgroups sharing a
//     row panel of H run on one XCD and reuse it from that XCD's L2.
// The MFMA row index is bound to the output column n and the column index to
// the output row m (accumulator layout on gfx950: lane l, element r holds row
// l/16 + 4 r, column l % 16), so each epilogue access is a 256-byte run of one
// column of the column-major output.
#include "common.hpp"
#include "kernels.hpp"

#ifndef ZF_CONFIG
#define ZF_CONFIG 1
#endif

namespace chase {

namespace {

struct alignas(16) zv {
  double re, im;
};

__device__ __forceinline__ bool map_tile(int64_t ntiles, int64_t tiles_n, int64_t& tm, int64_t& tn) {
  const int64_t bid = blockIdx.x;
  const int64_t per = (ntiles + 7) / 8;
  const int64_t tile = (bid % 8) * per + bid / 8;
  if (tile >= ntiles) return false;
  tm = tile / tiles_n;
  tn = tile % tiles_n;
  return true;
}

template <int WGM, int WGN, int TM, int TN, int BK>
struct Cfg {
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int BM = WGM * TM * 16;
  static constexpr int BN = WGN * TN * 16;
  static constexpr int APAD = BM + 2;
  static constexpr int BPAD = BN + 2;
  static constexpr int LA = (BM * BK) / NT;
  static constexpr int LB = (BN * BK) / NT;
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile not divisible by threads");
  static_assert(NT % BM == 0 || BM % NT == 0, "A load mapping");
};

template <class C, int BK>
struct Smem {
  double a[2][2][BK][C::APAD];  // [buffer][re/im][k][m]
  double b[2][2][BK][C::BPAD];  // [buffer][re/im][k][n]
};

template <int WGM, int WGN, int TM, int TN, int BK>
__device__ __forceinline__ void zbig_body(const GemmArgs& g) {
  using C = Cfg<WGM, WGN, TM, TN, BK>;
  constexpr int NT = C::NT, BM = C::BM, BN = C::BN, LA = C::LA, LB = C::LB;
  __shared__ Smem<C, BK> s;

  const int64_t tiles_m = (g.M + BM - 1) / BM;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  int64_t tm, tn;
  if (!map_tile(tiles_m * tiles_n, tiles_n, tm, tn)) return;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int l16 = lane & 15, kq = lane >> 4;

  f64x4 cr[TN][TM], ci[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      cr[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
      ci[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    }

  const zv* A = reinterpret_cast<const zv*>(g.A);
  const zv* B = reinterpret_cast<const zv*>(g.B);
  zv ra[LA], rb[LB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = t + NT * r;
      const int64_t m = m0 + (e % BM), k = k0 + (e / BM);
      ra[r] = (m < g.M && k < g.K) ? A[m + k * g.lda] : zv{0.0, 0.0};
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = t + NT * r;
      const int64_t k = k0 + (e % BK), n = n0 + (e / BK);
      rb[r] = (n < g.N && k < g.K) ? B[k + n * g.ldb] : zv{0.0, 0.0};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = t + NT * r;
      s.a[buf][0][e / BM][e % BM] = ra[r].re;
      s.a[buf][1][e / BM][e % BM] = ra[r].im;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = t + NT * r;
      s.b[buf][0][e % BK][e / BK] = rb[r].re;
      s.b[buf][1][e % BK][e / BK] = rb[r].im;
    }
  };

  const int64_t nkt = (g.K + BK - 1) / BK;
  if (nkt > 0) {
    gload(0);
    sstore(0);
    if (nkt > 1) gload(BK);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int buf = (int)(kt & 1);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + kq;
      double br[TN], bi[TN], ar[TM], ai[TM];
#pragma unroll
      for (int i = 0; i < TN; ++i) {
        br[i] = s.b[buf][0][kk][wn * TN * 16 + i * 16 + l16];
        bi[i] = s.b[buf][1][kk][wn * TN * 16 + i * 16 + l16];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        ar[i] = s.a[buf][0][kk][wm * TM * 16 + i * 16 + l16];
        ai[i] = s.a[buf][1][kk][wm * TM * 16 + i * 16 + l16];
      }
#pragma unroll
      for (int nb = 0; nb < TN; ++nb)
#pragma unroll
        for (int mb = 0; mb < TM; ++mb) {
          cr[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(br[nb], ar[mb], cr[nb][mb], 0, 0, 0);
          ci[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(br[nb], ai[mb], ci[nb][mb], 0, 0, 0);
        }
#pragma unroll
      for (int nb = 0; nb < TN; ++nb)
#pragma unroll
        for (int mb = 0; mb < TM; ++mb) {
          cr[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-bi[nb], ai[mb], cr[nb][mb], 0, 0, 0);
          ci[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bi[nb], ar[mb], ci[nb][mb], 0, 0, 0);
        }
    }
    if (kt + 1 < nkt) {
      sstore(buf ^ 1);
      if (kt + 2 < nkt) gload((kt + 2) * BK);
    }
    __syncthreads();
  }

  zv* Y = reinterpret_cast<zv*>(g.Y);
  const zv* Z = reinterpret_cast<const zv*>(g.Z);
#pragma unroll
  for (int nb = 0; nb < TN; ++nb)
#pragma unroll
    for (int mb = 0; mb < TM; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * TN * 16 + nb * 16 + kq + 4 * r;
        const int64_t m = m0 + wm * TM * 16 + mb * 16 + l16;
        if (m >= g.M || n >= g.N) continue;
        zv out{g.alpha * cr[nb][mb][r], g.alpha * ci[nb][mb][r]};
        if (g.beta != 0.0) {
          const zv y = Y[m + n * g.ldy];
          out.re += g.beta * y.re;
          out.im += g.beta * y.im;
        }
        if (g.gamma != 0.0) {
          const zv z = Z[m + n * g.ldz];
          out.re += g.gamma * z.re;
          out.im += g.gamma * z.im;
        }
        Y[m + n * g.ldy] = out;
      }
}

// Configuration: (waves along m, waves along n, 16-blocks per wave m, n, K tile)
#if ZF_CONFIG == 1
#define ZF_ARGS 2, 4, 4, 2, 16   // 128 x 128 tile, 8 waves of 64 x 32
#elif ZF_CONFIG == 2
#define ZF_ARGS 2, 2, 4, 2, 16   // 128 x 64 tile, 4 waves of 64 x 32
#elif ZF_CONFIG == 3
#define ZF_ARGS 4, 2, 2, 4, 16   // 128 x 128 tile, 8 waves of 32 x 64
#elif ZF_CONFIG == 4
#define ZF_ARGS 2, 4, 4, 2, 8    // 128 x 128 tile, 8 waves, K tile 8
#endif

using ZC = Cfg<ZF_ARGS>;

__global__ __launch_bounds__(ZC::NT, 1) void zfilter_step(GemmArgs g) { zbig_body<ZF_ARGS>(g); }
// Same schedule for the other large H-times-block products (Rayleigh-Ritz H C).
__global__ __launch_bounds__(ZC::NT, 1) void zgemm_nn_big(GemmArgs g) { zbig_body<ZF_ARGS>(g); }

}  // namespace

int zgemm_nn_big_launch(const GemmArgs& g, hipStream_t s, bool filter_symbol) {
  if (g.M <= 0 || g.N <= 0) return kOk;
  if (g.ws != nullptr || g.upper_b || g.lower_only || g.bscale != nullptr) return -1;
  const int64_t tiles = cdiv(g.M, ZC::BM) * cdiv(g.N, ZC::BN);
  const dim3 grid((unsigned)(8 * cdiv(tiles, 8)));
  GemmArgs a = g;
  if (a.K <= 0) a.alpha = 0.0;
  if (filter_symbol)
    hipLaunchKernelGGL(zfilter_step, grid, dim3(ZC::NT), 0, s, a);
  else
    hipLaunchKernelGGL(zgemm_nn_big, grid, dim3(ZC::NT), 0, s, a);
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
