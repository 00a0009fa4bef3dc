// Complex FP32 filter step on the gfx950 matrix cores (mixed precision):
//
//   Y = alpha * H X + beta * Y + gamma * X          (complex64, FP32 accumulate)
//
// Same tiling as the FP64 kernel (128 x 64 complex per workgroup, K step 16,
// four waves of 64 x 32, XCD-major tile order), built on
// V_MFMA_F32_16X16X4_F32.  Its accumulator layout on gfx950 (measured) is the
// usual one: lane l, element r holds row 4 (l/16) + r, column l % 16.  As in
// the FP64 kernel the MFMA row index is bound to the output column n and the
// column index to the output row m, so epilogue accesses are contiguous runs
// of 16 rows.
#include "common.hpp"
#include "kernels.hpp"

namespace chase {

namespace {

constexpr int BM = 128;
constexpr int BN = 64;
constexpr int BK = 16;
constexpr int NT = 256;
constexpr int APAD = BM + 1;
constexpr int BPAD = BN + 1;

struct alignas(8) cv {
  float re, im;
};

__device__ __forceinline__ bool map_tile(int64_t ntiles, int64_t tiles_n, int64_t& tm, int64_t& tn) {
  int64_t bid = blockIdx.x;
  int64_t per = (ntiles + 7) / 8;
  int64_t tile = (bid % 8) * per + bid / 8;
  if (tile >= ntiles) return false;
  tm = tile / tiles_n;
  tn = tile % tiles_n;
  return true;
}

__global__ __launch_bounds__(NT, 2) void cfilter_step(CGemmArgs g) {
  __shared__ float As[2][BK][APAD];
  __shared__ float Bs[2][BK][BPAD];

  const int64_t tiles_m = (g.M + BM - 1) / BM;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  int64_t tm, tn;
  if (!map_tile(tiles_m * tiles_n, tiles_n, tm, tn)) return;
  const int64_t m0 = tm * BM;
  const int64_t n0 = tn * BN;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave & 1;
  const int wn = wave >> 1;

  f32x4 acc_re[2][4], acc_im[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc_re[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc_im[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  const cv* Ap = reinterpret_cast<const cv*>(g.A);
  const cv* Bp = reinterpret_cast<const cv*>(g.B);
  cv ra[8], rb[4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int e = t + NT * r;
      int mm = e % BM, kk = e / BM;
      int64_t m = m0 + mm, k = k0 + kk;
      ra[r] = (m < g.M && k < g.K) ? Ap[m + k * g.lda] : cv{0.f, 0.f};
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int e = t + NT * r;
      int kk = e % BK, nn = e / BK;
      int64_t n = n0 + nn, k = k0 + kk;
      rb[r] = (n < g.N && k < g.K) ? Bp[k + n * g.ldb] : cv{0.f, 0.f};
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int e = t + NT * r;
      int mm = e % BM, kk = e / BM;
      As[0][kk][mm] = ra[r].re;
      As[1][kk][mm] = ra[r].im;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int e = t + NT * r;
      int kk = e % BK, nn = e / BK;
      Bs[0][kk][nn] = rb[r].re;
      Bs[1][kk][nn] = rb[r].im;
    }
  };

  if (g.K > 0) load(0);
  for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + BK < g.K) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      float bre[2], bim[2], are[4], aim[4];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        bre[nb] = Bs[0][kk][wn * 32 + nb * 16 + (lane & 15)];
        bim[nb] = Bs[1][kk][wn * 32 + nb * 16 + (lane & 15)];
      }
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        are[mb] = As[0][kk][wm * 64 + mb * 16 + (lane & 15)];
        aim[mb] = As[1][kk][wm * 64 + mb * 16 + (lane & 15)];
      }
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          acc_re[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bre[nb], are[mb], acc_re[nb][mb], 0, 0, 0);
          acc_im[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bre[nb], aim[mb], acc_im[nb][mb], 0, 0, 0);
        }
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          acc_re[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-bim[nb], aim[mb], acc_re[nb][mb], 0, 0, 0);
          acc_im[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bim[nb], are[mb], acc_im[nb][mb], 0, 0, 0);
        }
    }
  }

  cv* Y = reinterpret_cast<cv*>(g.Y);
  const cv* Z = reinterpret_cast<const cv*>(g.Z);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * 32 + nb * 16 + 4 * (lane >> 4) + r;
        const int64_t m = m0 + wm * 64 + mb * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        cv out;
        out.re = g.alpha * acc_re[nb][mb][r];
        out.im = g.alpha * acc_im[nb][mb][r];
        if (g.beta != 0.f) {
          cv y = Y[m + n * g.ldy];
          out.re += g.beta * y.re;
          out.im += g.beta * y.im;
        }
        if (g.gamma != 0.f) {
          cv z = Z[m + n * g.ldz];
          out.re += g.gamma * z.re;
          out.im += g.gamma * z.im;
        }
        Y[m + n * g.ldy] = out;
      }
}

}  // namespace

int cgemm_filter_launch(const CGemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return kOk;
  const int64_t tiles = cdiv(g.M, BM) * cdiv(g.N, BN);
  hipLaunchKernelGGL(cfilter_step, dim3((unsigned)(8 * cdiv(tiles, 8))), dim3(NT), 0, s, g);
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
