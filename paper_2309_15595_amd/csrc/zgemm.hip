// Complex FP64 GEMM on the gfx950 matrix cores.
//
//   Y[m, n] = alpha * sum_k opA(A)[m, k] * opB(B)[k, n] + beta * Y[m, n] + gamma * Z[m, n]
//
// opX is the identity (N) or the conjugate transpose (C).  All matrices are
// column-major complex128 with leading dimensions.  This one kernel body
// serves the Chebyshev filter step (Eq. 1: Y <- alpha (H - c I) X + beta Y,
// with Z = X and gamma = -alpha c, computed in place on the X_{k-1} buffer),
// the Rayleigh-Ritz products H C and C2 W, the Gram matrices X^H X of
// CholeskyQR (split over K, reduced deterministically), X R^{-1} with an
// explicit triangular inverse, the trailing updates of the blocked Cholesky
// and the eigenvalue-gradient product X diag(g) X^H.
//
// Mapping to the hardware.  The workgroup tile is 128 (m) x 64 (n) complex
// entries with a K step of 16; four waves own 64 x 32 each.  Re/Im planes of
// both operand tiles are staged in LDS (about 49 KB, two workgroups per CU).
// V_MFMA_F64_16X16X4_F64 has no complex form, so a complex product is four
// real ones.  The MFMA "row" index is bound to n and the "column" index to m:
// the accumulator lane layout then puts 16 consecutive m of one column in 16
// consecutive lanes, so epilogue loads/stores of Y and Z are 256-byte
// contiguous runs of the column-major output.  Measured accumulator layout of
// the f64 16x16x4 MFMA on gfx950: lane l, element r holds row l/16 + 4 r,
// column l % 16.  Tiles are assigned XCD-major: the 8 XCDs each take a
// contiguous range of tiles, ordered n-fastest, so the workgroups that share
// one 128-row panel of H run on the same XCD and share it through its L2.
#include "common.hpp"
#include "kernels.hpp"

namespace chase {

namespace {

constexpr int BM = 128;
constexpr int BN = 64;
constexpr int BK = 16;
constexpr int NT = 256;
#ifndef ZGEMM_WAVES
#define ZGEMM_WAVES 1
#endif
constexpr int APAD = BM + 1;
constexpr int BPAD = BN + 1;

struct alignas(16) zv {
  double re, im;
};

template <int OPA, int OPB>
struct ZTile {
  zv ra[8];
  zv rb[4];

  __device__ __forceinline__ void load(const GemmArgs& g, int64_t m0, int64_t n0, int64_t k0,
                                       int64_t kend, int t) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int e = t + NT * r;
      int mm, kk;
      if (OPA == 0) { mm = e % BM; kk = e / BM; }
      else          { kk = e % BK; mm = e / BK; }
      int64_t m = m0 + mm, k = k0 + kk;
      zv v = {0.0, 0.0};
      if (m < g.M && k < kend) {
        const zv* p = reinterpret_cast<const zv*>(g.A);
        if (OPA == 0) v = p[m + k * g.lda];
        else { v = p[k + m * g.lda]; v.im = -v.im; }
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int e = t + NT * r;
      int nn, kk;
      if (OPB == 0) { kk = e % BK; nn = e / BK; }
      else          { nn = e % BN; kk = e / BN; }
      int64_t n = n0 + nn, k = k0 + kk;
      zv v = {0.0, 0.0};
      if (n < g.N && k < kend) {
        const zv* p = reinterpret_cast<const zv*>(g.B);
        if (OPB == 0) v = p[k + n * g.ldb];
        else { v = p[n + k * g.ldb]; v.im = -v.im; }
        if (g.bscale != nullptr) {
          const double sc = g.bscale[k];
          v.re *= sc;
          v.im *= sc;
        }
      }
      rb[r] = v;
    }
  }

  __device__ __forceinline__ void store(double (*As)[BK][APAD], double (*Bs)[BK][BPAD], int t) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int e = t + NT * r;
      int mm, kk;
      if (OPA == 0) { mm = e % BM; kk = e / BM; }
      else          { kk = e % BK; mm = e / BK; }
      As[0][kk][mm] = ra[r].re;
      As[1][kk][mm] = ra[r].im;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int e = t + NT * r;
      int nn, kk;
      if (OPB == 0) { kk = e % BK; nn = e / BK; }
      else          { nn = e % BN; kk = e / BN; }
      Bs[0][kk][nn] = rb[r].re;
      Bs[1][kk][nn] = rb[r].im;
    }
  }
};

// Linear block id -> (tile_m, tile_n), XCD-major (see header comment).
__device__ __forceinline__ bool map_tile(int64_t ntiles, int64_t tiles_n, int64_t& tm, int64_t& tn) {
  int64_t bid = blockIdx.x;
  int64_t per = (ntiles + 7) / 8;
  int64_t tile = (bid % 8) * per + bid / 8;
  if (tile >= ntiles) return false;
  tm = tile / tiles_n;
  tn = tile % tiles_n;
  return true;
}

// MODE 0: the full complex product.  MODE 1 (real_b): opB(B) is real-valued,
// so the products with its imaginary part are skipped.  MODE 2 (real_out):
// only the real part of the product is wanted; the imaginary accumulators
// are not formed (and are stored as zero).
template <int OPA, int OPB, int MODE = 0>
__device__ __forceinline__ void zgemm_body(const GemmArgs& g) {
  __shared__ double As[2][BK][APAD];
  __shared__ double Bs[2][BK][BPAD];

  const int64_t tiles_m = (g.M + BM - 1) / BM;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  int64_t tm, tn;
  if (!map_tile(tiles_m * tiles_n, tiles_n, tm, tn)) return;
  const int64_t m0 = tm * BM;
  const int64_t n0 = tn * BN;
  if (g.lower_only && m0 + BM <= n0) return;  // tile entirely above the diagonal

  int64_t kbeg = 0, kend = g.K;
  if (g.ws != nullptr) {
    kbeg = (int64_t)blockIdx.y * g.k_chunk;
    kend = kbeg + g.k_chunk < g.K ? kbeg + g.k_chunk : g.K;
  }
  if (g.upper_b && n0 + BN < kend) kend = n0 + BN;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave & 1;   // 64-row half of the tile
  const int wn = wave >> 1;  // 32-column half of the tile

  f64x4 acc_re[2][4], acc_im[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc_re[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
      acc_im[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    }

  ZTile<OPA, OPB> tile;
  if (kbeg < kend) tile.load(g, m0, n0, kbeg, kend, t);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    tile.store(As, Bs, t);
    __syncthreads();
    if (k0 + BK < kend) tile.load(g, m0, n0, k0 + BK, kend, t);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double bre[2], bim[2], are[4], aim[4];
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
          acc_re[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bre[nb], are[mb], acc_re[nb][mb], 0, 0, 0);
          if (MODE != 2)
            acc_im[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bre[nb], aim[mb], acc_im[nb][mb], 0, 0, 0);
        }
      if (MODE != 1) {
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) {
            acc_re[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-bim[nb], aim[mb], acc_re[nb][mb], 0, 0, 0);
            if (MODE != 2)
              acc_im[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bim[nb], are[mb], acc_im[nb][mb], 0, 0, 0);
          }
      }
    }
  }

  // Epilogue.  Lane l, element r: n = l/16 + 4 r (+ block), m = l % 16 (+ block).
  zv* Y = reinterpret_cast<zv*>(g.Y);
  const zv* Z = reinterpret_cast<const zv*>(g.Z);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * 32 + nb * 16 + (lane >> 4) + 4 * r;
        const int64_t m = m0 + wm * 64 + mb * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        if (g.ws != nullptr) {
          zv* w = reinterpret_cast<zv*>(g.ws) + (int64_t)blockIdx.y * g.ws_stride;
          w[m + n * g.M] = zv{acc_re[nb][mb][r], acc_im[nb][mb][r]};
          continue;
        }
        zv out;
        out.re = g.alpha * acc_re[nb][mb][r];
        out.im = g.alpha * acc_im[nb][mb][r];
        if (g.beta != 0.0) {
          zv y = Y[m + n * g.ldy];
          out.re += g.beta * y.re;
          out.im += g.beta * y.im;
        }
        if (g.gamma != 0.0) {
          zv z = Z[m + n * g.ldz];
          out.re += g.gamma * z.re;
          out.im += g.gamma * z.im;
        }
        Y[m + n * g.ldy] = out;
      }
}

__global__ __launch_bounds__(NT, ZGEMM_WAVES) void zgemm_nn(GemmArgs g) { zgemm_body<0, 0>(g); }
__global__ __launch_bounds__(NT, ZGEMM_WAVES) void zgemm_cn(GemmArgs g) { zgemm_body<1, 0>(g); }
__global__ __launch_bounds__(NT, ZGEMM_WAVES) void zgemm_nc(GemmArgs g) { zgemm_body<0, 1>(g); }
// the real symmetric variant's products (row-pair view): real-valued small
// right operands, and real parts of products of two real blocks
__global__ __launch_bounds__(NT, ZGEMM_WAVES) void zgemm_nn_rb(GemmArgs g) { zgemm_body<0, 0, 1>(g); }
__global__ __launch_bounds__(NT, ZGEMM_WAVES) void zgemm_nc_rb(GemmArgs g) { zgemm_body<0, 1, 1>(g); }
__global__ __launch_bounds__(NT, ZGEMM_WAVES) void zgemm_cn_ro(GemmArgs g) { zgemm_body<1, 0, 2>(g); }

// Sum of split-K partials (fixed order), optionally Hermitised, written to Y
// with the epilogue alpha * S + beta * Y.
__global__ void zsplitk_reduce(const zv* ws, int64_t stride, int splits, int64_t M, int64_t N,
                               zv* Y, int64_t ldy, double alpha, double beta, int hermitise) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  int64_t m = idx % M, n = idx / M;
  if (hermitise >= 2 && m < n) return;  // lower triangle only
  double sr = 0.0, si = 0.0;
  for (int s = 0; s < splits; ++s) {
    zv v = ws[s * stride + m + n * M];
    sr += v.re;
    si += v.im;
  }
  if ((hermitise == 2 && m == n) || hermitise == 3) si = 0.0;  // real diagonal / real part
  if (hermitise == 1) {  // (S + S^H) / 2, M == N
    double tr = 0.0, ti = 0.0;
    for (int s = 0; s < splits; ++s) {
      zv v = ws[s * stride + n + m * M];
      tr += v.re;
      ti += v.im;
    }
    sr = 0.5 * (sr + tr);
    si = 0.5 * (si - ti);
  }
  zv out{alpha * sr, alpha * si};
  if (beta != 0.0) {
    zv y = Y[m + n * ldy];
    out.re += beta * y.re;
    out.im += beta * y.im;
  }
  Y[m + n * ldy] = out;
}

}  // namespace

int zgemm_launch(int opa, int opb, const GemmArgs& g_in, hipStream_t stream) {
  GemmArgs g = g_in;
  if (g.M <= 0 || g.N <= 0) return kOk;
  const int64_t tiles = cdiv(g.M, BM) * cdiv(g.N, BN);
  const int64_t grid = 8 * cdiv(tiles, 8);
  dim3 blocks((unsigned)grid, 1, 1);
  if (g.K <= 0) {  // nothing to accumulate: Y = beta Y + gamma Z
    g.alpha = 0.0;
  }
  g.ws = nullptr;
  if (opa == 0 && opb == 0) {
    if (g.real_b) hipLaunchKernelGGL(zgemm_nn_rb, blocks, dim3(NT), 0, stream, g);
    else hipLaunchKernelGGL(zgemm_nn, blocks, dim3(NT), 0, stream, g);
  } else if (opa == 1 && opb == 0) {
    if (g.real_out) hipLaunchKernelGGL(zgemm_cn_ro, blocks, dim3(NT), 0, stream, g);
    else hipLaunchKernelGGL(zgemm_cn, blocks, dim3(NT), 0, stream, g);
  } else if (opa == 0 && opb == 1) {
    if (g.real_b) hipLaunchKernelGGL(zgemm_nc_rb, blocks, dim3(NT), 0, stream, g);
    else hipLaunchKernelGGL(zgemm_nc, blocks, dim3(NT), 0, stream, g);
  } else {
    return -1;
  }
  CHASE_CHK_LAUNCH();
  return kOk;
}

int64_t zgemm_splitk_workspace(int64_t M, int64_t N, int splits) {
  return (int64_t)splits * M * N;  // complex entries
}

int choose_splits(int64_t M, int64_t N, int64_t K, int max_splits, bool lower) {
  int64_t tiles = cdiv(M, BM) * cdiv(N, BN);
  if (lower) {  // tiles holding an element on or below the diagonal
    tiles = 0;
    for (int64_t n0 = 0; n0 < N; n0 += BN) tiles += cdiv(M - (n0 / BM) * BM, BM);
  }
  int64_t want = cdiv(1024, tiles);                 // aim at ~1024 workgroups
  int64_t cap = K / (4 * BK) > 1 ? K / (4 * BK) : 1; // at least 4 K-steps per split
  int64_t s = want < cap ? want : cap;
  if (s > max_splits) s = max_splits;
  if (s < 1) s = 1;
  return (int)s;
}

int zgemm_splitk(int opa, int opb, const GemmArgs& g_in, void* ws, int splits, int hermitise,
                 hipStream_t stream) {
  GemmArgs g = g_in;
  if (g.M <= 0 || g.N <= 0) return kOk;
  int64_t kchunk = cdiv(cdiv(g.K, splits), BK) * BK;
  if (kchunk <= 0) kchunk = BK;
  splits = (int)cdiv(g.K, kchunk);
  if (splits < 1) splits = 1;
  g.ws = reinterpret_cast<z64*>(ws);
  g.ws_stride = g.M * g.N;
  g.k_chunk = kchunk;
  if (hermitise >= 2) g.lower_only = 1;  // tiles wholly above the diagonal are never read
  const int64_t tiles = cdiv(g.M, BM) * cdiv(g.N, BN);
  dim3 blocks((unsigned)(8 * cdiv(tiles, 8)), (unsigned)splits, 1);
  if (opa == 1 && opb == 0) {
    if (g.real_out) hipLaunchKernelGGL(zgemm_cn_ro, blocks, dim3(NT), 0, stream, g);
    else hipLaunchKernelGGL(zgemm_cn, blocks, dim3(NT), 0, stream, g);
  } else if (opa == 0 && opb == 0) {
    if (g.real_b) hipLaunchKernelGGL(zgemm_nn_rb, blocks, dim3(NT), 0, stream, g);
    else hipLaunchKernelGGL(zgemm_nn, blocks, dim3(NT), 0, stream, g);
  } else if (opa == 0 && opb == 1) {
    if (g.real_b) hipLaunchKernelGGL(zgemm_nc_rb, blocks, dim3(NT), 0, stream, g);
    else hipLaunchKernelGGL(zgemm_nc, blocks, dim3(NT), 0, stream, g);
  } else {
    return -1;
  }
  CHASE_CHK_LAUNCH();
  const int64_t total = g.M * g.N;
  hipLaunchKernelGGL(zsplitk_reduce, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, stream,
                     reinterpret_cast<const zv*>(ws), g.ws_stride, splits, g.M, g.N,
                     reinterpret_cast<zv*>(g.Y), g.ldy, g.alpha, g.beta, hermitise);
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
