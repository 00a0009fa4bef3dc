// Backward of the eigenvalue loss: G = X diag(s) X^H (N x N, complex FP64;
// X is N x K with K = nev), the adjoint of the eigenvalues through the
// eigenvectors (gradient of sum_i s_i lambda_i with respect to H).
//
// It is the filter's tile schedule turned around: both operands are columns
// of X read straight into LDS with global_load_lds_dwordx4 (one instruction
// moves 64 consecutive rows of one column), stored [k][row] with 2 KB per k
// row on both sides, so the X^H side needs no transposed load: a fragment
// read of 16 consecutive columns of X^H at one k is one 256-byte run of row k.
// Conjugation and the scale s_k are applied as the B fragment is read; the K
// slice of s sits in LDS beside the operand tiles.  K-tile 16, two LDS stages,
// 8 waves of 64 x 32 on a 128 x 128 tile, MFMA V_MFMA_F64_16X16X4_F64 (four
// real products per complex one).  The two waves that share a SIMD (w, w + 4)
// issue their loads at different K-substeps.
//
// The tiles are uniform, so one workgroup per tile (XCD-major) is enough; with
// the lower triangle requested only tiles that hold an element on or below
// the diagonal are launched.
#include "common.hpp"
#include "kernels.hpp"

namespace chase {

namespace {

struct alignas(16) gz {
  double re, im;
};

constexpr int BM = 128, BN = 128, BK = 16, NT = 512;
constexpr int WGM = 2, WGN = 4, TM = 4, TN = 2;
constexpr int ROW = 128 * 16;            // one k row of a 128-row operand tile
constexpr int OP_BYTES = BK * ROW;       // one operand tile
constexpr int S_OFF = 2 * OP_BYTES;      // the K slice of s
constexpr int STAGE = 2 * OP_BYTES + BK * 8;

// Loads of K-tile [k0, k0 + 16) of rows r0 .. r0 + 127 of X into `dst`: 32
// instructions, 4 per wave.  Rows beyond `rows` are not loaded (they only
// reach discarded outputs); k beyond kend is written as zero.
template <bool EDGE>
__device__ __forceinline__ void zg_issue_side(const gz* X, int64_t ldx, int64_t rows, int64_t r0, int64_t k0,
                                              int64_t kend, unsigned char* dst0, int wave, int lane) {
  const bool kfull = k0 + BK <= kend;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ia = wave * 4 + r;
    const int kr = ia >> 1, half = ia & 1;
    const int64_t k = k0 + kr;
    unsigned char* dst = dst0 + kr * ROW + half * 1024;
    const int64_t m = r0 + half * 64 + lane;
    if (kfull || k < kend) {
      if (!EDGE || m < rows) __builtin_amdgcn_global_load_lds(X + m + k * ldx, dst, 16, 0, 0);
    } else {
      reinterpret_cast<gz*>(dst)[lane] = gz{0.0, 0.0};
    }
  }
}

template <bool EDGE>
__device__ __forceinline__ void zg_tile(const GemmArgs& g, int64_t tm, int64_t tn, unsigned char* lds) {
  const gz* A = reinterpret_cast<const gz*>(g.A);
  const gz* B = reinterpret_cast<const gz*>(g.B);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave % WGM, wn = wave / WGM;
  const int l16 = lane & 15, kq = lane >> 4;
  const bool active = !EDGE || (m0 + wm * TM * 16 < g.M && n0 + wn * TN * 16 < g.N);
  const int issue_at = wave < 4 ? 0 : 2;
  f64x4 cr[TN][TM], ci[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      cr[a][b] = f64x4{0, 0, 0, 0};
      ci[a][b] = f64x4{0, 0, 0, 0};
    }
  const int64_t K = g.K;
  const int64_t nkt = (K + BK - 1) / BK;
  // the K slice of s for the next stage: wave 0, lanes 0..15 (one value each)
  const bool s_lane = wave == 0 && lane < BK;
  double s_next = 0.0;
  if (nkt > 0) {
    zg_issue_side<EDGE>(A, g.lda, g.M, m0, 0, K, lds, wave, lane);
    zg_issue_side<EDGE>(B, g.ldb, g.N, n0, 0, K, lds + OP_BYTES, wave, lane);
    if (s_lane) reinterpret_cast<double*>(lds + S_OFF)[lane] = lane < K ? g.bscale[lane] : 0.0;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const unsigned char* cur = lds + (kt & 1) * STAGE;
    unsigned char* nxt = lds + ((kt + 1) & 1) * STAGE;
    const int64_t k1 = (kt + 1) * BK;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      if (ks == issue_at && kt + 1 < nkt) {
        zg_issue_side<EDGE>(A, g.lda, g.M, m0, k1, K, nxt, wave, lane);
        zg_issue_side<EDGE>(B, g.ldb, g.N, n0, k1, K, nxt + OP_BYTES, wave, lane);
        if (s_lane) s_next = k1 + lane < K ? g.bscale[k1 + lane] : 0.0;
      }
      if (!active) continue;
      const int kk = ks * 4 + kq;
      const double sk = reinterpret_cast<const double*>(cur + S_OFF)[kk];
      double br[TN], bi[TN], ar[TM], ai[TM];
#pragma unroll
      for (int j = 0; j < TN; ++j) {  // B = diag(s) X^H: conjugate and scale
        const int n = wn * TN * 16 + j * 16 + l16;
        const gz v = *reinterpret_cast<const gz*>(cur + OP_BYTES + kk * ROW + (n << 4));
        br[j] = v.re * sk;
        bi[j] = -v.im * sk;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int m = wm * TM * 16 + i * 16 + l16;
        const gz v = *reinterpret_cast<const gz*>(cur + kk * ROW + (m << 4));
        ar[i] = v.re;
        ai[i] = v.im;
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
    // stage kt + 1 was last read before the previous barrier
    if (s_lane && kt + 1 < nkt) reinterpret_cast<double*>(nxt + S_OFF)[lane] = s_next;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  // accumulator layout on gfx950: lane l, element r holds row l/16 + 4 r
  // (the output column) and column l % 16 (the output row)
  gz* Y = reinterpret_cast<gz*>(g.Y);
#pragma unroll
  for (int nb = 0; nb < TN; ++nb)
#pragma unroll
    for (int mb = 0; mb < TM; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * TN * 16 + nb * 16 + kq + 4 * r;
        const int64_t m = m0 + wm * TM * 16 + mb * 16 + l16;
        if (m >= g.M || n >= g.N) continue;
        Y[m + n * g.ldy] = gz{g.alpha * cr[nb][mb][r], g.alpha * ci[nb][mb][r]};
      }
}

// Tile of workgroup blockIdx.x (XCD-major); lower: tiles with tn <= tm only.
__device__ __forceinline__ bool zg_map(const GemmArgs& g, int64_t* tm, int64_t* tn) {
  const int64_t tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const int64_t ntiles = g.lower_only ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
  const int64_t bid = blockIdx.x;
  const int64_t per = (ntiles + 7) / 8;
  const int64_t tile = (bid % 8) * per + bid / 8;
  if (tile >= ntiles) return false;
  if (!g.lower_only) {
    *tm = tile / tiles_n;
    *tn = tile % tiles_n;
    return true;
  }
  // tile = tm (tm + 1) / 2 + tn, 0 <= tn <= tm
  int64_t r = (int64_t)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > tile) --r;
  while ((r + 1) * (r + 2) / 2 <= tile) ++r;
  *tm = r;
  *tn = tile - r * (r + 1) / 2;
  return true;
}

__global__ __launch_bounds__(NT, 1) void zgrad_nc(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];
  int64_t tm, tn;
  if (!zg_map(g, &tm, &tn)) return;
  if ((tm + 1) * BM <= g.M && (tn + 1) * BN <= g.N)
    zg_tile<false>(g, tm, tn, lds);
  else
    zg_tile<true>(g, tm, tn, lds);
}

}  // namespace

int zgrad_launch(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return kOk;
  if (!g.bscale || g.lower_only && g.M != g.N) return -1;
  const int64_t tiles_m = cdiv(g.M, BM), tiles_n = cdiv(g.N, BN);
  const int64_t ntiles = g.lower_only ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
  hipLaunchKernelGGL(zgrad_nc, dim3((unsigned)(8 * cdiv(ntiles, 8))), dim3(NT), 0, s, g);
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
