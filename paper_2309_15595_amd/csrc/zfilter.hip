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
#include "sched.hpp"


namespace chase {

namespace {

struct alignas(16) zv {
  double re, im;
};

// Precision of one filter instantiation: element and accumulator types, the
// MFMA, and the row of accumulator element r in lane group kq (16x16x4 f64:
// kq + 4 r; 16x16x4 f32: 4 kq + r, both measured on gfx950).
struct PF64 {
  using real = double;
  struct alignas(16) cplx {
    double re, im;
  };
  using acc = f64x4;
  static __device__ __forceinline__ acc mma(real a, real b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return kq + 4 * r; }
};
struct PF32 {
  using real = float;
  struct alignas(8) cplx {
    float re, im;
  };
  using acc = f32x4;
  static __device__ __forceinline__ acc mma(real a, real b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
};

template <int WGM, int WGN, int TM, int TN, int BK>
struct Cfg {
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int BK_ = BK;
  static constexpr int WGM_ = WGM, WGN_ = WGN;
  static constexpr int BM = WGM * TM * 16;
  static constexpr int BN = WGN * TN * 16;
  static constexpr int APAD = BM + 2;
  static constexpr int BPAD = BN + 2;
  static constexpr int LA = (BM * BK) / NT;
  static constexpr int LB = (BN * BK) / NT;
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile not divisible by threads");
  static_assert(NT % BM == 0 || BM % NT == 0, "A load mapping");
};

template <class P, class C, int BK>
struct Smem {
  typename P::real a[2][2][BK][C::APAD];  // [buffer][re/im][k][m]
  typename P::real b[2][2][BK][C::BPAD];  // [buffer][re/im][k][n]
};

// One BM x BN output tile (tm, tn) of g.  EDGE tiles overhang the output: a
// wave whose sub-tile lies wholly outside it skips its fragment reads and
// MFMAs (the padded columns of the last column tile are most of its work
// when n_act is small); a wave that touches the output computes its whole
// sub-tile on the zero-filled operands.  The test is one branch per K-tile on
// a wave-uniform (scalar) value: a per-block test would split the MFMA stream
// into exec-masked basic blocks and stall the matrix pipe.
//
// kbeg/kend (multiples of BK) restrict the K range; with part != nullptr the
// raw accumulator tile is stored there (tile-local, m fastest) instead of
// applying the epilogue.
template <class P, int WGM, int WGN, int TM, int TN, int BK, bool EDGE>
__device__ __forceinline__ void zbig_tile_impl(const GemmArgs& g, int64_t tm, int64_t tn, int64_t kbeg,
                                               int64_t kend, typename P::cplx* part,
                                               Smem<P, Cfg<WGM, WGN, TM, TN, BK>, BK>& s) {
  using C = Cfg<WGM, WGN, TM, TN, BK>;
  using zv = typename P::cplx;
  using real = typename P::real;
  using accv = typename P::acc;
  constexpr int NT = C::NT, BM = C::BM, BN = C::BN, LA = C::LA, LB = C::LB;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave % WGM, wn = wave / WGM;
  const int l16 = lane & 15, kq = lane >> 4;
  // does this wave's sub-tile touch the output? (wave-uniform)
  const bool active = !EDGE || (m0 + wm * TM * 16 < g.M && n0 + wn * TN * 16 < g.N);
  // K-substep at which the wave stores the next K-tile to LDS and loads the
  // one after: waves w and w + 4 of an 8-wave workgroup share a SIMD, and
  // staggering them keeps one wave's store / load issue under the other's
  // MFMAs instead of both stalling the matrix pipe after each barrier
  const int stage_at = (WGM * WGN == 8 && wave >= 4) ? BK / 8 : 0;

  accv cr[TN][TM], ci[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      cr[a][b] = accv{0, 0, 0, 0};
      ci[a][b] = accv{0, 0, 0, 0};
    }

  const zv* A = reinterpret_cast<const zv*>(g.A);
  const zv* B = reinterpret_cast<const zv*>(g.B);
  zv ra[LA], rb[LB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = t + NT * r;
      const int64_t m = m0 + (e % BM), k = k0 + (e / BM);
      ra[r] = (m < g.M && k < kend) ? A[m + k * g.lda] : zv{0, 0};
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = t + NT * r;
      const int64_t k = k0 + (e % BK), n = n0 + (e / BK);
      rb[r] = (n < g.N && k < kend) ? B[k + n * g.ldb] : zv{0, 0};
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

  const int64_t nkt = (kend - kbeg + BK - 1) / BK;
  if (nkt > 0) {
    gload(kbeg);
    sstore(0);
    if (nkt > 1) gload(kbeg + BK);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int buf = (int)(kt & 1);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      // buffer buf ^ 1 was last read before the previous barrier
      if (ks == stage_at && kt + 1 < nkt) {
        sstore(buf ^ 1);
        if (kt + 2 < nkt) gload(kbeg + (kt + 2) * BK);
      }
      if (!active) continue;
      const int kk = ks * 4 + kq;
      real br[TN], bi[TN], ar[TM], ai[TM];
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
          cr[nb][mb] = P::mma(br[nb], ar[mb], cr[nb][mb]);
          ci[nb][mb] = P::mma(br[nb], ai[mb], ci[nb][mb]);
        }
#pragma unroll
      for (int nb = 0; nb < TN; ++nb)
#pragma unroll
        for (int mb = 0; mb < TM; ++mb) {
          cr[nb][mb] = P::mma(-bi[nb], ai[mb], cr[nb][mb]);
          ci[nb][mb] = P::mma(bi[nb], ar[mb], ci[nb][mb]);
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
          const int nl = wn * TN * 16 + nb * 16 + P::row(kq, r);
          const int ml = wm * TM * 16 + mb * 16 + l16;
          part[ml + nl * BM] = zv{cr[nb][mb][r], ci[nb][mb][r]};
        }
    return;
  }
  zv* Y = reinterpret_cast<zv*>(g.Y);
  const zv* Z = reinterpret_cast<const zv*>(g.Z);
#pragma unroll
  for (int nb = 0; nb < TN; ++nb)
#pragma unroll
    for (int mb = 0; mb < TM; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * TN * 16 + nb * 16 + P::row(kq, r);
        const int64_t m = m0 + wm * TM * 16 + mb * 16 + l16;
        if (m >= g.M || n >= g.N) continue;
        const real al = (real)g.alpha, be = (real)g.beta, ga = (real)g.gamma;
        zv out{al * cr[nb][mb][r], al * ci[nb][mb][r]};
        if (g.beta != 0.0) {
          const zv y = Y[m + n * g.ldy];
          out.re += be * y.re;
          out.im += be * y.im;
        }
        if (g.gamma != 0.0) {
          const zv z = Z[m + n * g.ldz];
          out.re += ga * z.re;
          out.im += ga * z.im;
        }
        Y[m + n * g.ldy] = out;
      }
}

template <class P, int WGM, int WGN, int TM, int TN, int BK>
__device__ __forceinline__ void zbig_tile(const GemmArgs& g, int64_t tm, int64_t tn,
                                          Smem<P, Cfg<WGM, WGN, TM, TN, BK>, BK>& s, int64_t kbeg = 0,
                                          int64_t kend = -1, typename P::cplx* part = nullptr) {
  using C = Cfg<WGM, WGN, TM, TN, BK>;
  if (kend < 0) kend = g.K;
  if ((tm + 1) * C::BM <= g.M && (tn + 1) * C::BN <= g.N)
    zbig_tile_impl<P, WGM, WGN, TM, TN, BK, false>(g, tm, tn, kbeg, kend, part, s);
  else
    zbig_tile_impl<P, WGM, WGN, TM, TN, BK, true>(g, tm, tn, kbeg, kend, part, s);
}

// A segment has stored its partial product: count it in.  The last segment
// of a tile to arrive sums the partials in segment order (deterministic),
// applies the epilogue and resets the tile's counter for the next launch.
template <class P, int WGM, int WGN, int TM, int TN, int BK>
__device__ __forceinline__ void zbig_arrive(const GemmArgs& g, const TailSplit& tail, const WorkItem& w,
                                            int* last) {
  using C = Cfg<WGM, WGN, TM, TN, BK>;
  using zv = typename P::cplx;
  using real = typename P::real;
  constexpr int BM = C::BM, BN = C::BN;
  const int64_t tl = w.seg / tail.ksplit;
  const int64_t tm = w.tm, tn = w.tn;
  __threadfence();
  if (wg_fetch_add(tail.counters + tl, 1, last) != tail.ksplit - 1) return;
  __threadfence();
  const zv* parts = reinterpret_cast<const zv*>(tail.ws) + tl * tail.ksplit * (int64_t)(BM * BN);
  zv* Y = reinterpret_cast<zv*>(g.Y);
  const zv* Z = reinterpret_cast<const zv*>(g.Z);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  for (int e = threadIdx.x; e < BM * BN; e += C::NT) {
    const int64_t m = m0 + e % BM, n = n0 + e / BM;
    if (m >= g.M || n >= g.N) continue;
    real sr = 0, si = 0;
    for (int q = 0; q < tail.ksplit; ++q) {
      const zv v = parts[q * (int64_t)(BM * BN) + e];
      sr += v.re;
      si += v.im;
    }
    const real al = (real)g.alpha, be = (real)g.beta, ga = (real)g.gamma;
    zv out{al * sr, al * si};
    if (g.beta != 0.0) {
      const zv y = Y[m + n * g.ldy];
      out.re += be * y.re;
      out.im += be * y.im;
    }
    if (g.gamma != 0.0) {
      const zv z = Z[m + n * g.ldz];
      out.re += ga * z.re;
      out.im += ga * z.im;
    }
    Y[m + n * g.ldy] = out;
  }
  if (threadIdx.x == 0) tail.counters[tl] = 0;
}

// Whole launch: a persistent grid takes whole tiles and tail segments from
// the per-XCD work queue (sched.hpp) until its XCD's share is done.
template <class P, int WGM, int WGN, int TM, int TN, int BK>
__device__ __forceinline__ void zbig_body(const GemmArgs& g, const TailSplit& tail) {
  using C = Cfg<WGM, WGN, TM, TN, BK>;
  using zv = typename P::cplx;
  constexpr int BM = C::BM, BN = C::BN;
  __shared__ Smem<P, C, BK> s;
  __shared__ int last, item;
  const TileOrder o = tile_order(g.M, g.N, BM, BN);
  const QueueShare q = queue_share(tail, o);
  for (int64_t i; (i = queue_next(tail, q, &item)) >= 0;) {
    const WorkItem w = work_item(tail, o, i, g.K, BK);
    zv* part = w.seg < 0 ? nullptr : reinterpret_cast<zv*>(tail.ws) + w.seg * (int64_t)(BM * BN);
    zbig_tile<P, WGM, WGN, TM, TN, BK>(g, w.tm, w.tn, s, w.kbeg, w.kend, part);
    if (w.seg >= 0) zbig_arrive<P, WGM, WGN, TM, TN, BK>(g, tail, w, &last);
  }
  queue_leave(tail);
}

// ---------------------------------------------------------------------------
// FP64 step with direct-to-LDS operand loads.
//
// global_load_lds_dwordx4 moves each lane's 16 bytes (one complex128) from
// any global address straight to LDS at base + 16 * lane, so the operands
// need no staging registers and the loads leave the waves' instruction
// stream almost empty; the freed registers buy a K-tile of 16 (half the
// barriers of the staged schedule) with two LDS stages of 64 KB.
//   H: [k][m], 2 KB per k row; one instruction moves 64 consecutive rows of
//      one column of H (coalesced), a fragment read (16 lanes, consecutive
//      m, one k) is one 256-byte run.
//   X: [n][k ^ (n & 15)], 256 B per column; one instruction moves 16 k of
//      each of 4 columns (coalesced, permuted inside the 256-byte run), and
//      the XOR makes the 16 lanes of a fragment read (consecutive n, one k)
//      hit 16 different 16-byte bank groups.
// Complex values stay interleaved: one 16-byte LDS read yields both the
// real and the imaginary operand of a lane.  Rows of H beyond M and columns
// of X beyond N are not loaded (they only reach discarded outputs); k beyond
// the K range is written as zero.
// ---------------------------------------------------------------------------
namespace dz {
constexpr int BM = 128, BN = 128, BK = 16, NT = 512;
constexpr int WGM = 2, WGN = 4, TM = 4, TN = 2;
constexpr int A_BYTES = BK * BM * 16;
constexpr int B_BYTES = BN * BK * 16;
constexpr int STAGE = A_BYTES + B_BYTES;
// real B operand (RB): 8 chunks of two consecutive k (16 bytes) per column
constexpr int RB_COL = BK * 8;
}  // namespace dz

// Loads of K-tile [k0, k0 + 16) of tile (m0, n0) into `stage`: 64
// instructions, 8 per wave (48, 6 per wave, with a real B operand).
//
// RB: B is a real K x n block and A the complex view of a real matrix whose
// row pairs (2 m', 2 m' + 1) are the real and imaginary parts of complex row
// m' (the same memory).  Then complex row m' of A B holds rows 2 m' and
// 2 m' + 1 of the real product, so the complex tile computes a real GEMM of
// twice the rows with two real MFMA products per complex-by-real one, none of
// them wasted.  The B tile is [n][chunk position] with 8 chunks of two
// consecutive k (16 bytes) per column; chunk c of column n sits at position
// c ^ ((n >> 1) & 7), so 16 consecutive columns reading the same chunk hit
// 16 distinct pairs of banks.  One instruction moves 8 columns.  K and kend
// must be even (a chunk never straddles kend).
template <bool EDGE, bool RB>
__device__ __forceinline__ void dz_issue(const GemmArgs& g, int64_t m0, int64_t n0, int64_t k0, int64_t kend,
                                         unsigned char* stage, int wave, int lane) {
  using namespace dz;
  const zv* A = reinterpret_cast<const zv*>(g.A);
  const zv* B = reinterpret_cast<const zv*>(g.B);
  const bool kfull = k0 + BK <= kend;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ia = wave * 4 + r;  // k row ia / 2, rows 64 * (ia % 2) ..
    const int kr = ia >> 1, half = ia & 1;
    const int64_t k = k0 + kr;
    unsigned char* dst = stage + kr * (BM * 16) + half * 1024;
    const int64_t m = m0 + half * 64 + lane;
    if (kfull || k < kend) {
      if (!EDGE || m < g.M) __builtin_amdgcn_global_load_lds(A + m + k * g.lda, dst, 16, 0, 0);
    } else {
      reinterpret_cast<zv*>(dst)[lane] = zv{0.0, 0.0};
    }
  }
  if constexpr (RB) {
    const double* Br = reinterpret_cast<const double*>(g.B);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int ib = wave * 2 + r;  // columns 8 ib .. 8 ib + 7
      const int nl = ib * 8 + (lane >> 3);
      const int c = (lane & 7) ^ ((nl >> 1) & 7);  // chunk stored at position lane & 7
      const int64_t n = n0 + nl, k = k0 + 2 * c;
      unsigned char* dst = stage + A_BYTES + ib * 1024;
      if (kfull || k < kend) {
        if (!EDGE || n < g.N) __builtin_amdgcn_global_load_lds(Br + k + n * g.ldb, dst, 16, 0, 0);
      } else {
        reinterpret_cast<zv*>(dst)[lane] = zv{0.0, 0.0};
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ib = wave * 4 + r;  // columns 4 ib .. 4 ib + 3
      const int nl = ib * 4 + (lane >> 4);
      const int kl = (lane & 15) ^ (nl & 15);
      const int64_t n = n0 + nl, k = k0 + kl;
      unsigned char* dst = stage + A_BYTES + ib * 1024;
      if (kfull || k < kend) {
        if (!EDGE || n < g.N) __builtin_amdgcn_global_load_lds(B + k + n * g.ldb, dst, 16, 0, 0);
      } else {
        reinterpret_cast<zv*>(dst)[lane] = zv{0.0, 0.0};
      }
    }
  }
}

// Wave layout: LWGM waves along m of LTM 16-row blocks each, 8 / LWGM waves
// along n of two 16-column blocks each.  The main layout is 2 x 4 waves of
// 64 x 32.  A last column tile with at most 32 live columns uses 8 x 1 waves
// of 16 x 32, which puts two busy waves on every SIMD (a quarter of a tile's
// time) instead of one busy wave on two SIMDs (half of it); one with at most
// 64 uses 4 x 2 waves of 32 x 32 (half a tile, with two busy waves per SIMD to
// cover each other's LDS and barrier waits instead of one).
template <bool EDGE, int LWGM, int LTM, bool RB>
__device__ __forceinline__ void zdma_tile_impl(const GemmArgs& g, int64_t tm, int64_t tn, int64_t kbeg, int64_t kend,
                                               zv* part, unsigned char* lds) {
  using dz::BM;
  using dz::BN;
  using dz::BK;
  using dz::A_BYTES;
  using dz::STAGE;
  constexpr int WGM = LWGM, TM = LTM, WGN = 8 / LWGM, TN = 2;
  static_assert(WGM * TM * 16 == BM && WGN * TN * 16 <= BN, "wave layout");
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
  const int64_t nkt = (kend - kbeg + BK - 1) / BK;
  if (nkt > 0) dz_issue<EDGE, RB>(g, m0, n0, kbeg, kend, lds, wave, lane);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const unsigned char* cur = lds + (kt & 1) * STAGE;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      // waves w and w + 4 share a SIMD: the first issues its loads before
      // K-substep 0, the second before substep 2, so one wave's load issue
      // always overlaps the other's MFMAs
      if (ks == issue_at && kt + 1 < nkt)
        dz_issue<EDGE, RB>(g, m0, n0, kbeg + (kt + 1) * BK, kend, lds + ((kt + 1) & 1) * STAGE, wave, lane);
      if (!active) continue;
      if constexpr (RB) {
        // lane group kq takes k = 2 c + e, c = kq + 4 (ks / 2), e = ks % 2:
        // each k of the tile once, the two halves of a chunk in consecutive
        // substeps
        const int c = kq + 4 * (ks >> 1), e = ks & 1;
        const int kk = 2 * c + e;
        double x[TN], ar[TM], ai[TM];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int n = wn * TN * 16 + j * 16 + l16;
          x[j] = *reinterpret_cast<const double*>(cur + A_BYTES + n * dz::RB_COL + ((c ^ ((n >> 1) & 7)) << 4) +
                                                  e * 8);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const int m = wm * TM * 16 + i * 16 + l16;
          const zv v = *reinterpret_cast<const zv*>(cur + kk * (BM * 16) + (m << 4));
          ar[i] = v.re;
          ai[i] = v.im;
        }
#pragma unroll
        for (int nb = 0; nb < TN; ++nb)
#pragma unroll
          for (int mb = 0; mb < TM; ++mb) {
            cr[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[nb], ar[mb], cr[nb][mb], 0, 0, 0);
            ci[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[nb], ai[mb], ci[nb][mb], 0, 0, 0);
          }
        continue;
      }
      const int kk = ks * 4 + kq;
      double br[TN], bi[TN], ar[TM], ai[TM];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn * TN * 16 + j * 16 + l16;
        const zv v = *reinterpret_cast<const zv*>(cur + A_BYTES + n * (BK * 16) + ((kk ^ (n & 15)) << 4));
        br[j] = v.re;
        bi[j] = v.im;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int m = wm * TM * 16 + i * 16 + l16;
        const zv v = *reinterpret_cast<const zv*>(cur + kk * (BM * 16) + (m << 4));
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
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next K-tile have landed
    __syncthreads();
  }

  if (part != nullptr) {
#pragma unroll
    for (int nb = 0; nb < TN; ++nb)
#pragma unroll
      for (int mb = 0; mb < TM; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int nl = wn * TN * 16 + nb * 16 + PF64::row(kq, r);
          const int ml = wm * TM * 16 + mb * 16 + l16;
          part[ml + nl * BM] = zv{cr[nb][mb][r], ci[nb][mb][r]};
        }
    return;
  }
  zv* Y = reinterpret_cast<zv*>(g.Y);
  const zv* Z = reinterpret_cast<const zv*>(g.Z);
#pragma unroll
  for (int nb = 0; nb < TN; ++nb)
#pragma unroll
    for (int mb = 0; mb < TM; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * TN * 16 + nb * 16 + PF64::row(kq, r);
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

// One tile (or K range of one) in the layout its live region calls for.
template <bool RB>
__device__ __forceinline__ void zdma_tile(const GemmArgs& g, int64_t tm, int64_t tn, int64_t kbeg, int64_t kend,
                                          zv* part, unsigned char* lds) {
  using namespace dz;
  if ((tm + 1) * BM <= g.M && (tn + 1) * BN <= g.N)
    zdma_tile_impl<false, WGM, TM, RB>(g, tm, tn, kbeg, kend, part, lds);
  else if (g.N - tn * BN <= 32)
    zdma_tile_impl<true, 8, 1, RB>(g, tm, tn, kbeg, kend, part, lds);
  else if (g.N - tn * BN <= 64)
    zdma_tile_impl<true, 4, 2, RB>(g, tm, tn, kbeg, kend, part, lds);
  else
    zdma_tile_impl<true, WGM, TM, RB>(g, tm, tn, kbeg, kend, part, lds);
}

// Whole launch of the direct-to-LDS step on the per-XCD work queue.
template <bool RB>
__device__ __forceinline__ void zdma_body(const GemmArgs& g, const TailSplit& tail) {
  using namespace dz;
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];
  __shared__ int last, item;
  const TileOrder o = tile_order(g.M, g.N, BM, BN);
  const QueueShare q = queue_share(tail, o);
  for (int64_t i; (i = queue_next(tail, q, &item)) >= 0;) {
    const WorkItem w = work_item(tail, o, i, g.K, BK);
    zv* part = w.seg < 0 ? nullptr : reinterpret_cast<zv*>(tail.ws) + w.seg * (int64_t)(BM * BN);
    zdma_tile<RB>(g, w.tm, w.tn, w.kbeg, w.kend, part, lds);
    if (w.seg >= 0) zbig_arrive<PF64, WGM, WGN, TM, TN, BK>(g, tail, w, &last);
  }
  queue_leave(tail);
}

// Grouped, persistent form for many problems at once: row `step` of the
// descriptor table lists one GEMM per problem with its tile count as a running
// prefix sum.  A fixed grid (a multiple of 8 workgroups) walks the tiles
// XCD-major; every parameter comes from device memory, so a captured graph
// of these launches stays valid while degrees, columns and scalars change.
template <int WGM, int WGN, int TM, int TN, int BK>
__device__ __forceinline__ void zbig_grouped(const GroupEntry* __restrict__ table, int count, int step) {
  using C = Cfg<WGM, WGN, TM, TN, BK>;
  __shared__ Smem<PF64, C, BK> s;
  const GroupEntry* __restrict__ row = table + (int64_t)step * count;
  const int64_t total = row[count - 1].tile_end;
  if (total <= 0) return;
  const int64_t xcd = blockIdx.x % 8, slot = blockIdx.x / 8, slots = gridDim.x / 8;
  const int64_t per = (total + 7) / 8;
  int p = 0;
  for (int64_t i = slot; i < per; i += slots) {
    const int64_t t = xcd * per + i;
    if (t >= total) break;
    while (row[p].tile_end <= t) ++p;   // tiles are visited in increasing order
    p = __builtin_amdgcn_readfirstlane(p);  // uniform: entry fields go to SGPRs
    const int64_t begin = p > 0 ? row[p - 1].tile_end : 0;
    const int64_t lt = t - begin;
    const GemmArgs g = row[p].g;
    const int64_t tiles_n = row[p].tiles_n;
    zbig_tile<PF64, WGM, WGN, TM, TN, BK>(g, lt / tiles_n, lt % tiles_n, s);
  }
}

// ---------------------------------------------------------------------------
// FP32 step (mixed precision) with direct-to-LDS operand loads: the FP64
// schedule on complex64 data.  One 16-byte DMA lane carries two complex64
// values, so
//   H: [k][m], 1 KB per k row; one instruction moves the 128 rows of one
//      column of H (two rows per lane);
//   X: [n][chunk ^ (n mod 16)] in 16-byte chunks of two consecutive k, 256 B
//      per column (K-tile 32); one instruction moves 4 columns.
// The pairs never straddle the end of a row range or of K when M, K, the
// leading dimensions and every segment boundary are even and the operands
// 16-byte aligned; the launcher checks this and otherwise runs the staged
// FP32 kernel.  k beyond the K range is written as zero.
// ---------------------------------------------------------------------------
namespace dc {
constexpr int BM = 128, BN = 128, BK = 32, NT = 512;
constexpr int WGM = 2, WGN = 4, TM = 4, TN = 2;
constexpr int A_ROW = BM * 8;
constexpr int A_BYTES = BK * A_ROW;
constexpr int B_COL = BK * 8;
constexpr int B_BYTES = BN * B_COL;
constexpr int STAGE = A_BYTES + B_BYTES;
}  // namespace dc

template <bool EDGE>
__device__ __forceinline__ void dc_issue(const GemmArgs& g, int64_t m0, int64_t n0, int64_t k0, int64_t kend,
                                         unsigned char* stage, int wave, int lane) {
  using namespace dc;
  using cv = PF32::cplx;
  const cv* A = reinterpret_cast<const cv*>(g.A);
  const cv* B = reinterpret_cast<const cv*>(g.B);
  const bool kfull = k0 + BK <= kend;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int kr = wave * 4 + r;  // one k row of 128 rows of H
    const int64_t k = k0 + kr;
    unsigned char* dst = stage + kr * A_ROW;
    const int64_t m = m0 + 2 * lane;
    if (kfull || k < kend) {
      if (!EDGE || m < g.M) __builtin_amdgcn_global_load_lds(A + m + k * g.lda, dst, 16, 0, 0);
    } else {
      reinterpret_cast<uint4*>(dst)[lane] = uint4{0u, 0u, 0u, 0u};
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ib = wave * 4 + r;  // columns 4 ib .. 4 ib + 3
    const int nl = ib * 4 + (lane >> 4);
    const int c = (lane & 15) ^ (nl & 15);  // chunk of k pair 2c, 2c + 1
    const int64_t n = n0 + nl, k = k0 + 2 * c;
    unsigned char* dst = stage + A_BYTES + ib * 1024;
    if (kfull || k < kend) {
      if (!EDGE || n < g.N) __builtin_amdgcn_global_load_lds(B + k + n * g.ldb, dst, 16, 0, 0);
    } else {
      reinterpret_cast<uint4*>(dst)[lane] = uint4{0u, 0u, 0u, 0u};
    }
  }
}

template <bool EDGE>
__device__ __forceinline__ void cdma_tile_impl(const GemmArgs& g, int64_t tm, int64_t tn, int64_t kbeg, int64_t kend,
                                               PF32::cplx* part, unsigned char* lds) {
  using namespace dc;
  using cv = PF32::cplx;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave % WGM, wn = wave / WGM;
  const int l16 = lane & 15, kq = lane >> 4;
  const bool active = !EDGE || (m0 + wm * TM * 16 < g.M && n0 + wn * TN * 16 < g.N);
  const int issue_at = wave < 4 ? 0 : BK / 8;  // waves w and w + 4 share a SIMD
  f32x4 cr[TN][TM], ci[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      cr[a][b] = f32x4{0, 0, 0, 0};
      ci[a][b] = f32x4{0, 0, 0, 0};
    }
  const int64_t nkt = (kend - kbeg + BK - 1) / BK;
  if (nkt > 0) dc_issue<EDGE>(g, m0, n0, kbeg, kend, lds, wave, lane);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const unsigned char* cur = lds + (kt & 1) * STAGE;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      if (ks == issue_at && kt + 1 < nkt)
        dc_issue<EDGE>(g, m0, n0, kbeg + (kt + 1) * BK, kend, lds + ((kt + 1) & 1) * STAGE, wave, lane);
      if (!active) continue;
      const int kk = ks * 4 + kq;
      float br[TN], bi[TN], ar[TM], ai[TM];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn * TN * 16 + j * 16 + l16;
        const cv v = *reinterpret_cast<const cv*>(cur + A_BYTES + n * B_COL + (((kk >> 1) ^ (n & 15)) << 4) +
                                                  ((kk & 1) << 3));
        br[j] = v.re;
        bi[j] = v.im;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int m = wm * TM * 16 + i * 16 + l16;
        const cv v = *reinterpret_cast<const cv*>(cur + kk * A_ROW + (m << 3));
        ar[i] = v.re;
        ai[i] = v.im;
      }
#pragma unroll
      for (int nb = 0; nb < TN; ++nb)
#pragma unroll
        for (int mb = 0; mb < TM; ++mb) {
          cr[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(br[nb], ar[mb], cr[nb][mb], 0, 0, 0);
          ci[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(br[nb], ai[mb], ci[nb][mb], 0, 0, 0);
        }
#pragma unroll
      for (int nb = 0; nb < TN; ++nb)
#pragma unroll
        for (int mb = 0; mb < TM; ++mb) {
          cr[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-bi[nb], ai[mb], cr[nb][mb], 0, 0, 0);
          ci[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bi[nb], ar[mb], ci[nb][mb], 0, 0, 0);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next K-tile have landed
    __syncthreads();
  }

  if (part != nullptr) {
#pragma unroll
    for (int nb = 0; nb < TN; ++nb)
#pragma unroll
      for (int mb = 0; mb < TM; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int nl = wn * TN * 16 + nb * 16 + PF32::row(kq, r);
          const int ml = wm * TM * 16 + mb * 16 + l16;
          part[ml + nl * BM] = cv{cr[nb][mb][r], ci[nb][mb][r]};
        }
    return;
  }
  cv* Y = reinterpret_cast<cv*>(g.Y);
  const cv* Z = reinterpret_cast<const cv*>(g.Z);
  const float al = (float)g.alpha, be = (float)g.beta, ga = (float)g.gamma;
#pragma unroll
  for (int nb = 0; nb < TN; ++nb)
#pragma unroll
    for (int mb = 0; mb < TM; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + wn * TN * 16 + nb * 16 + PF32::row(kq, r);
        const int64_t m = m0 + wm * TM * 16 + mb * 16 + l16;
        if (m >= g.M || n >= g.N) continue;
        cv out{al * cr[nb][mb][r], al * ci[nb][mb][r]};
        if (g.beta != 0.0) {
          const cv y = Y[m + n * g.ldy];
          out.re += be * y.re;
          out.im += be * y.im;
        }
        if (g.gamma != 0.0) {
          const cv z = Z[m + n * g.ldz];
          out.re += ga * z.re;
          out.im += ga * z.im;
        }
        Y[m + n * g.ldy] = out;
      }
}

// Whole launch of the direct-to-LDS FP32 step on the per-XCD work queue.
__device__ __forceinline__ void cdma_body(const GemmArgs& g, const TailSplit& tail) {
  using namespace dc;
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];
  __shared__ int last, item;
  const TileOrder o = tile_order(g.M, g.N, BM, BN);
  const QueueShare q = queue_share(tail, o);
  for (int64_t i; (i = queue_next(tail, q, &item)) >= 0;) {
    const WorkItem w = work_item(tail, o, i, g.K, BK);
    PF32::cplx* part = w.seg < 0 ? nullptr : reinterpret_cast<PF32::cplx*>(tail.ws) + w.seg * (int64_t)(BM * BN);
    if ((w.tm + 1) * BM <= g.M && (w.tn + 1) * BN <= g.N)
      cdma_tile_impl<false>(g, w.tm, w.tn, w.kbeg, w.kend, part, lds);
    else
      cdma_tile_impl<true>(g, w.tm, w.tn, w.kbeg, w.kend, part, lds);
    if (w.seg >= 0) zbig_arrive<PF32, WGM, WGN, TM, TN, BK>(g, tail, w, &last);
  }
  queue_leave(tail);
}

// Grouped step for many problems at once, on the direct-to-LDS tile: row
// `step` of the descriptor table lists one GEMM per problem with its tile
// count as a running prefix sum.  A persistent grid takes the step's tiles
// (all problems, problem by problem) from per-XCD counters; every parameter
// comes from device memory, so a captured graph of these launches stays
// valid while degrees, columns and scalars change.  A step with no work
// still passes through the queue, so the counters are always reset.
__device__ __forceinline__ void zdma_grouped_body(const GroupEntry* __restrict__ table, int count, int step,
                                                  int* queue) {
  using namespace dz;
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];
  __shared__ int item;
  const GroupEntry* __restrict__ row = table + (int64_t)step * count;
  TailSplit t;
  t.full = row[count - 1].tile_end;
  t.ksplit = 1;
  t.queue = queue;
  // Tiles are dealt to the XCDs in rotation (tile i to XCD i % 8): the table
  // lists the problems longest first, so every XCD gets the same mix of long
  // and short tiles, each longest first.  (Contiguous shares would give one
  // XCD the largest problems' tiles.)  No L2 reuse is lost that matters: a
  // tile's operands at 32 flop per byte stay well inside HBM's rate.
  const int xcd = (int)(blockIdx.x % 8);
  const int64_t mine = t.full > xcd ? (t.full - xcd + 7) / 8 : 0;
  int p = 0;
  for (int64_t it; (it = wg_fetch_add(queue + xcd, 1, &item)) < mine;) {
    const int64_t i = xcd + 8 * it;
    while (row[p].tile_end <= i) ++p;  // items arrive in increasing order
    p = __builtin_amdgcn_readfirstlane(p);
    const int64_t begin = p > 0 ? row[p - 1].tile_end : 0;
    const GemmArgs g = row[p].g;
    int64_t tm, tn;
    tile_rc(tile_order(g.M, g.N, BM, BN), i - begin, &tm, &tn);
    zdma_tile<false>(g, tm, tn, 0, g.K, nullptr, lds);
  }
  queue_leave(t);
}

// Tile configurations (waves along m, waves along n, 16-blocks per wave
// along m and n, K tile):
//   T0: 128 x 128 complex tile, 8 waves of 64 x 32, one workgroup per CU;
//   T1: 128 x 64, 4 waves of 64 x 32, two workgroups per CU (finer tiles
//       for few active columns).
// Which one a launch uses is decided by the autotuner in the driver.
#define T0_ARGS 2, 4, 4, 2, 8
#define T1_ARGS 2, 2, 4, 2, 8
using C0 = Cfg<T0_ARGS>;
using C1 = Cfg<T1_ARGS>;

__global__ __launch_bounds__(dz::NT, 1) void zfilter_step(GemmArgs g, TailSplit t) { zdma_body<false>(g, t); }
// real symmetric H (row-pair view) times a real block
__global__ __launch_bounds__(dz::NT, 1) void dfilter_step(GemmArgs g, TailSplit t) { zdma_body<true>(g, t); }
__global__ __launch_bounds__(C1::NT, 2) void zfilter_step_n64(GemmArgs g, TailSplit t) {
  zbig_body<PF64, T1_ARGS>(g, t);
}
// Same schedule for the other large H-times-block products (Rayleigh-Ritz H C).
__global__ __launch_bounds__(dz::NT, 1) void zgemm_nn_big(GemmArgs g, TailSplit t) { zdma_body<false>(g, t); }
// FP32 filter step of the mixed-precision solve (complex64 H and X, FP32
// accumulation): 128 x 128 tile, 8 waves of 64 x 32, K tile 16.
#define TF32_ARGS 2, 4, 4, 2, 16
using CF = Cfg<TF32_ARGS>;
__global__ __launch_bounds__(CF::NT, 1) void cfilter_step(GemmArgs g, TailSplit t) { zbig_body<PF32, TF32_ARGS>(g, t); }
// direct-to-LDS FP32 step (even M, K, leading dimensions)
__global__ __launch_bounds__(dc::NT, 1) void cfilter_step_dma(GemmArgs g, TailSplit t) { cdma_body(g, t); }
__global__ __launch_bounds__(dz::NT, 1) void zfilter_grouped(const GroupEntry* __restrict__ table, int count,
                                                             int step, int* queue) {
  zdma_grouped_body(table, count, step, queue);
}
__global__ __launch_bounds__(C1::NT, 2) void zfilter_grouped_n64(const GroupEntry* __restrict__ table, int count,
                                                                 int step) {
  zbig_grouped<T1_ARGS>(table, count, step);
}
__global__ void counters_zero(int* c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0;
}

struct CfgInfo {
  int bm, bn, bk, nt, wg_per_cu, wgm, wgn;
};
constexpr CfgInfo kCfg[2] = {{C0::BM, C0::BN, C0::BK_, C0::NT, 1, C0::WGM_, C0::WGN_},
                             {C1::BM, C1::BN, C1::BK_, C1::NT, 2, C1::WGM_, C1::WGN_}};
// the direct-to-LDS FP64 step (zfilter_step, zgemm_nn_big)
constexpr CfgInfo kDma = {dz::BM, dz::BN, dz::BK, dz::NT, 1, dz::WGM, dz::WGN};

}  // namespace

static int cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

int64_t zfilter_tiles(int64_t M, int64_t N, int64_t* tiles_n, int cfg) {
  const CfgInfo& c = kCfg[cfg & 1];
  if (tiles_n) *tiles_n = cdiv(N, c.bn);
  if (M <= 0 || N <= 0) return 0;
  return cdiv(M, c.bm) * cdiv(N, c.bn);
}

int zfilter_grouped_launch(const GroupEntry* table, int count, int step, int grid, hipStream_t s, int cfg,
                           int* queue) {
  if (count <= 0 || grid <= 0 || grid % 8) return -1;
  if (cfg == 1)
    hipLaunchKernelGGL(zfilter_grouped_n64, dim3((unsigned)grid), dim3(C1::NT), 0, s, table, count, step);
  else if (queue == nullptr)
    return -1;
  else
    hipLaunchKernelGGL(zfilter_grouped, dim3((unsigned)grid), dim3(dz::NT), 0, s, table, count, step, queue);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int grouped_grid(int cfg) { return (int)(8 * cdiv((int64_t)cu_count() * kCfg[cfg & 1].wg_per_cu, 8)); }

int64_t tail_workspace_bytes() { return (int64_t)kTailMaxSegments * C0::BM * C0::BN * 16; }

int queue_counters_init(int* queue, hipStream_t s) {
  hipLaunchKernelGGL(counters_zero, dim3(1), dim3(64), 0, s, queue, kQueueInts);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int tail_counters_init(int* counters, hipStream_t s) {
  hipLaunchKernelGGL(counters_zero, dim3((kTailCounterInts + 255) / 256), dim3(256), 0, s, counters,
                     kTailCounterInts);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int zgemm_nn_big_launch(const GemmArgs& g, hipStream_t s, bool filter_symbol, void* tail_ws, int* tail_counters,
                        int choice, int max_segments) {
  if (g.M <= 0 || g.N <= 0) return kOk;
  if (g.ws != nullptr || g.upper_b || g.lower_only || g.bscale != nullptr) return -1;
  if (!tail_ws || !tail_counters) return -1;
  const int cfg = (choice == kChoiceT1Tail && filter_symbol) ? 1 : 0;
  const CfgInfo& c = cfg == 1 ? kCfg[1] : kDma;
  TileGeom geo;
  geo.M = g.M; geo.N = g.N; geo.bm = c.bm; geo.bn = c.bn; geo.wgm = c.wgm; geo.wgn = c.wgn;
  if (cfg == 0) geo.narrow_cols = 32;  // the direct-to-LDS step's narrow edge layout
  TailSplit t;
  const int64_t grid = plan_schedule(geo, cdiv(g.K, c.bk), (int64_t)cu_count() * c.wg_per_cu, 16,
                                     choice != kChoiceT0NoTail, tail_ws, tail_counters, &t, max_segments);
  if ((cdiv(g.M, c.bm) * cdiv(g.N, c.bn) - t.full) * t.ksplit > max_segments)
    return -1;  // the planner keeps to the cap; a split past it would overrun tail_ws
  GemmArgs a = g;
  if (a.K <= 0) a.alpha = 0.0;
  if (!filter_symbol)
    hipLaunchKernelGGL(zgemm_nn_big, dim3((unsigned)grid), dim3(dz::NT), 0, s, a, t);
  else if (cfg == 1)
    hipLaunchKernelGGL(zfilter_step_n64, dim3((unsigned)grid), dim3(C1::NT), 0, s, a, t);
  else
    hipLaunchKernelGGL(zfilter_step, dim3((unsigned)grid), dim3(dz::NT), 0, s, a, t);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int dfilter_big_launch(const GemmArgs& g, hipStream_t s, void* tail_ws, int* tail_counters) {
  if (g.M <= 0 || g.N <= 0) return kOk;
  if (g.ws != nullptr || g.upper_b || g.lower_only || g.bscale != nullptr) return -1;
  if (!tail_ws || !tail_counters) return -1;
  // 16-byte lanes: two k of a column of B, one complex row pair of A
  if (g.K % 2 != 0 || g.ldb % 2 != 0 || reinterpret_cast<uintptr_t>(g.A) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(g.B) % 16 != 0)
    return -1;
  TileGeom geo;
  geo.M = g.M; geo.N = g.N; geo.bm = kDma.bm; geo.bn = kDma.bn; geo.wgm = kDma.wgm; geo.wgn = kDma.wgn;
  geo.narrow_cols = 32;
  TailSplit t;
  const int64_t grid = plan_schedule(geo, cdiv(g.K, kDma.bk), (int64_t)cu_count() * kDma.wg_per_cu, 16, true,
                                     tail_ws, tail_counters, &t);
  GemmArgs a = g;
  if (a.K <= 0) a.alpha = 0.0;
  hipLaunchKernelGGL(dfilter_step, dim3((unsigned)grid), dim3(dz::NT), 0, s, a, t);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int cfilter_big_launch(const CGemmArgs& c, hipStream_t s, void* tail_ws, int* tail_counters) {
  if (c.M <= 0 || c.N <= 0) return kOk;
  if (!tail_ws || !tail_counters) return -1;
  // The kernel reads operands through the same argument block as the FP64
  // one; pointers are reinterpreted as complex64 inside.
  GemmArgs g;
  g.M = c.M; g.N = c.N; g.K = c.K;
  g.A = reinterpret_cast<const z64*>(c.A); g.lda = c.lda;
  g.B = reinterpret_cast<const z64*>(c.B); g.ldb = c.ldb;
  g.Y = reinterpret_cast<z64*>(c.Y); g.ldy = c.ldy;
  g.Z = reinterpret_cast<const z64*>(c.Z); g.ldz = c.ldz;
  g.alpha = c.alpha; g.beta = c.beta; g.gamma = c.gamma;
  if (g.K <= 0) g.alpha = 0.0;
  // two complex64 per 16-byte load: pairs must not straddle a row range, K
  // or an alignment boundary
  const bool dma = g.M % 2 == 0 && g.K % 2 == 0 && g.lda % 2 == 0 && g.ldb % 2 == 0 &&
                   reinterpret_cast<uintptr_t>(c.A) % 16 == 0 && reinterpret_cast<uintptr_t>(c.B) % 16 == 0;
  TileGeom geo;
  geo.M = g.M; geo.N = g.N; geo.bm = CF::BM; geo.bn = CF::BN; geo.wgm = CF::WGM_; geo.wgn = CF::WGN_;
  TailSplit t;
  if (dma) {
    const int64_t grid = plan_schedule(geo, cdiv(g.K, dc::BK), cu_count(), 8, true, tail_ws, tail_counters, &t);
    hipLaunchKernelGGL(cfilter_step_dma, dim3((unsigned)grid), dim3(dc::NT), 0, s, g, t);
  } else {
    const int64_t grid = plan_schedule(geo, cdiv(g.K, CF::BK_), cu_count(), 16, true, tail_ws, tail_counters, &t);
    hipLaunchKernelGGL(cfilter_step, dim3((unsigned)grid), dim3(CF::NT), 0, s, g, t);
  }
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
