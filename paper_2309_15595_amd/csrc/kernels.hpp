// Launchers of the hand-written gfx950 kernels used by the ChASE driver.
#pragma once
#include "common.hpp"

namespace chase {

// Arguments of the complex FP64 GEMM (see zgemm.hip):
//   Y = alpha * opA(A) opB(B) + beta * Y + gamma * Z       (M x N, K inner)
struct GemmArgs {
  int64_t M = 0, N = 0, K = 0;
  const z64* A = nullptr; int64_t lda = 0;
  const z64* B = nullptr; int64_t ldb = 0;
  z64* Y = nullptr;       int64_t ldy = 0;
  const z64* Z = nullptr; int64_t ldz = 0;
  double alpha = 1.0, beta = 0.0, gamma = 0.0;
  z64* ws = nullptr;      int64_t ws_stride = 0; int64_t k_chunk = 0;
  const double* bscale = nullptr;  // optional: opB(B)[k][n] *= bscale[k] (diag(g) X^H)
  int upper_b = 0;     // opB(B) upper triangular: skip its zero K range
  int lower_only = 0;  // skip tiles strictly above the diagonal (m < n everywhere)
  int real_b = 0;      // zgemm_launch nn / nc: opB(B) is real-valued (its imaginary parts are not read)
  int real_out = 0;    // zgemm cn (also split over K): only the real part is formed, the imaginary is zero
};

// opa/opb: 0 = as stored, 1 = conjugate transpose.
int zgemm_launch(int opa, int opb, const GemmArgs& g, hipStream_t s);
// Schedule of the large tiled products (see sched.hpp): whole tiles plus the
// last, partial round of tiles split along K, handed out by per-XCD work
// queues to a persistent grid.
constexpr int kTailMaxSegments = 1024;
constexpr int kQueueInts = 16;  // 8 per-XCD item counters, a finished-workgroup count, spare
// ints of the counter block: kTailMaxSegments arrival counters + the queue
constexpr int kTailCounterInts = kTailMaxSegments + kQueueInts;
struct TailSplit {
  int64_t full = 0;        // tiles computed whole
  int64_t ksplit = 1;      // K segments per remaining tile
  void* ws = nullptr;      // kTailMaxSegments partial tiles
  int* counters = nullptr; // kTailMaxSegments arrival counters, zero between launches
  int* queue = nullptr;    // kQueueInts queue counters, zero between launches
};
// Output tiling of one launch, for the schedule's cost model: bm x bn tiles
// of an M x N output, each computed by wgm x wgn waves (wave w owns sub-tile
// (w % wgm, w / wgm)); on gfx950 waves w and w + 4 of a workgroup share a
// SIMD.
struct TileGeom {
  int64_t M = 0, N = 0;
  int bm = 128, bn = 128, wgm = 2, wgn = 4;
  // last column tiles with at most narrow_cols live columns are computed by
  // 8 x 1 waves of (bm / 8) x (bn / wgn), those with at most 2 narrow_cols by
  // 4 x 2 waves of (bm / 4) x (bn / wgn) (0: neither layout)
  int narrow_cols = 0;
};
// Split and grid of one launch of `nkt` K-tiles per tile with `resident`
// workgroups resident at once (schedule.cpp).  Candidate splits of the last
// round(s) of tiles along K (segments of at least min_kt_per_seg K-tiles) are
// compared by simulating the per-XCD queues with a per-tile cost (a tile
// costs its busiest SIMD's share of MFMA work: an edge tile whose live
// columns fit in the first half of the waves costs half a tile).
// counters: kTailCounterInts ints.  Returns the grid.
// max_segments (<= kTailMaxSegments) caps the partial tiles of the split, for
// callers whose workspace holds fewer than kTailMaxSegments of them.
int64_t plan_schedule(const TileGeom& geo, int64_t nkt, int64_t resident, int min_kt_per_seg, bool allow_split,
                      void* ws, int* counters, TailSplit* t, int max_segments = kTailMaxSegments);
int64_t tail_workspace_bytes();
int tail_counters_init(int* counters, hipStream_t s);
// Large NN products (filter step, H C): 128 x 128 tiles, double-buffered LDS
// (zfilter.hip), on the persistent work-queue schedule of plan_schedule; the
// last partial round of tiles is split along K.  tail_ws / tail_counters
// (tail_workspace_bytes(), kTailCounterInts ints, zeroed once by
// tail_counters_init) are required and serialise launches that share them.
// filter_symbol selects the kernel name reported by profilers.  choice
// (filter only): tile configuration and tail policy picked by the autotuner.
constexpr int kChoiceT0Tail = 0;    // 128 x 128, split-K tail
constexpr int kChoiceT0NoTail = 1;  // 128 x 128, no tail split
constexpr int kChoiceT1Tail = 2;    // 128 x 64, split-K tail
constexpr int kNumChoices = 3;
int zgemm_nn_big_launch(const GemmArgs& g, hipStream_t s, bool filter_symbol, void* tail_ws, int* tail_counters,
                        int choice = kChoiceT0Tail, int max_segments = kTailMaxSegments);
// One problem's filter GEMM in a grouped launch: tiles [tile_end - tiles,
// tile_end) of the step's running tile count belong to it.
struct GroupEntry {
  GemmArgs g;
  int64_t tiles_n = 1;
  int64_t tile_end = 0;
};
// Tiles of filter configuration cfg (0: 128 x 128, 1: 128 x 64) for an
// M x N output (tiles_n: column tiles).
int64_t zfilter_tiles(int64_t M, int64_t N, int64_t* tiles_n, int cfg = 0);
// Persistent grouped filter step over row `step` of a device table of
// `count` entries per step; grid a multiple of 8 (see grouped_grid).  cfg 0
// (128 x 128 direct-to-LDS tile) takes tiles from the work queue `queue`
// (kQueueInts ints, zeroed once by queue_counters_init; launches sharing it
// must be serialised); cfg 1 (128 x 64 staged tile) needs none.
int zfilter_grouped_launch(const GroupEntry* table, int count, int step, int grid, hipStream_t s, int cfg,
                           int* queue);
int queue_counters_init(int* queue, hipStream_t s);
// Grid filling every CU with resident workgroups of configuration cfg.
int grouped_grid(int cfg);
// Split over K into `splits` partial products in `ws`, summed in fixed order;
// hermitise = 1 stores (S + S^H)/2 (M == N); hermitise = 2 computes and
// stores only the lower triangle of a Hermitian product (M == N), with a real
// diagonal, leaving the strict upper triangle of Y untouched; hermitise = 3
// does the same keeping only real parts (the product of two real blocks read
// as complex row pairs: its real part is X^T Y, its imaginary part is not
// part of the product).
int zgemm_splitk(int opa, int opb, const GemmArgs& g, void* ws, int splits, int hermitise,
                 hipStream_t s);
int64_t zgemm_splitk_workspace(int64_t M, int64_t N, int splits);
int choose_splits(int64_t M, int64_t N, int64_t K, int max_splits, bool lower = false);

// G = X diag(s) X^H (zgrad.hip): g.A = g.B = X (M x K, ld), g.bscale = s (K,
// device), g.Y = G; g.lower_only computes only the tiles that hold an element
// on or below the diagonal (M == N).  Allocates nothing.
int zgrad_launch(const GemmArgs& g, hipStream_t s);

// Real filter step (zfilter.hip): Y = alpha A B + beta Y + gamma Z for a real
// matrix read as complex row pairs.  A: M x K complex view (2M real rows,
// lda in complex units), B: real K x N block (double*, ldb in doubles, even),
// Y, Z: complex views of real 2M x N blocks.  K and ldb even, A and B 16-byte
// aligned; otherwise -1.  Same schedule and split-K tail as the FP64 step.
int dfilter_big_launch(const GemmArgs& g, hipStream_t s, void* tail_ws, int* tail_counters);

// Complex FP32 GEMM (mixed-precision filter): same contract with complex64 data.
struct CGemmArgs {
  int64_t M = 0, N = 0, K = 0;
  const c32* A = nullptr; int64_t lda = 0;
  const c32* B = nullptr; int64_t ldb = 0;
  c32* Y = nullptr;       int64_t ldy = 0;
  const c32* Z = nullptr; int64_t ldz = 0;
  float alpha = 1.0f, beta = 0.0f, gamma = 0.0f;
};
// FP32 filter step (zfilter.hip): same schedule, split-K tail and epilogue as
// the FP64 one, on complex64 data with FP32 accumulation.
int cfilter_big_launch(const CGemmArgs& g, hipStream_t s, void* tail_ws, int* tail_counters);

// BF16x3 filter step (bfilter.hip): H as four bfloat16 planes (Re hi, Re lo,
// Im hi, Im lo of conj(H) in H's memory order, rows padded to ldp), X, Y, Z
// complex64.
struct BGemmArgs {
  int64_t M = 0, N = 0, K = 0;
  const uint16_t* P = nullptr; int64_t ldp = 0; int64_t plane_stride = 0;
  const c32* X = nullptr; int64_t ldx = 0;
  c32* Y = nullptr;       int64_t ldy = 0;
  const c32* Z = nullptr; int64_t ldz = 0;
  float alpha = 1.f, beta = 0.f, gamma = 0.f;
  // bfloat16 planes (Re hi, Re lo, Im hi, Im lo) of X (read) and of Y
  // (written with Y): column n of plane p at Xp + p xps + n ldxp, k padded
  // with zeros to a multiple of 32 (ldxp)
  const uint16_t* Xp = nullptr; int64_t ldxp = 0; int64_t xps = 0;
  uint16_t* Yp = nullptr;       int64_t ldyp = 0; int64_t yps = 0;
};
int64_t bsplit_ld(int64_t N);
// The planes of a complex64 block (rows x ncols, rows padded with zeros to ldxp).
int bsplit_block(const c32* X, int64_t ldx, int64_t rows, int64_t ncols, uint16_t* Xp, int64_t ldxp, int64_t xps,
                 hipStream_t s);
int bsplit_planes(const z64* H, int64_t lda, int64_t N, uint16_t* P, hipStream_t s);
int bfilter_launch(const BGemmArgs& g, hipStream_t s, void* tail_ws, int* tail_counters);

// ---- Householder QR (hhqr.hip) ---------------------------------------------
// Blocked Householder QR of the M x n block X (n <= M) in LAPACK's
// conventions, then X <- the explicit M x n factor Q.  Device scratch:
constexpr int kHouseholderPanel = 32;
constexpr int kHouseholderMaxWg = 128;  // workgroups per reflector launch
struct HouseholderWs {
  z64* V = nullptr;       // M x panel (explicit reflectors of one panel)
  z64* T = nullptr;       // cdiv(n, panel) x panel x panel (block reflector factors)
  z64* W1 = nullptr;      // panel x n
  z64* W2 = nullptr;      // panel x n
  double* part = nullptr; // kHouseholderMaxWg x 2 panel partial sums
  z64* rowj = nullptr;    // panel
  z64* tau = nullptr;     // n
  z64* Q = nullptr;       // M x n (leading dimension M)
  z64* splitk = nullptr;  // split-K partials: 16 x panel x n
  z64* R = nullptr;       // optional n x n output (leading dimension n): the R factor, zero below the diagonal
};
int householder_qr(z64* X, int64_t ldx, int64_t M, int64_t n, const HouseholderWs& ws, hipStream_t s);

// The 2n x 2n Hermitian [[0, R], [R^H, 0]] of an n x n R (lower triangle
// written: the R^H block; the diagonal blocks zero), whose eigenvalues are
// the singular values of R and their negatives.
int augment_hermitian(const z64* R, int64_t n, z64* Aug, hipStream_t s);

// ---- small dense kernels (small.hip) --------------------------------------
// Blocked lower Cholesky G = L L^H in place (lower part), n x n, ld.
// *info (device) receives 0, or j+1 for the first non-positive pivot j.
int potrf_lower(z64* G, int64_t ld, int64_t n, int* info, z64* ws_gemm, hipStream_t s);
// Lower-triangular inverse Linv = L^{-1} (n x n); tmp is n x n scratch.
int trtri_lower(const z64* L, int64_t ldl, z64* Linv, int64_t ldi, int64_t n, z64* tmp,
                hipStream_t s);
// G[j][j] += s where s = 11 (m n + n (n+1)) u ||X||_F^2 and ||X||_F^2 = trace(G),
// computed on the device; shift_out (device, 1 double) keeps s.
int add_cholqr_shift(z64* G, int64_t ld, int64_t n, int64_t m, double* shift_out, hipStream_t s);
// Zero the strictly upper part of an n x n matrix.
int zero_upper(z64* G, int64_t ld, int64_t n, hipStream_t s);
// out[j] = || Y[:, j] - theta[j] X[:, j] ||_2 for j < n (theta device).
int residual_norms(const z64* Y, int64_t ldy, const z64* X, int64_t ldx, const double* theta,
                   int64_t N, int64_t n, double* out, hipStream_t s);
// dst[:, j] = src[:, perm[j]], j < n (perm device).
int gather_columns(const z64* src, int64_t lds, z64* dst, int64_t ldd, const int* perm,
                   int64_t N, int64_t n, hipStream_t s);
// Column block copy (N x n).
int copy_columns(const z64* src, int64_t lds, z64* dst, int64_t ldd, int64_t N, int64_t n,
                 hipStream_t s);
// W = A V for Hermitian A (reads A's columns), V: N x nv (nv <= 8).
int hemv_block(const z64* A, int64_t lda, const z64* V, int64_t ldv, z64* W, int64_t ldw,
               int64_t N, int nv, hipStream_t s);
// The same for complex64 H (products accumulated in FP64).
int hemv_block_c64(const c32* A, int64_t lda, const z64* V, int64_t ldv, z64* W, int64_t ldw,
                   int64_t N, int nv, hipStream_t s);
// One Lanczos step for nv independent vectors (see small.hip).
int lanczos_step(z64* V, z64* Vold, z64* W, int64_t N, int nv, int step, int ksteps,
                 double* alpha, double* beta, hipStream_t s);
int lanczos_init(const z64* starts, int64_t ld, z64* V, z64* Vold, int64_t N, int nv,
                 hipStream_t s);
// Gaussian (re + i im)/sqrt(2) fill from a counter-based generator (splitmix64).
int fill_gaussian(z64* X, int64_t ld, int64_t N, int64_t n, uint64_t seed, hipStream_t s);
// X[:, j] *= g[j] (g device, real).
int scale_columns(const z64* X, int64_t ldx, const double* g, z64* out, int64_t ldo, int64_t N,
                  int64_t n, hipStream_t s);
// Non-finite detection over n doubles: *flag (device int) = 1 if any.
int check_finite(const double* x, int64_t n, int* flag, hipStream_t s);
// Mirror the lower triangle into the upper one (Hermitian full storage).
int hermitian_mirror_lower(z64* G, int64_t ld, int64_t n, hipStream_t s);
// Real symmetric problems.  W[:, c] = H V[:, c] (c < nv <= 8) for real
// symmetric H of order N; rows N .. rows_out - 1 of W are set to zero.
int symv_block(const double* H, int64_t ldh, const double* V, int64_t ldv, double* W, int64_t ldw, int64_t N,
               int64_t rows_out, int nv, hipStream_t s);
// dst (rows_dst x cols_dst) = src (rows_src x cols_src) extended with zeros.
int dcopy_pad(const double* src, int64_t lds, int64_t rows_src, int64_t cols_src, double* dst, int64_t ldd,
              int64_t rows_dst, int64_t cols_dst, hipStream_t s);
// R = Re(G) and G = R + 0 i for n x n blocks.
// A real M x n block (leading dimension ldr, in doubles) as a complex128
// block with zero imaginary parts, and back (the real parts).
int widen_real_block(const double* R, int64_t ldr, z64* X, int64_t ldx, int64_t M, int64_t n, hipStream_t s);
int real_part_block(const z64* X, int64_t ldx, double* R, int64_t ldr, int64_t M, int64_t n, hipStream_t s);
// complex128 <-> complex64 conversions (column blocks); the widening one
// multiplies by `scale` in FP64 (1 leaves the values as they are).
int convert_z_to_c(const z64* src, int64_t lds, c32* dst, int64_t ldd, int64_t N, int64_t n,
                   hipStream_t s);
int convert_c_to_z(const c32* src, int64_t lds, z64* dst, int64_t ldd, int64_t N, int64_t n,
                   hipStream_t s, double scale = 1.0);

// Eigen-decomposition of the n x n Hermitian matrix G (lower triangle read,
// leading dimension ldg) by two-sided block Jacobi (heevj.hip): ascending
// eigenvalues into theta (device, n), eigenvectors written over G.  ws:
// heevj_workspace_bytes(n) bytes.  Host-synchronous once per sweep; returns
// kBreakdown for non-finite input or no convergence in 40 sweeps.
int64_t heevj_workspace_bytes(int64_t n);
int heevj(z64* G, int64_t ldg, int64_t n, double* theta, void* ws, int* sweeps_out, hipStream_t s);

// Argument checks of chase_filter (driver.cpp): 0, or the negative status.
int filter_check_args(const void* A, int64_t lda, const void* V, int64_t ldv, const void* W, int64_t ldw, int64_t N,
                      int64_t n, const int32_t* degs, double e);
// chase_filter's steps on caller-owned tail scratch: max_segments partial
// 128 x 128 complex128 tiles at tail_ws and kTailCounterInts ints at
// tail_counters (cleared by a fill kernel first); enqueued on s, no wait.
int filter_on_scratch(const void* A, int64_t lda, void* V, int64_t ldv, void* W, int64_t ldw, int64_t N, int64_t n,
                      const int32_t* degs, double c, double e, double mu_1, int64_t* matvecs, void* tail_ws,
                      int* tail_counters, int max_segments, hipStream_t s);

}  // namespace chase
