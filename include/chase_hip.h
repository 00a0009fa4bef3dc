/*
 * chase_hip.h -- C ABI of the MI355X (gfx950) ChASE hot path.
 *
 * ChASE finds the nev lowest eigenpairs of a dense Hermitian matrix H by
 * Chebyshev-filtered subspace iteration (Wu & Di Napoli, arXiv 2309.15595):
 * Lanczos spectral bounds, then a loop of {Chebyshev filter (Eq. 1),
 * condition-number estimate (Alg. 5), 1D-CAQR (Alg. 3 and Alg. 4),
 * Rayleigh-Ritz, residuals, deflation and locking, degree optimisation} as in
 * Alg. 1 and Alg. 2, here on one GPU (a 1 x 1 grid: every AllReduce is the
 * identity and B2 aliases C2).
 *
 * Conventions for every entry point:
 *   - matrices are column-major complex128 ((re, im) double pairs) unless the
 *     entry point says float64 (the real symmetric variant) or complex64, with
 *     a leading dimension >= the row count, addressed by DEVICE pointers
 *     unless an argument says (host);
 *   - device pointers must be 16-byte aligned;
 *   - sizes are int64_t;
 *   - work is ordered on `stream` after the caller's earlier work on it; an
 *     entry point returns once its results are complete on the device
 *     (host-synchronous) unless it says otherwise;
 *   - the caller owns every buffer it passes; the library never frees or
 *     retains a caller pointer after returning.
 *
 * Return codes (LAPACK-like): 0 success; -k argument k invalid; 1 the solve
 * stopped at max_iter before nev pairs converged (outputs hold the best
 * approximations); 2 device allocation failed; 3 HIP runtime error (see
 * chase_last_error); 4 numerical breakdown (non-finite values, or every QR
 * route failed).
 */
#ifndef CHASE_HIP_H
#define CHASE_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* chase_stream_t; /* a hipStream_t; NULL = the default stream */

enum {
  CHASE_FP64 = 0,       /* every step in FP64 */
  CHASE_FP32_MIXED = 1, /* filter GEMMs in FP32 until a vector's residual reaches
                           the FP32 floor, then FP64; QR, RR, residuals in FP64 */
  CHASE_BF16X3_MIXED = 2 /* filter in BF16x3 split products (FP32 accumulate)
                            down to the BF16x3 floor, then FP32, then FP64 */
};

enum {
  CHASE_QR_AUTO = -1,  /* Alg. 4's choice from CondEst */
  CHASE_QR_CHOLQR1 = 0,
  CHASE_QR_CHOLQR2 = 1,
  CHASE_QR_SHIFTED = 2,
  CHASE_QR_HOUSEHOLDER = 3
};

/* Inputs of Alg. 2 (nev, nex, deg, tol, MaxIter, opt) plus the readings the
 * paper leaves open.  Fill with chase_default_params first. */
typedef struct {
  int32_t nev;          /* wanted eigenpairs, >= 1 */
  int32_t nex;          /* search-space increment, >= 0, nev + nex < N */
  int32_t deg;          /* initial filter degree, even, >= 2 (20) */
  int32_t max_deg;      /* cap on optimised degrees, even (36) */
  int32_t deg_extra;    /* margin added by degree optimisation, even; negative
                           (default -1): 4 when every column is filtered in
                           FP64, 2 on the FP32 / BF16x3 ladders and complex64 */
  int32_t max_iter;     /* MaxIter (25) */
  int32_t opt;          /* 1 = per-vector degree optimisation (1) */
  int32_t precision;    /* CHASE_FP64, CHASE_FP32_MIXED or CHASE_BF16X3_MIXED */
  int32_t lanczos_steps;/* steps per Lanczos run (25) */
  int32_t force_qr;     /* CHASE_QR_AUTO, or force one QR variant (testing) */
  int32_t bounds_given; /* 1 = skip Lanczos and use b_sup, mu_1, mu_ne, norm_est */
  int32_t autotune;     /* 1 = pick the filter's tile shape per size by timing the
                           candidates (results kept for the process); 0 = default */
  double tol;           /* residual threshold relative to ||H|| (1e-10) */
  double b_sup, mu_1, mu_ne, norm_est;
  double mixed_switch;  /* FP32 -> FP64 switch at resd <= mixed_switch * ||H|| (5e-6) */
  double bf16_switch;   /* BF16x3 -> FP32 switch at resd <= bf16_switch * ||H|| (5e-5) */
  uint64_t seed;        /* generator of the initial block / Lanczos starts when
                           the caller supplies none */
} chase_params_t;

typedef struct {
  int32_t status;
  int32_t iterations;
  int32_t locked;
  int32_t qr_count[4];      /* CholQR1, CholQR2, shifted CholQR2, Householder */
  int32_t eig_sweeps;       /* block-Jacobi sweeps of the quotient eigensolves, summed */
  int64_t filter_matvecs;   /* sum over iterations of sum_j d_j */
  int64_t filter_matvecs_fp32; /* of which in FP32 (mixed precision) */
  int64_t filter_matvecs_bf16; /* of which in BF16x3 (mixed precision) */
  int64_t total_matvecs;    /* filter + Lanczos + Rayleigh-Ritz + residual */
  int64_t filter_launches;  /* filter GEMM launches (one per degree step) */
  double filter_flops;      /* 8 N^2 filter_matvecs (algorithmic, any precision) */
  double t_total, t_lanczos, t_filter, t_qr, t_rr, t_resid; /* seconds (HIP events) */
  double bounds[4];         /* b_sup, mu_1, mu_ne, norm_est actually used */
} chase_stats_t;

typedef struct chase_handle_s* chase_handle_t;

/* Defaults of the experiments (deg 20, max_deg 36, tol 1e-10, opt on). */
int chase_default_params(chase_params_t* p);

/* Allocates the device workspace for problems of order N with the given
 * nev + nex: C2 and B (N x n_e each, Alg. 2's buffers; the caller's V is C),
 * the n_e x n_e Rayleigh quotient A / Gram matrix, split-K partials, the
 * Lanczos vectors and, for CHASE_FP32_MIXED, an FP32 copy of H (8 N^2 bytes)
 * and two FP32 N x n_e blocks.  Memory model of Eq. (2) at p = q = 1.
 * Returns 2 when an allocation fails (nothing is leaked). */
int chase_create(int64_t N, const chase_params_t* p, chase_handle_t* h);

/* Device bytes that creating a handle for order N and these params
 * allocates, computed on the host by the same code path that allocates
 * (nothing is allocated and no device call is made; no GPU is needed).
 * This is the library's share of Eq. (2)'s memory model at p = q = 1
 * (N^2 + 4 N n_e + n_e^2 words): the caller holds H and V (N^2 + N n_e
 * words); the library holds C2 and B (2 N n_e words), three n_e x n_e
 * matrices and the 16 split-K partials of the n_e x n_e products
 * (19 n_e^2 words), a fixed 256 MiB of split-K tail partials for the filter,
 * O(N + n_e) Lanczos, Householder-panel and scalar vectors, and the
 * low-precision copies listed under chase_create.
 *   variant  0: chase_create (complex128), 1: chase_create_real (float64;
 *            an odd N includes the zero-padded copy of H that every solve
 *            of an odd order uses; an odd lda at even N adds the same
 *            (N+1)^2 doubles on first use, and its first Householder QR
 *            two N x n_e and one N x 32 complex128 blocks), 2: chase_create_c64
 *   bytes    (host) out
 * Not counted: the buffers of the level-2 trace, allocated on its first use
 * (an N x n_e copy of the block, and 2 (2 n_e)^2 + 5 n_e^2 words for the
 * singular values of its R).
 * Returns -1 for N < 2, -2 for invalid params (or a precision the variant
 * does not offer), -3 for an unknown variant, -4 for a null bytes. */
int chase_workspace_bytes(int64_t N, const chase_params_t* p, int32_t variant, int64_t* bytes);

/* Solves for the nev lowest eigenpairs of Hermitian H (Alg. 2).
 *   A      (device) N x N, full Hermitian storage, read only
 *   V      (device) N x (nev+nex), in/out.  On entry the initial block when
 *          use_v0 = 1 (random or approximate eigenvectors, Sec. 1 / Sec. 3.1);
 *          otherwise it is filled from params.seed.  On return columns
 *          0..nev-1 hold the eigenvectors, ascending eigenvalues.
 *   starts (device, nullable) N x nstarts Lanczos start vectors; NULL draws
 *          4 from params.seed
 *   ritzv, resid (host) nev doubles each: eigenvalues ascending, residual
 *          norms ||H x - lambda x||_2
 *   stats  (host, nullable)
 * With CHASE_LOG=1 in the environment (read once per process) every solve
 * (all variants, and each problem of chase_solve_batched) prints one line per
 * outer iteration on stderr: the locked count, CondEst and the QR variant it
 * chose, the active residuals' range against tol, the filter degrees' range
 * and the eigensolve's Jacobi sweeps. */
int chase_solve(chase_handle_t h, const void* A, int64_t lda, void* V, int64_t ldv, int32_t use_v0,
                const void* starts, int64_t ld_starts, int32_t nstarts, double* ritzv, double* resid,
                chase_stats_t* stats, chase_stream_t stream);  /* -1: null, real or complex64 handle */

/* Frees every device buffer chase_create (or chase_create_real /
 * chase_create_c64) allocated, and the handle itself; h must not be used
 * afterwards.  The caller's buffers (H, V, starts) are never owned by the
 * handle and stay untouched.  The caller must not destroy a handle while a
 * solve on it is running.  Returns -1 for a null handle. */
int chase_destroy(chase_handle_t h);

/* Many independent problems of uneven N, each with its own params (FP64),
 * solved together.  Every degree step of all problems' Chebyshev filters runs
 * as one persistent grouped launch over a device descriptor table (one GEMM
 * per problem per step); the launches of all steps are captured once in a HIP
 * graph and replayed each outer iteration after the table is refreshed.  QR,
 * Rayleigh-Ritz, residuals and locking run per problem (Alg. 2).  Arrays have
 * length `count`; pointers as in chase_solve.  starts / ld_starts / nstarts /
 * use_v0 may be NULL (then: library-drawn starts, use_v0 = 1).  stats[i]
 * (nullable array) reports the shared filter and total times.  Returns the
 * worst status over the problems. */
int chase_solve_batched(int32_t count, const int64_t* N, const void* const* A, const int64_t* lda,
                        void* const* V, const int64_t* ldv, const int32_t* use_v0,
                        const void* const* starts, const int64_t* ld_starts, const int32_t* nstarts,
                        const chase_params_t* params, double* const* ritzv, double* const* resid,
                        chase_stats_t* stats, chase_stream_t stream);

/* Gradient of L = sum_i g_i lambda_i with respect to H (Hellmann-Feynman:
 * d lambda_i = x_i^H dH x_i):  G = X diag(g) X^H.
 *   X (device) N x nev eigenvectors, g (device) nev doubles, G (device) N x N.
 *   fill = 0 writes the full Hermitian G, 1 only its lower triangle.
 * Asynchronous on `stream` (allocates nothing). */
int chase_eigval_grad(int64_t N, int32_t nev, const void* X, int64_t ldx, const double* g, void* G,
                      int64_t ldg, int32_t fill, chase_stream_t stream);

/* ---- real symmetric H (the library's real type variant) ------------------
 * The same method on a real symmetric matrix with real vectors: every
 * matrix argument is a column-major double array (device, 16-byte aligned),
 * and each filter MatVec costs 2 N^2 flops instead of 8 N^2.  Inside, a real
 * column of even length is read as complex numbers of its row pairs, so the
 * filter runs on a real variant of the complex kernel (real H read as
 * complex row pairs times the real block) and the other steps on the complex
 * kernels, keeping the real part where a product of two real blocks is
 * formed.  FP64 only (params.precision must be CHASE_FP64). */

/* Workspace for real symmetric problems of order N (any N >= 2): the complex
 * buffers of chase_create at N/2 rows plus an internal copy of the block, an
 * n_e x n_e real buffer and, for odd N or odd lda, a padded copy of H made at
 * the first such solve.  A handle from here serves chase_solve_real only. */
int chase_create_real(int64_t N, const chase_params_t* p, chase_handle_t* h);

/* chase_solve for real symmetric A (N x N, full storage, read only): V
 * (N x (nev+nex), in/out), starts (N x nstarts, nullable), ritzv and resid
 * (host) as there.  Returns -1 for a handle not made by chase_create_real. */
int chase_solve_real(chase_handle_t h, const double* A, int64_t lda, double* V, int64_t ldv, int32_t use_v0,
                     const double* starts, int64_t ld_starts, int32_t nstarts, double* ritzv, double* resid,
                     chase_stats_t* stats, chase_stream_t stream);

/* chase_filter on real data; N, lda, ldv and ldw must be even (-7, -2, -4,
 * -6 otherwise). */
int chase_filter_real(const double* A, int64_t lda, double* V, int64_t ldv, double* W, int64_t ldw, int64_t N,
                      int64_t n, const int32_t* degs, double c, double e, double mu_1, int64_t* matvecs,
                      chase_stream_t stream);

/* ---- complex64 H (the library's single-precision complex variant) --------
 * A, V and starts are complex64 ((re, im) float pairs, device, 16-byte
 * aligned).  H is used in place (8 N^2 bytes, no copy): the filter and the
 * Rayleigh-Ritz product H Q run on the FP32 matrix kernels; QR, the small
 * eigensolve, residuals and locking run in FP64 on an internal complex128
 * copy of the block, which is rounded back to complex64 in V at the end.
 * The attainable residual is set by the FP32 products, about sqrt(N) u_32
 * ||H||: choose tol accordingly (1e-5 at N = 20000).  params.precision must
 * not be CHASE_BF16X3_MIXED; it is otherwise not used. */
int chase_create_c64(int64_t N, const chase_params_t* p, chase_handle_t* h);
/* chase_solve for complex64 data; -1 for a handle not made by chase_create_c64. */
int chase_solve_c64(chase_handle_t h, const void* A, int64_t lda, void* V, int64_t ldv, int32_t use_v0,
                    const void* starts, int64_t ld_starts, int32_t nstarts, double* ritzv, double* resid,
                    chase_stats_t* stats, chase_stream_t stream);

/* ---- steps of the loop, exposed for element-wise checks ------------------
 * These run one step of Alg. 2 exactly as chase_solve does. */

/* Chebyshev filter (Eq. 1, scaled three-term recurrence): column j of V
 * (N x n) becomes p_{d_j}(H) v_j, p_m(x) = T_m((x-c)/e) / T_m((mu_1-c)/e).
 * degs (host) n even degrees >= 2 sorted ascending; W (device) N x n
 * scratch (the ping-pong partner).  Returns sum_j d_j in *matvecs (host). */
int chase_filter(const void* A, int64_t lda, void* V, int64_t ldv, void* W, int64_t ldw, int64_t N,
                 int64_t n, const int32_t* degs, double c, double e, double mu_1, int64_t* matvecs,
                 chase_stream_t stream);

/* Allocation-free chase_filter, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, layout and result as chase_filter;
 * W stays the caller's ping-pong buffer.  The split-K tail's partial tiles
 * and counters live in one fixed device array of the library (the scratch:
 * CHASE_FILTER_NOALLOC_SEGMENTS partial 128 x 128 complex128 tiles plus 4160
 * bytes of counters, 64 MiB + 4160 B, chase_filter_noalloc_scratch_bytes()),
 * which every GPU the library runs on holds until the process ends; its
 * address is looked up on the first call on each device.  No device memory
 * is allocated or freed.  Every call on a GPU shares that GPU's scratch, and
 * the counters are cleared by a fill kernel at the start of each call: calls
 * that overlap on one GPU (different streams, threads or processes) race;
 * calls on one stream are ordered.  The work is enqueued on stream and the
 * call returns without waiting (*matvecs, host, is set at once).  The tail
 * split of every step is planned within the scratch, so every N and n is
 * accepted; a step whose split would not fit is rejected with -12 and a
 * message in chase_last_error().  Other statuses as chase_filter
 * (3: HIP error, e.g. the scratch's address could not be found). */
#define CHASE_FILTER_NOALLOC_SEGMENTS 256
int chase_filter_noalloc(const void* A, int64_t lda, void* V, int64_t ldv, void* W, int64_t ldw, int64_t N,
                         int64_t n, const int32_t* degs, double c, double e, double mu_1, int64_t* matvecs,
                         chase_stream_t stream);
/* Bytes of the scratch array of chase_filter_noalloc. */
int64_t chase_filter_noalloc_scratch_bytes(void);

/* 1D-CAQR (Alg. 4): V (N x n) is replaced by an orthonormal basis of its
 * span with the variant chosen from cond (or forced, CHASE_QR_*).
 * *variant (host) receives the variant that succeeded (after escalation
 * CholQR1/2 -> shifted CholQR2 -> Householder). */
int chase_caqr(void* V, int64_t ldv, int64_t N, int64_t n, double cond, int32_t force,
               int32_t* variant, chase_stream_t stream);

/* chase_caqr for a real block (float64, N x n, n <= N): the real solve's own
 * route, the block read as complex row pairs (an odd order gets one zero
 * row), Gram and quotient products keeping the real part, and the
 * Householder branch on the block widened to complex128 with zero imaginary
 * parts (LAPACK's real Q).  Allocates its workspace per call (2 on
 * failure).  -1 null/unaligned V, -2 ldv < N, -3 N < 2, -4 n outside
 * [1, N], -6 bad force. */
int chase_caqr_real(double* V, int64_t ldv, int64_t N, int64_t n, double cond, int32_t force,
                    int32_t* variant, chase_stream_t stream);

/* The low-precision filter of the mixed solve (a column on the FP32 or the
 * BF16x3 rung), as one call: the result approximates chase_filter's
 * p_{d_j}(H) v_j (Eq. 1 with the same scaled coefficients) with FP32
 * accumulation.
 *   precision  CHASE_FP32_MIXED: complex64 copies of H and of the block,
 *              FP32 matrix products; CHASE_BF16X3_MIXED: the four bfloat16
 *              planes of H and of each iterate, three bfloat16 products per
 *              real product (hi hi + hi lo + lo hi), FP32 accumulation
 *   A (device) N x N complex128, read only; V (device) N x n complex128,
 *   in/out (widened back to complex128 as each column reaches its degree);
 *   degs (host) n even degrees >= 2, ascending; *matvecs (host) sum_j d_j.
 *   n = 0 is a no-op (0 MatVecs, nothing allocated), as for chase_filter.
 * The copies of H (8 N^2 bytes for FP32, four bfloat16 planes for BF16x3)
 * and the complex64 blocks are allocated per call (2 on failure).
 * -1 null/unaligned A, -2 lda < N, -3 null/unaligned V, -4 ldv < N,
 * -5 N < 2, -6 n outside [0, N], -7 bad degrees, -9 e <= 0, -11 precision. */
int chase_filter_lowp(const void* A, int64_t lda, void* V, int64_t ldv, int64_t N, int64_t n,
                      const int32_t* degs, double c, double e, double mu_1, int32_t precision,
                      int64_t* matvecs, chase_stream_t stream);

/* Rayleigh-Ritz (Alg. 2): Q (N x n, orthonormal) -> Ritz values theta
 * (host, n, ascending) and Ritz vectors written over Q; resid (host, n)
 * receives ||H x_j - theta_j x_j||. */
int chase_rayleigh_ritz(const void* A, int64_t lda, void* Q, int64_t ldq, int64_t N, int64_t n,
                        double* theta, double* resid, chase_stream_t stream);

/* The small eigensolve of Rayleigh-Ritz (Alg. 2: the n x n Hermitian
 * quotient; Sec. 3.1's dense solver step), as chase_solve runs it: two-sided
 * block Jacobi on the GPU (blocks of 16, pairs of blocks diagonalised in
 * LDS by cyclic complex plane rotations, the 32 x 32 products applied to the
 * whole matrix and to the eigenvector accumulator), until the largest
 * off-diagonal entry of a sweep is below 1e-10 max|G_ii| (the sweep then
 * ends at rounding level).
 *   G (device) n x n, leading dimension ldg >= n, column-major complex128:
 *   the lower triangle is read (the diagonal's imaginary parts are taken as
 *   zero); on return G holds the orthonormal eigenvectors, column j for
 *   theta[j].  A real symmetric G (zero imaginary parts) gets real
 *   eigenvectors.  theta (host) n eigenvalues, ascending.  *sweeps (host,
 *   nullable) the number of sweeps made.
 * Workspace (2 (n rounded up to 32)^2 complex128 and less than 1 MiB more)
 * is allocated per call (2 on failure).  Host-synchronous.
 * -1 null/unaligned G, -2 ldg < n, -3 n outside [1, 65536], -4 null theta;
 * 4 non-finite entries (or no convergence in 40 sweeps). */
int chase_heev(void* G, int64_t ldg, int64_t n, double* theta, int32_t* sweeps, chase_stream_t stream);

/* Lanczos bounds (reading of Alg. 1's first line): (b_sup, mu_1, mu_ne,
 * norm_est) into out[4] (host) from nstarts runs of ksteps. */
int chase_lanczos(const void* A, int64_t lda, int64_t N, const void* starts, int64_t ld_starts,
                  int32_t nstarts, int32_t ksteps, int32_t ne, double* out, chase_stream_t stream);

/* Alg. 5: condition-number estimate (host computation). */
double chase_cond_est(const double* lam, double c, double e, const int32_t* degs, int32_t ne,
                      int32_t locked);

/* Per-vector filter degrees of Alg. 2's degree optimisation (host
 * computation, the solve's own routine): for each of the n pairs, the
 * number of Chebyshev steps that takes resd[j] below tol_abs at the growth
 * rate rho((lam[j] - c) / e), plus `extra`, clamped to [2, max_deg] and
 * rounded up to even; max_deg inside the damped interval or for a
 * non-finite residual.  resd, lam, degs (host) n entries each.  Returns -1
 * for a null array, -3 for n < 0, -5 for e <= 0 or tol_abs <= 0, -7 for an
 * odd or too small max_deg or a negative extra. */
int chase_degree_opt(const double* resd, const double* lam, int32_t n, double c, double e, double tol_abs,
                     int32_t max_deg, int32_t extra, int32_t* degs);

/* ---- per-iteration trace (Sec. 4.2 and 4.3: CondEst against the computed
 * condition number of the filtered vectors, QR variant and phase times per
 * outer iteration) ----------------------------------------------------------- */
#define CHASE_TRACE_MAX 256
typedef struct {
  int32_t iteration;       /* 1-based outer iteration */
  int32_t locked;          /* pairs locked when the iteration started */
  int32_t n_active;        /* columns filtered */
  int32_t qr_variant;      /* CHASE_QR_* that produced the basis (after escalation) */
  int64_t filter_matvecs;  /* sum of this iteration's filter degrees */
  double kappa_est;        /* Alg. 5 estimate for the filtered block */
  /* Trace level 2, else NaN: sigma_max / sigma_min of the n_e columns 1D-CAQR
   * receives (locked and filtered); of the filtered columns alone; of all n_e
   * columns scaled to unit norm (CholeskyQR is invariant to column scaling,
   * so this is the figure its accuracy depends on). */
  double kappa_com, kappa_com_active, kappa_com_equil;
  double t_filter, t_qr, t_rr;  /* seconds, HIP events on the solve's stream */
  int32_t eig_sweeps;      /* block-Jacobi sweeps of this iteration's quotient eigensolve */
  int32_t pad0;
} chase_trace_t;

/* Trace the next chase_solve calls on h: level 0 off (default), 1 records a
 * chase_trace_t per outer iteration, 2 also computes the kappa_com figures
 * from singular values of the block before each CAQR (Householder QR of an
 * N x n_e copy, then the singular values of R as the eigenvalues of
 * [[0, R], [R^H, 0]] by the block-Jacobi eigensolver: expensive, for studies
 * only; the buffers are allocated on the first such solve and the iteration
 * is not changed).  At most CHASE_TRACE_MAX
 * iterations are kept.  Returns -1 for a null handle, -2 for a bad level. */
int chase_set_trace(chase_handle_t h, int32_t level);

/* Copies up to cap records of the last traced solve on h to out (host);
 * *count (host) receives the number copied. */
int chase_get_trace(chase_handle_t h, chase_trace_t* out, int32_t cap, int32_t* count);

/* The active columns of one traced iteration, in the order they were
 * filtered (trace level >= 1). */
typedef struct {
  int32_t origin;  /* the pair's rank in ascending Ritz value in the previous
                      iteration's Rayleigh-Ritz output (its column index in
                      the first iteration) */
  int32_t rung;    /* precision of its filter: 0 FP64, 1 FP32, 2 BF16x3 */
  int32_t degree;  /* its filter degree */
  int32_t pad0;
  double ritz;     /* its Ritz value from the previous iteration (0 in the first) */
  double resid;    /* its FP64 residual norm from the previous iteration (inf in the first) */
} chase_trace_column_t;

/* Copies up to cap column records of iteration `iteration` (1-based) of the
 * last traced solve on h to out (host); *count (host) receives the number
 * copied.  -1 null handle, -2 no such traced iteration, -4 cap < 0 or a
 * null out with cap > 0. */
int chase_get_trace_columns(chase_handle_t h, int32_t iteration, chase_trace_column_t* out, int32_t cap,
                            int32_t* count);

const char* chase_status_string(int status);
const char* chase_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CHASE_HIP_H */
