// Kernels of the ChASE loop other than the big GEMMs: blocked Cholesky and
// triangular inverse of the n_e x n_e Gram matrix (Alg. 3 / Alg. 4), the
// s-CholeskyQR2 shift (Alg. 4), column residual norms (Alg. 2 residual),
// column permutations (locking, sort by degree), Lanczos (spectral bounds)
// and small helpers.  Everything is column-major complex128 unless noted.
#include "common.hpp"
#include "kernels.hpp"

#include <cmath>

namespace chase {

namespace {

struct alignas(16) zv {
  double re, im;
};

__device__ __forceinline__ zv zmul(zv a, zv b) { return zv{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ zv zmulc(zv a, zv b) {  // a * conj(b)
  return zv{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

constexpr int NB = 64;  // panel width of the blocked Cholesky / inverse

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  // wave reduction, then across waves through LDS
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    red[NT / 64] = s;
  }
  __syncthreads();
  return red[NT / 64];
}

__global__ void init_int_kernel(int* p, int v) { *p = v; }

// ---- Cholesky --------------------------------------------------------------

// Unblocked Cholesky of the jb x jb diagonal block (lower), in LDS.
__global__ __launch_bounds__(256) void potrf_diag_kernel(zv* G, int64_t ld, int jb, int* info, int64_t j0) {
  __shared__ zv L[NB][NB + 1];  // L[c][r] = G[r][c]
  __shared__ int fail;
  const int t = threadIdx.x;
  if (*info != 0) return;  // an earlier panel failed: leave the rest untouched
  for (int idx = t; idx < jb * jb; idx += 256) {
    int r = idx % jb, c = idx / jb;
    L[c][r] = (r >= c) ? G[r + c * ld] : zv{0.0, 0.0};
  }
  if (t == 0) fail = 0;
  __syncthreads();
  for (int c = 0; c < jb; ++c) {
    if (t == 0) {
      double d = L[c][c].re;
      if (!(d > 0.0) || !isfinite(d)) {
        fail = c + 1;
      } else {
        L[c][c] = zv{sqrt(d), 0.0};
      }
    }
    __syncthreads();
    if (fail) break;
    const double inv = 1.0 / L[c][c].re;
    for (int r = c + 1 + t; r < jb; r += 256) {
      L[c][r].re *= inv;
      L[c][r].im *= inv;
    }
    __syncthreads();
    const int w = jb - c - 1;
    for (int idx = t; idx < w * w; idx += 256) {
      int r = c + 1 + idx % w, q = c + 1 + idx / w;
      if (r >= q) {
        zv p = zmulc(L[c][r], L[c][q]);
        L[q][r].re -= p.re;
        L[q][r].im -= p.im;
      }
    }
    __syncthreads();
  }
  if (fail) {
    if (t == 0) *info = (int)j0 + fail;
    return;
  }
  for (int idx = t; idx < jb * jb; idx += 256) {
    int r = idx % jb, c = idx / jb;
    if (r >= c) G[r + c * ld] = L[c][r];
  }
}

// Panel solve P <- P L11^{-H}: row r of P solves x L11^H = p by forward
// substitution.  One thread per row; L11 staged in LDS.
__global__ __launch_bounds__(64) void potrf_panel_kernel(const zv* L11, zv* P, int64_t ld, int64_t rows, int jb,
                                                         const int* info) {
  __shared__ zv L[NB][NB + 1];  // L[c][s] = L11[c][s] (row c, col s), lower
  if (*info != 0) return;
  for (int idx = threadIdx.x; idx < jb * jb; idx += 64) {
    int c = idx % jb, s = idx / jb;
    L[c][s] = (c >= s) ? L11[c + s * ld] : zv{0.0, 0.0};
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (r >= rows) return;
  for (int c = 0; c < jb; ++c) {
    zv acc = P[r + c * ld];
    for (int s = 0; s < c; ++s) {
      zv p = zmulc(P[r + s * ld], L[c][s]);  // x_s conj(L[c][s])
      acc.re -= p.re;
      acc.im -= p.im;
    }
    const double inv = 1.0 / L[c][c].re;
    P[r + c * ld] = zv{acc.re * inv, acc.im * inv};
  }
}

// ---- triangular inverse -----------------------------------------------------

// Inverse of each NB x NB diagonal block of lower-triangular L; thread c
// computes column c by forward substitution.
__global__ __launch_bounds__(64) void trtri_diag_kernel(const zv* L, int64_t ldl, zv* X, int64_t ldx, int64_t n) {
  __shared__ zv Ls[NB][NB + 1];  // Ls[r][s] = L[r][s]
  __shared__ zv Xs[NB][NB + 1];  // Xs[c][r] = X[r][c]
  const int64_t off = (int64_t)blockIdx.x * NB;
  const int jb = (int)((n - off) < NB ? (n - off) : NB);
  for (int idx = threadIdx.x; idx < jb * jb; idx += 64) {
    int r = idx % jb, s = idx / jb;
    Ls[r][s] = (r >= s) ? L[(off + r) + (off + s) * ldl] : zv{0.0, 0.0};
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < jb) {
    for (int r = 0; r < c; ++r) Xs[c][r] = zv{0.0, 0.0};
    {
      zv d = Ls[c][c];
      double den = d.re * d.re + d.im * d.im;
      Xs[c][c] = zv{d.re / den, -d.im / den};
    }
    for (int r = c + 1; r < jb; ++r) {
      zv acc{0.0, 0.0};
      for (int s = c; s < r; ++s) {
        zv p = zmul(Ls[r][s], Xs[c][s]);
        acc.re += p.re;
        acc.im += p.im;
      }
      zv d = Ls[r][r];
      double den = d.re * d.re + d.im * d.im;
      // -acc / d
      zv q{-(acc.re * d.re + acc.im * d.im) / den, -(acc.im * d.re - acc.re * d.im) / den};
      Xs[c][r] = q;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < jb * jb; idx += 64) {
    int r = idx % jb, cc = idx / jb;
    X[(off + r) + (off + cc) * ldx] = Xs[cc][r];
  }
}

__global__ void zero_upper_kernel(zv* G, int64_t ld, int64_t n) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  int64_t r = idx % n, c = idx / n;
  if (r < c) G[r + c * ld] = zv{0.0, 0.0};
}

__global__ void mirror_lower_kernel(zv* G, int64_t ld, int64_t n) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  int64_t r = idx % n, c = idx / n;
  if (r < c) {
    zv v = G[c + r * ld];
    G[r + c * ld] = zv{v.re, -v.im};
  }
}

// G += s I with s = 11 (m n + n (n + 1)) u trace(G) (Alg. 4 shift).
__global__ __launch_bounds__(256) void cholqr_shift_kernel(zv* G, int64_t ld, int64_t n, int64_t m, double* s_out) {
  __shared__ double red[8];
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) acc += G[j + j * ld].re;
  const double fro2 = block_sum<256>(acc, red);
  const double u = 1.1102230246251565e-16;  // 2^-53
  const double s = 11.0 * ((double)m * (double)n + (double)n * (double)(n + 1)) * u * fro2;
  for (int64_t j = threadIdx.x; j < n; j += 256) G[j + j * ld].re += s;
  if (threadIdx.x == 0) *s_out = s;
}

// ---- residuals, permutations, copies ---------------------------------------

__global__ __launch_bounds__(256) void residual_kernel(const zv* Y, int64_t ldy, const zv* X, int64_t ldx,
                                                       const double* theta, int64_t N, double* out) {
  __shared__ double red[8];
  const int64_t j = blockIdx.x;
  const double th = theta[j];
  double acc = 0.0;
  for (int64_t m = threadIdx.x; m < N; m += 256) {
    zv y = Y[m + j * ldy], x = X[m + j * ldx];
    double dr = y.re - th * x.re, di = y.im - th * x.im;
    acc += dr * dr + di * di;
  }
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) out[j] = sqrt(s);
}

__global__ void gather_kernel(const zv* src, int64_t lds, zv* dst, int64_t ldd, const int* perm, int64_t N) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= N) return;
  dst[m + j * ldd] = src[m + (int64_t)perm[j] * lds];
}

__global__ void copy_kernel(const zv* src, int64_t lds, zv* dst, int64_t ldd, int64_t N) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= N) return;
  dst[m + j * ldd] = src[m + j * lds];
}

__global__ void scale_kernel(const zv* X, int64_t ldx, const double* g, zv* out, int64_t ldo, int64_t N) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= N) return;
  zv v = X[m + j * ldx];
  const double s = g[j];
  out[m + j * ldo] = zv{s * v.re, s * v.im};
}

__global__ void finite_kernel(const double* x, int64_t n, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) *flag = 1;
}

__global__ void z2c_kernel(const zv* src, int64_t lds, c32* dst, int64_t ldd, int64_t N) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= N) return;
  zv v = src[m + j * lds];
  dst[m + j * ldd] = c32{(float)v.re, (float)v.im};
}

__global__ void c2z_kernel(const c32* src, int64_t lds, zv* dst, int64_t ldd, int64_t N, double scale) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= N) return;
  c32 v = src[m + j * lds];
  dst[m + j * ldd] = zv{(double)v.re * scale, (double)v.im * scale};
}

// real M x n block <-> complex128 block with zero imaginary parts
__global__ void widen_real_kernel(const double* R, int64_t ldr, zv* X, int64_t ldx, int64_t M) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= M) return;
  X[m + j * ldx] = zv{R[m + j * ldr], 0.0};
}

__global__ void real_part_block_kernel(const zv* X, int64_t ldx, double* R, int64_t ldr, int64_t M) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= M) return;
  R[m + j * ldr] = X[m + j * ldx].re;
}

// ---- Lanczos ----------------------------------------------------------------

// W[m, c] = sum_k A[m, k] V[k, c] = sum_k conj(A[k, m]) V[k, c]  (A Hermitian):
// one wave per output row reads column m of A contiguously.
// H's element type HT is complex128 (zv) or complex64 (c32, the complex64
// variant); products accumulate in FP64 either way.
template <class HT>
__global__ __launch_bounds__(256) void hemv_kernel(const HT* A, int64_t lda, const zv* V, int64_t ldv, zv* W,
                                                   int64_t ldw, int64_t N, int nv) {
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= N) return;
  double ar[8] = {0, 0, 0, 0, 0, 0, 0, 0}, ai[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const HT* col = A + m * lda;
  for (int64_t k = lane; k < N; k += 64) {
    const zv a{(double)col[k].re, (double)col[k].im};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c < nv) {
        zv v = V[k + c * ldv];
        // conj(a) * v
        ar[c] += a.re * v.re + a.im * v.im;
        ai[c] += a.re * v.im - a.im * v.re;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (c < nv) {
      double r = ar[c], i = ai[c];
      for (int off = 32; off > 0; off >>= 1) {
        r += __shfl_down(r, off, 64);
        i += __shfl_down(i, off, 64);
      }
      if (lane == 0) W[m + c * ldw] = zv{r, i};
    }
  }
}

// Four Lanczos vectors at once (the batched starts): W[:, c] = H^H V[:, c].
// Each wave takes RPW columns of H (contiguous, coalesced) and each K chunk
// of V is staged in LDS once for the workgroup's 4 * RPW columns, so V is
// read from L2 once per workgroup instead of once per column (at one column
// per wave the re-reads of V outweighed the stream of H five to one).  H is
// read once from HBM.
template <class HT, int NV, int RPW>
__global__ __launch_bounds__(256) void hemv_panel_kernel(const HT* __restrict__ A, int64_t lda,
                                                         const zv* __restrict__ V, int64_t ldv, zv* W,
                                                         int64_t ldw, int64_t N) {
  constexpr int KC = 256;  // k per chunk
  __shared__ zv vs[NV][KC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t m0 = ((int64_t)blockIdx.x * 4 + wave) * RPW;  // first column of this wave
  double ar[RPW][NV], ai[RPW][NV];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int c = 0; c < NV; ++c) ar[r][c] = ai[r][c] = 0.0;
  for (int64_t k0 = 0; k0 < N; k0 += KC) {  // every wave takes part in the barriers
    __syncthreads();                         // the previous chunk has been used
    for (int e = threadIdx.x; e < NV * KC; e += 256) {
      const int c = e / KC, kk = e % KC;
      const int64_t k = k0 + kk;
      vs[c][kk] = k < N ? V[k + c * ldv] : zv{0.0, 0.0};
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KC / 64; ++u) {
      const int kk = u * 64 + lane;
      const int64_t k = k0 + kk;
      zv v[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) v[c] = vs[c][kk];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int64_t m = m0 + r;
        if (m < N && k < N) {
          const zv a{(double)A[k + m * lda].re, (double)A[k + m * lda].im};  // conj(a) v
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            ar[r][c] += a.re * v[c].re + a.im * v[c].im;
            ai[r][c] += a.re * v[c].im - a.im * v[c].re;
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double x = ar[r][c], y = ai[r][c];
      for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_down(x, off, 64);
        y += __shfl_down(y, off, 64);
      }
      const int64_t m = m0 + r;
      if (lane == 0 && m < N) W[m + c * ldw] = zv{x, y};
    }
}

__global__ __launch_bounds__(1024) void lanczos_init_kernel(const zv* S, int64_t ld, zv* V, zv* Vold, int64_t N) {
  __shared__ double red[17];
  const int64_t c = blockIdx.x;
  double acc = 0.0;
  for (int64_t m = threadIdx.x; m < N; m += 1024) {
    zv s = S[m + c * ld];
    acc += s.re * s.re + s.im * s.im;
  }
  const double nrm = sqrt(block_sum<1024>(acc, red));
  for (int64_t m = threadIdx.x; m < N; m += 1024) {
    zv s = S[m + c * ld];
    V[m + c * N] = zv{s.re / nrm, s.im / nrm};
    Vold[m + c * N] = zv{0.0, 0.0};
  }
}

// w = W - beta_{j-1} v_old; alpha = Re(v^H w); w -= alpha v; beta = ||w||;
// v_old <- v; v <- w / beta.  One block per vector; alpha/beta[c*ksteps + j].
__global__ __launch_bounds__(1024) void lanczos_step_kernel(zv* V, zv* Vold, zv* W, int64_t N, int step, int ksteps,
                                                            double* alpha, double* beta) {
  __shared__ double red[17];
  const int64_t c = blockIdx.x;
  zv* v = V + c * N;
  zv* vo = Vold + c * N;
  zv* w = W + c * N;
  const double bold = step > 0 ? beta[c * ksteps + step - 1] : 0.0;
  double acc = 0.0;
  for (int64_t m = threadIdx.x; m < N; m += 1024) {
    zv x = v[m], y = w[m], z = vo[m];
    y.re -= bold * z.re;
    y.im -= bold * z.im;
    w[m] = y;
    acc += x.re * y.re + x.im * y.im;  // Re(conj(x) y)
  }
  const double a = block_sum<1024>(acc, red);
  acc = 0.0;
  for (int64_t m = threadIdx.x; m < N; m += 1024) {
    zv x = v[m], y = w[m];
    y.re -= a * x.re;
    y.im -= a * x.im;
    w[m] = y;
    acc += y.re * y.re + y.im * y.im;
  }
  const double b = sqrt(block_sum<1024>(acc, red));
  if (threadIdx.x == 0) {
    alpha[c * ksteps + step] = a;
    beta[c * ksteps + step] = b;
  }
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  for (int64_t m = threadIdx.x; m < N; m += 1024) {
    zv x = v[m], y = w[m];
    vo[m] = x;
    v[m] = zv{y.re * inv, y.im * inv};
  }
}

// ---- real symmetric problems ------------------------------------------------

// W[:, c] = H V[:, c] (c < nv <= 8) for real symmetric H of order N: column m
// of H is row m, so one wave per output row reads it coalesced.  Rows
// N .. rows_out - 1 of W are written as zero (the padding row of the row-pair
// layout).
__global__ __launch_bounds__(256) void symv_kernel(const double* __restrict__ H, int64_t ldh,
                                                   const double* __restrict__ V, int64_t ldv, double* W,
                                                   int64_t ldw, int64_t N, int64_t rows_out, int nv) {
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= rows_out) return;  // whole waves
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (m < N) {
    const double* col = H + m * ldh;
    for (int64_t k = lane; k < N; k += 64) {
      const double h = col[k];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < nv) acc[c] += h * V[k + c * ldv];
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (c >= nv) break;
    double x = acc[c];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) W[m + c * ldw] = x;
  }
}

// dst (rows_dst x cols_dst) = src (rows_src x cols_src) zero-extended.
__global__ void dcopy_pad_kernel(const double* src, int64_t lds, int64_t rows_src, int64_t cols_src, double* dst,
                                 int64_t ldd, int64_t rows_dst) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= rows_dst) return;
  dst[m + j * ldd] = (m < rows_src && j < cols_src) ? src[m + j * lds] : 0.0;
}

// ---- counter-based Gaussian fill (splitmix64 + Box-Muller) ------------------

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void gaussian_kernel(zv* X, int64_t ld, int64_t N, uint64_t seed) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= N) return;
  const uint64_t idx = (uint64_t)(m + j * N);
  const uint64_t a = splitmix64(seed ^ (2 * idx)), b = splitmix64(seed ^ (2 * idx + 1));
  const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
  const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);          // [0, 1)
  const double r = sqrt(-2.0 * log(u1)) * 0.7071067811865476;
  double sn, cs;
  sincos(6.283185307179586 * u2, &sn, &cs);
  X[m + j * ld] = zv{r * cs, r * sn};
}

}  // namespace

// ============================================================================

int potrf_lower(z64* G, int64_t ld, int64_t n, int* info, z64* /*ws*/, hipStream_t s) {
  hipLaunchKernelGGL(init_int_kernel, dim3(1), dim3(1), 0, s, info, 0);
  CHASE_CHK_LAUNCH();
  zv* g = reinterpret_cast<zv*>(G);
  for (int64_t j0 = 0; j0 < n; j0 += NB) {
    const int jb = (int)((n - j0) < NB ? (n - j0) : NB);
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, g + j0 + j0 * ld, ld, jb, info, j0);
    CHASE_CHK_LAUNCH();
    const int64_t rem = n - j0 - jb;
    if (rem <= 0) break;
    hipLaunchKernelGGL(potrf_panel_kernel, dim3((unsigned)cdiv(rem, 64)), dim3(64), 0, s,
                       g + j0 + j0 * ld, g + (j0 + jb) + j0 * ld, ld, rem, jb, info);
    CHASE_CHK_LAUNCH();
    GemmArgs a;
    a.M = rem; a.N = rem; a.K = jb;
    a.A = G + (j0 + jb) + j0 * ld; a.lda = ld;
    a.B = G + (j0 + jb) + j0 * ld; a.ldb = ld;
    a.Y = G + (j0 + jb) + (j0 + jb) * ld; a.ldy = ld;
    a.alpha = -1.0; a.beta = 1.0;
    a.lower_only = 1;
    int st = zgemm_launch(0, 1, a, s);
    if (st) return st;
  }
  return kOk;
}

static int trtri_rec(const z64* L, int64_t ldl, z64* X, int64_t ldx, int64_t off, int64_t size, z64* tmp,
                     int64_t ldt, hipStream_t s) {
  if (size <= NB) return kOk;
  const int64_t n1 = NB * cdiv(cdiv(size, NB), 2);
  const int64_t n2 = size - n1;
  int st = trtri_rec(L, ldl, X, ldx, off, n1, tmp, ldt, s);
  if (st) return st;
  st = trtri_rec(L, ldl, X, ldx, off + n1, n2, tmp, ldt, s);
  if (st) return st;
  GemmArgs a;  // T = L21 X11
  a.M = n2; a.N = n1; a.K = n1;
  a.A = L + (off + n1) + off * ldl; a.lda = ldl;
  a.B = X + off + off * ldx; a.ldb = ldx;
  a.Y = tmp; a.ldy = ldt;
  st = zgemm_launch(0, 0, a, s);
  if (st) return st;
  GemmArgs b;  // X21 = -X22 T
  b.M = n2; b.N = n1; b.K = n2;
  b.A = X + (off + n1) + (off + n1) * ldx; b.lda = ldx;
  b.B = tmp; b.ldb = ldt;
  b.Y = X + (off + n1) + off * ldx; b.ldy = ldx;
  b.alpha = -1.0;
  return zgemm_launch(0, 0, b, s);
}

int trtri_lower(const z64* L, int64_t ldl, z64* Linv, int64_t ldi, int64_t n, z64* tmp, hipStream_t s) {
  if (n <= 0) return kOk;
  hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)cdiv(n * n, 256)), dim3(256), 0, s,
                     reinterpret_cast<zv*>(Linv), ldi, n);
  CHASE_CHK_LAUNCH();
  hipLaunchKernelGGL(trtri_diag_kernel, dim3((unsigned)cdiv(n, NB)), dim3(64), 0, s,
                     reinterpret_cast<const zv*>(L), ldl, reinterpret_cast<zv*>(Linv), ldi, n);
  CHASE_CHK_LAUNCH();
  return trtri_rec(L, ldl, Linv, ldi, 0, n, tmp, n, s);
}

int add_cholqr_shift(z64* G, int64_t ld, int64_t n, int64_t m, double* shift_out, hipStream_t s) {
  hipLaunchKernelGGL(cholqr_shift_kernel, dim3(1), dim3(256), 0, s, reinterpret_cast<zv*>(G), ld, n, m, shift_out);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int zero_upper(z64* G, int64_t ld, int64_t n, hipStream_t s) {
  if (n <= 0) return kOk;
  hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)cdiv(n * n, 256)), dim3(256), 0, s,
                     reinterpret_cast<zv*>(G), ld, n);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int hermitian_mirror_lower(z64* G, int64_t ld, int64_t n, hipStream_t s) {
  if (n <= 0) return kOk;
  hipLaunchKernelGGL(mirror_lower_kernel, dim3((unsigned)cdiv(n * n, 256)), dim3(256), 0, s,
                     reinterpret_cast<zv*>(G), ld, n);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int residual_norms(const z64* Y, int64_t ldy, const z64* X, int64_t ldx, const double* theta, int64_t N,
                   int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return kOk;
  hipLaunchKernelGGL(residual_kernel, dim3((unsigned)n), dim3(256), 0, s, reinterpret_cast<const zv*>(Y), ldy,
                     reinterpret_cast<const zv*>(X), ldx, theta, N, out);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int gather_columns(const z64* src, int64_t lds, z64* dst, int64_t ldd, const int* perm, int64_t N, int64_t n,
                   hipStream_t s) {
  if (n <= 0 || N <= 0) return kOk;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)cdiv(N, 256), (unsigned)n), dim3(256), 0, s,
                     reinterpret_cast<const zv*>(src), lds, reinterpret_cast<zv*>(dst), ldd, perm, N);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int copy_columns(const z64* src, int64_t lds, z64* dst, int64_t ldd, int64_t N, int64_t n, hipStream_t s) {
  if (n <= 0 || N <= 0) return kOk;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)cdiv(N, 256), (unsigned)n), dim3(256), 0, s,
                     reinterpret_cast<const zv*>(src), lds, reinterpret_cast<zv*>(dst), ldd, N);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int scale_columns(const z64* X, int64_t ldx, const double* g, z64* out, int64_t ldo, int64_t N, int64_t n,
                  hipStream_t s) {
  if (n <= 0 || N <= 0) return kOk;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)cdiv(N, 256), (unsigned)n), dim3(256), 0, s,
                     reinterpret_cast<const zv*>(X), ldx, g, reinterpret_cast<zv*>(out), ldo, N);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int check_finite(const double* x, int64_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(init_int_kernel, dim3(1), dim3(1), 0, s, flag, 0);
  CHASE_CHK_LAUNCH();
  if (n <= 0) return kOk;
  hipLaunchKernelGGL(finite_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, x, n, flag);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int convert_z_to_c(const z64* src, int64_t lds, c32* dst, int64_t ldd, int64_t N, int64_t n, hipStream_t s) {
  if (n <= 0 || N <= 0) return kOk;
  hipLaunchKernelGGL(z2c_kernel, dim3((unsigned)cdiv(N, 256), (unsigned)n), dim3(256), 0, s,
                     reinterpret_cast<const zv*>(src), lds, dst, ldd, N);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int convert_c_to_z(const c32* src, int64_t lds, z64* dst, int64_t ldd, int64_t N, int64_t n, hipStream_t s,
                   double scale) {
  if (n <= 0 || N <= 0) return kOk;
  hipLaunchKernelGGL(c2z_kernel, dim3((unsigned)cdiv(N, 256), (unsigned)n), dim3(256), 0, s, src, lds,
                     reinterpret_cast<zv*>(dst), ldd, N, scale);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int widen_real_block(const double* R, int64_t ldr, z64* X, int64_t ldx, int64_t M, int64_t n, hipStream_t s) {
  if (n <= 0 || M <= 0) return kOk;
  hipLaunchKernelGGL(widen_real_kernel, dim3((unsigned)cdiv(M, 256), (unsigned)n), dim3(256), 0, s, R, ldr,
                     reinterpret_cast<zv*>(X), ldx, M);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int real_part_block(const z64* X, int64_t ldx, double* R, int64_t ldr, int64_t M, int64_t n, hipStream_t s) {
  if (n <= 0 || M <= 0) return kOk;
  hipLaunchKernelGGL(real_part_block_kernel, dim3((unsigned)cdiv(M, 256), (unsigned)n), dim3(256), 0, s,
                     reinterpret_cast<const zv*>(X), ldx, R, ldr, M);
  CHASE_CHK_LAUNCH();
  return kOk;
}

template <class HT>
static int hemv_any(const HT* A, int64_t lda, const z64* V, int64_t ldv, z64* W, int64_t ldw, int64_t N, int nv,
                    hipStream_t s) {
  if (nv < 1 || nv > 8) return -1;
  if (nv == 4) {
    constexpr int RPW = 4;
    hipLaunchKernelGGL((hemv_panel_kernel<HT, 4, RPW>), dim3((unsigned)cdiv(N, 4 * RPW)), dim3(256), 0, s, A, lda,
                       reinterpret_cast<const zv*>(V), ldv, reinterpret_cast<zv*>(W), ldw, N);
    CHASE_CHK_LAUNCH();
    return kOk;
  }
  hipLaunchKernelGGL(hemv_kernel<HT>, dim3((unsigned)cdiv(N, 4)), dim3(256), 0, s, A, lda,
                     reinterpret_cast<const zv*>(V), ldv, reinterpret_cast<zv*>(W), ldw, N, nv);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int hemv_block(const z64* A, int64_t lda, const z64* V, int64_t ldv, z64* W, int64_t ldw, int64_t N, int nv,
               hipStream_t s) {
  return hemv_any(reinterpret_cast<const zv*>(A), lda, V, ldv, W, ldw, N, nv, s);
}

int hemv_block_c64(const c32* A, int64_t lda, const z64* V, int64_t ldv, z64* W, int64_t ldw, int64_t N, int nv,
                   hipStream_t s) {
  return hemv_any(A, lda, V, ldv, W, ldw, N, nv, s);
}

int symv_block(const double* H, int64_t ldh, const double* V, int64_t ldv, double* W, int64_t ldw, int64_t N,
               int64_t rows_out, int nv, hipStream_t s) {
  if (nv < 1 || nv > 8 || rows_out < N) return -1;
  if (rows_out <= 0) return kOk;
  hipLaunchKernelGGL(symv_kernel, dim3((unsigned)cdiv(rows_out, 4)), dim3(256), 0, s, H, ldh, V, ldv, W, ldw, N,
                     rows_out, nv);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int dcopy_pad(const double* src, int64_t lds, int64_t rows_src, int64_t cols_src, double* dst, int64_t ldd,
              int64_t rows_dst, int64_t cols_dst, hipStream_t s) {
  if (rows_dst <= 0 || cols_dst <= 0) return kOk;
  hipLaunchKernelGGL(dcopy_pad_kernel, dim3((unsigned)cdiv(rows_dst, 256), (unsigned)cols_dst), dim3(256), 0, s,
                     src, lds, rows_src, cols_src, dst, ldd, rows_dst);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int lanczos_init(const z64* starts, int64_t ld, z64* V, z64* Vold, int64_t N, int nv, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_init_kernel, dim3(nv), dim3(1024), 0, s, reinterpret_cast<const zv*>(starts), ld,
                     reinterpret_cast<zv*>(V), reinterpret_cast<zv*>(Vold), N);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int lanczos_step(z64* V, z64* Vold, z64* W, int64_t N, int nv, int step, int ksteps, double* alpha, double* beta,
                 hipStream_t s) {
  hipLaunchKernelGGL(lanczos_step_kernel, dim3(nv), dim3(1024), 0, s, reinterpret_cast<zv*>(V),
                     reinterpret_cast<zv*>(Vold), reinterpret_cast<zv*>(W), N, step, ksteps, alpha, beta);
  CHASE_CHK_LAUNCH();
  return kOk;
}

int fill_gaussian(z64* X, int64_t ld, int64_t N, int64_t n, uint64_t seed, hipStream_t s) {
  if (n <= 0 || N <= 0) return kOk;
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)cdiv(N, 256), (unsigned)n), dim3(256), 0, s,
                     reinterpret_cast<zv*>(X), ld, N, seed);
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
