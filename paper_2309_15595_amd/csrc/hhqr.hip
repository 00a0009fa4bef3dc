// Householder QR of a tall complex block and its explicit unitary factor:
// the last-resort branch of 1D-CAQR (Alg. 4), taken when shifted
// CholeskyQR2 breaks down.  Conventions are LAPACK's (geqrf / ungqr), so Q
// is the one a LAPACK Householder QR returns, up to rounding:
//   reflector H = I - tau v v^H with v_0 = 1, beta real,
//   beta = -sign(Re alpha) ||(alpha, x)||, tau = (beta - alpha) / beta,
//   v = x / (alpha - beta); the trailing columns get H^H.
//
// Panels of HB = 32 columns.  One column's reflector takes two launches over
// the rows below its diagonal, spread over many workgroups: the first forms
// per-workgroup partial sums of |x_i|^2 and of conj(x_i) A[i, k] for the
// panel's later columns k; the second has every workgroup sum the partials in
// the same order, form beta, tau and w_k = v^H A_k, scale its rows of x into
// v and apply (I - conj(tau) v v^H) to them.  Row j itself is read from a
// copy taken by the first launch, so no workgroup reads what another writes.
// The trailing matrix then gets the block reflector (I - V T V^H)^H through
// three GEMMs, with T built as in LAPACK's larft (forward, columnwise); Q is
// accumulated backwards over the panels with the same GEMMs.
#include "common.hpp"
#include "kernels.hpp"

#include <vector>

namespace chase {

namespace {

struct alignas(16) zv {
  double re, im;
};

constexpr int HB = kHouseholderPanel;
constexpr int NT = 256;
constexpr int PS = 2 * HB;  // doubles per workgroup partial: |x|^2 and HB - 1 complex products

__device__ __forceinline__ zv zconj_mul(zv a, zv b) {  // conj(a) * b
  return zv{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__device__ __forceinline__ zv zmul(zv a, zv b) { return zv{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Rows j + 1 .. M - 1 split into nwg contiguous chunks.
__device__ __forceinline__ void hh_chunk(int64_t M, int64_t j, int nwg, int64_t* r0, int64_t* r1) {
  const int64_t rows = M - j - 1;
  const int64_t per = (rows + nwg - 1) / nwg;
  *r0 = j + 1 + (int64_t)blockIdx.x * per;
  *r1 = *r0 + per < M ? *r0 + per : M;
}

// Column j (global), later panel columns j + 1 .. jend - 1.
__global__ __launch_bounds__(NT) void hh_col_reduce(const zv* __restrict__ A, int64_t lda, int64_t M, int64_t j,
                                                    int64_t jend, int nwg, double* __restrict__ part,
                                                    zv* __restrict__ rowj) {
  __shared__ double red[NT / 64][PS];
  const int nk = (int)(jend - j - 1);
  int64_t r0, r1;
  hh_chunk(M, j, nwg, &r0, &r1);
  double sig = 0.0;
  zv s[HB - 1];
#pragma unroll
  for (int k = 0; k < HB - 1; ++k) s[k] = zv{0.0, 0.0};
  for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
    const zv x = A[i + j * lda];
    sig += x.re * x.re + x.im * x.im;
#pragma unroll
    for (int k = 0; k < HB - 1; ++k)
      if (k < nk) {
        const zv p = zconj_mul(x, A[i + (j + 1 + k) * lda]);
        s[k].re += p.re;
        s[k].im += p.im;
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave sums, then the workgroup's in a fixed order
  for (int off = 32; off > 0; off >>= 1) sig += __shfl_down(sig, off, 64);
#pragma unroll
  for (int k = 0; k < HB - 1; ++k)
    for (int off = 32; off > 0; off >>= 1) {
      s[k].re += __shfl_down(s[k].re, off, 64);
      s[k].im += __shfl_down(s[k].im, off, 64);
    }
  if (lane == 0) {
    red[wave][0] = sig;
#pragma unroll
    for (int k = 0; k < HB - 1; ++k) {
      red[wave][1 + 2 * k] = s[k].re;
      red[wave][2 + 2 * k] = s[k].im;
    }
  }
  __syncthreads();
  if (threadIdx.x < PS - 1) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w][threadIdx.x];
    part[(int64_t)blockIdx.x * PS + threadIdx.x] = t;
  }
  if (blockIdx.x == 0 && threadIdx.x <= nk) rowj[threadIdx.x] = A[j + (j + threadIdx.x) * lda];
}

__global__ __launch_bounds__(NT) void hh_col_apply(zv* __restrict__ A, int64_t lda, int64_t M, int64_t j,
                                                   int64_t jend, int nwg, const double* __restrict__ part,
                                                   const zv* __restrict__ rowj, zv* __restrict__ tau_out) {
  __shared__ double sum[PS];
  __shared__ zv w[HB];
  __shared__ zv sc[3];  // tau, scale, (beta, 0)
  const int nk = (int)(jend - j - 1);
  if (threadIdx.x < PS - 1) {
    double t = 0.0;
    for (int g = 0; g < nwg; ++g) t += part[(int64_t)g * PS + threadIdx.x];
    sum[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const zv alpha = rowj[0];
    const double xnorm = sqrt(sum[0]);
    zv tau{0.0, 0.0}, scale{0.0, 0.0};
    double beta = alpha.re;
    if (xnorm > 0.0 || alpha.im != 0.0) {
      const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + sum[0]);
      beta = alpha.re >= 0.0 ? -nrm : nrm;
      tau = zv{(beta - alpha.re) / beta, -alpha.im / beta};
      const zv d{alpha.re - beta, alpha.im};  // scale = 1 / (alpha - beta)
      const double dd = d.re * d.re + d.im * d.im;
      scale = zv{d.re / dd, -d.im / dd};
    }
    sc[0] = tau;
    sc[1] = scale;
    sc[2] = zv{beta, 0.0};
    // w_k = v^H A_k = A[j, k] + conj(scale) s_k
    for (int k = 0; k < nk; ++k) {
      const zv sk{sum[1 + 2 * k], sum[2 + 2 * k]};
      const zv t = zconj_mul(scale, sk);
      w[k] = zv{rowj[1 + k].re + t.re, rowj[1 + k].im + t.im};
    }
  }
  __syncthreads();
  const zv tau = sc[0], scale = sc[1];
  if (tau.re == 0.0 && tau.im == 0.0) {  // H = I
    if (blockIdx.x == 0 && threadIdx.x == 0) tau_out[j] = tau;
    return;
  }
  const zv ctau{tau.re, -tau.im};
  int64_t r0, r1;
  hh_chunk(M, j, nwg, &r0, &r1);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
    const zv v = zmul(scale, A[i + j * lda]);
    A[i + j * lda] = v;
    const zv cv = zmul(ctau, v);
    for (int k = 0; k < nk; ++k) {
      zv& a = A[i + (j + 1 + k) * lda];
      const zv p = zmul(cv, w[k]);
      a.re -= p.re;
      a.im -= p.im;
    }
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      A[j + j * lda] = sc[2];
      tau_out[j] = tau;
    }
    if (threadIdx.x < nk) {  // row j: A[j, k] - conj(tau) w_k
      const zv p = zmul(ctau, w[threadIdx.x]);
      const zv r = rowj[1 + threadIdx.x];
      A[j + (j + 1 + threadIdx.x) * lda] = zv{r.re - p.re, r.im - p.im};
    }
  }
}

// Explicit V of the panel at column j0 (jb columns, rows j0 .. M - 1):
// unit diagonal, zeros above, the stored reflectors below.
__global__ void hh_build_v(const zv* A, int64_t lda, int64_t M, int64_t j0, zv* V, int64_t ldv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= M - j0) return;
  zv v;
  if (r == c) v = zv{1.0, 0.0};
  else if (r < c) v = zv{0.0, 0.0};
  else v = A[j0 + r + (j0 + c) * lda];
  V[r + c * ldv] = v;
}

// T (jb x jb, upper triangular, ld HB) from G = V^H V and tau (larft).
__global__ __launch_bounds__(64) void hh_build_t(const zv* G, int64_t ldg, const zv* tau, int jb, zv* T) {
  __shared__ zv t[HB][HB + 1];  // t[row][col]
  __shared__ zv u[HB];
  const int r = threadIdx.x;
  for (int e = r; e < HB * HB; e += 64) t[e % HB][e / HB] = zv{0.0, 0.0};
  __syncthreads();
  for (int i = 0; i < jb; ++i) {
    const zv ti = tau[i];
    if (r < i) {  // u_r = -tau_i G[r, i]
      const zv p = zmul(ti, G[r + (int64_t)i * ldg]);
      u[r] = zv{-p.re, -p.im};
    }
    __syncthreads();
    if (r < i) {  // T[r, i] = sum_{c >= r, c < i} T[r, c] u_c
      zv acc{0.0, 0.0};
      for (int c = r; c < i; ++c) {
        const zv p = zmul(t[r][c], u[c]);
        acc.re += p.re;
        acc.im += p.im;
      }
      t[r][i] = acc;
    }
    if (r == i) t[i][i] = ti;
    __syncthreads();
  }
  for (int e = r; e < HB * HB; e += 64) T[e] = t[e % HB][e / HB];
}

__global__ void hh_init_q(zv* Q, int64_t ldq, int64_t M) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < M) Q[r + c * ldq] = zv{r == c ? 1.0 : 0.0, 0.0};
}

int reflector_workgroups(int64_t rows) {
  const int64_t g = cdiv(rows, 4 * NT);
  return (int)(g < 1 ? 1 : (g > kHouseholderMaxWg ? kHouseholderMaxWg : g));
}

// R[r][c] = A[r][c] for r <= c, 0 below (n x n, leading dimension n).
__global__ void hh_copy_r(const zv* A, int64_t ldx, int64_t n, zv* R) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r < n) R[r + c * n] = r <= c ? A[r + c * ldx] : zv{0.0, 0.0};
}

// Aug (2n x 2n, leading dimension 2n) = [[0, R], [R^H, 0]]: entry (n + i, j)
// = conj(R[j][i]), entry (j, n + i) = R[j][i], zero elsewhere.
__global__ void hh_augment(const zv* R, int64_t n, zv* Aug) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r >= 2 * n) return;
  zv v{0.0, 0.0};
  if (r >= n && c < n) {
    const zv x = R[c + (r - n) * n];
    v = zv{x.re, -x.im};
  } else if (r < n && c >= n) {
    v = R[r + (c - n) * n];
  }
  Aug[r + c * 2 * n] = v;
}

}  // namespace

int augment_hermitian(const z64* R, int64_t n, z64* Aug, hipStream_t s) {
  if (n <= 0) return kOk;
  hipLaunchKernelGGL(hh_augment, dim3((unsigned)cdiv(2 * n, 256), (unsigned)(2 * n)), dim3(256), 0, s,
                     reinterpret_cast<const zv*>(R), n, reinterpret_cast<zv*>(Aug));
  CHASE_CHK_LAUNCH();
  return kOk;
}

int householder_qr(z64* X, int64_t ldx, int64_t M, int64_t n, const HouseholderWs& ws, hipStream_t s) {
  if (n <= 0) return kOk;
  if (n > M || !ws.V || !ws.T || !ws.W1 || !ws.W2 || !ws.part || !ws.rowj || !ws.tau || !ws.Q || !ws.splitk)
    return -1;
  zv* A = reinterpret_cast<zv*>(X);
  zv* tau = reinterpret_cast<zv*>(ws.tau);
  const int64_t npan = cdiv(n, HB);
  int st = kOk;
  for (int64_t p = 0; p < npan; ++p) {
    const int64_t j0 = p * HB, jb = n - j0 < HB ? n - j0 : HB, jend = j0 + jb;
    for (int64_t j = j0; j < jend; ++j) {
      const int nwg = reflector_workgroups(M - j - 1);
      hipLaunchKernelGGL(hh_col_reduce, dim3(nwg), dim3(NT), 0, s, A, ldx, M, j, jend, nwg, ws.part,
                         reinterpret_cast<zv*>(ws.rowj));
      CHASE_CHK_LAUNCH();
      hipLaunchKernelGGL(hh_col_apply, dim3(nwg), dim3(NT), 0, s, A, ldx, M, j, jend, nwg, ws.part,
                         reinterpret_cast<const zv*>(ws.rowj), tau);
      CHASE_CHK_LAUNCH();
    }
    // V, T of the panel
    hipLaunchKernelGGL(hh_build_v, dim3((unsigned)cdiv(M - j0, 256), (unsigned)jb), dim3(256), 0, s, A, ldx, M, j0,
                       reinterpret_cast<zv*>(ws.V), M);
    CHASE_CHK_LAUNCH();
    GemmArgs g;  // W1 = V^H V (jb x jb)
    g.M = jb; g.N = jb; g.K = M - j0;
    g.A = ws.V; g.lda = M;
    g.B = ws.V; g.ldb = M;
    g.Y = ws.W1; g.ldy = jb;
    if ((st = zgemm_splitk(1, 0, g, ws.splitk, choose_splits(jb, jb, M - j0, 16, false), 0, s))) return st;
    z64* Tp = ws.T + p * HB * HB;
    hipLaunchKernelGGL(hh_build_t, dim3(1), dim3(64), 0, s, reinterpret_cast<const zv*>(ws.W1), jb, tau + j0,
                       (int)jb, reinterpret_cast<zv*>(Tp));
    CHASE_CHK_LAUNCH();
    const int64_t nt = n - jend;
    if (nt <= 0) continue;
    // trailing columns: A <- (I - V T V^H)^H A = A - V (T^H (V^H A))
    GemmArgs a;  // W1 = V^H A_trail (jb x nt)
    a.M = jb; a.N = nt; a.K = M - j0;
    a.A = ws.V; a.lda = M;
    a.B = X + j0 + jend * ldx; a.ldb = ldx;
    a.Y = ws.W1; a.ldy = jb;
    if ((st = zgemm_splitk(1, 0, a, ws.splitk, choose_splits(jb, nt, M - j0, 16, false), 0, s))) return st;
    GemmArgs b;  // W2 = T^H W1
    b.M = jb; b.N = nt; b.K = jb;
    b.A = Tp; b.lda = HB;
    b.B = ws.W1; b.ldb = jb;
    b.Y = ws.W2; b.ldy = jb;
    if ((st = zgemm_launch(1, 0, b, s))) return st;
    GemmArgs c;  // A_trail -= V W2
    c.M = M - j0; c.N = nt; c.K = jb;
    c.A = ws.V; c.lda = M;
    c.B = ws.W2; c.ldb = jb;
    c.Y = X + j0 + jend * ldx; c.ldy = ldx;
    c.alpha = -1.0; c.beta = 1.0;
    if ((st = zgemm_launch(0, 0, c, s))) return st;
  }
  if (ws.R) {  // R: the upper triangle of the factored block
    hipLaunchKernelGGL(hh_copy_r, dim3((unsigned)cdiv(n, 256), (unsigned)n), dim3(256), 0, s, A, ldx, n,
                       reinterpret_cast<zv*>(ws.R));
    CHASE_CHK_LAUNCH();
  }
  // Q = H_1 ... H_npan [I; 0], accumulated backwards; panel p only changes
  // rows and columns from j0 on
  zv* Q = reinterpret_cast<zv*>(ws.Q);
  hipLaunchKernelGGL(hh_init_q, dim3((unsigned)cdiv(M, 256), (unsigned)n), dim3(256), 0, s, Q, M, M);
  CHASE_CHK_LAUNCH();
  for (int64_t p = npan - 1; p >= 0; --p) {
    const int64_t j0 = p * HB, jb = n - j0 < HB ? n - j0 : HB, nq = n - j0;
    hipLaunchKernelGGL(hh_build_v, dim3((unsigned)cdiv(M - j0, 256), (unsigned)jb), dim3(256), 0, s, A, ldx, M, j0,
                       reinterpret_cast<zv*>(ws.V), M);
    CHASE_CHK_LAUNCH();
    GemmArgs a;  // W1 = V^H Q[j0:, j0:]
    a.M = jb; a.N = nq; a.K = M - j0;
    a.A = ws.V; a.lda = M;
    a.B = ws.Q + j0 + j0 * M; a.ldb = M;
    a.Y = ws.W1; a.ldy = jb;
    if ((st = zgemm_splitk(1, 0, a, ws.splitk, choose_splits(jb, nq, M - j0, 16, false), 0, s))) return st;
    GemmArgs b;  // W2 = T W1
    b.M = jb; b.N = nq; b.K = jb;
    b.A = ws.T + p * HB * HB; b.lda = HB;
    b.B = ws.W1; b.ldb = jb;
    b.Y = ws.W2; b.ldy = jb;
    if ((st = zgemm_launch(0, 0, b, s))) return st;
    GemmArgs c;  // Q[j0:, j0:] -= V W2
    c.M = M - j0; c.N = nq; c.K = jb;
    c.A = ws.V; c.lda = M;
    c.B = ws.W2; c.ldb = jb;
    c.Y = ws.Q + j0 + j0 * M; c.ldy = M;
    c.alpha = -1.0; c.beta = 1.0;
    if ((st = zgemm_launch(0, 0, c, s))) return st;
  }
  return copy_columns(ws.Q, M, X, ldx, M, n, s);
}

}  // namespace chase
