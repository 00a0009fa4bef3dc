// Eigen-decomposition of the n x n Hermitian Rayleigh quotient (Alg. 2's
// small eigensolve) on the GPU: two-sided block Jacobi.
//
// The quotient is copied into an npad x npad working matrix A (npad = nb *
// 16, nb even, the extra rows and columns zero with a zero diagonal: they are
// never coupled to the rest, so no rotation ever touches them) and V = I.
// A sweep visits every pair of the nb diagonal blocks of 16 once, nb / 2
// disjoint pairs at a time in the circle (round-robin) order:
//   1. per pair, the 32 x 32 Hermitian subproblem S = A[P, P] (P the 32
//      indices of its two blocks) gets one cyclic Jacobi sweep in LDS
//      with complex plane rotations J = [[c, w], [-conj(w), c]] (c real,
//      |w| = s, |angle| <= pi/4, so J stays close to the identity and the
//      block method converges), then U, the product of the rotations, is
//      taken one Newton-Schulz step towards the nearest unitary
//      (U (3I - U^H U) / 2), which keeps V orthonormal to a few ulps over
//      many rounds;
//   2. A <- J^H A J and V <- V J for the block-diagonal J of the pairs'
//      U: the 32 x 32 tiles A[P_a, P_c] become U_a^H A[P_a, P_c] U_c (the
//      tiles on and below the block diagonal, each written with its mirror)
//      and the tiles of V's row blocks become V[r, P_c] U_c.
// The host ends the sweeps once the largest off-diagonal entry seen by the
// pair solves of a sweep is below 1e-10 max|A_ii|: the quadratic convergence
// of the final sweep takes it to rounding level.  The eigenvalues are the
// diagonal of A, ranked ascending on the device, and the eigenvectors the
// matching columns of V.
#include "common.hpp"
#include "kernels.hpp"

#include <cmath>
#include <cstring>
#include <vector>

namespace chase {

namespace {

struct alignas(16) zv {
  double re, im;
};

__device__ __forceinline__ zv zadd(zv a, zv b) { return zv{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ zv zsub(zv a, zv b) { return zv{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ zv zscale(double s, zv a) { return zv{s * a.re, s * a.im}; }
__device__ __forceinline__ zv zmul(zv a, zv b) { return zv{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ zv zconj(zv a) { return zv{a.re, -a.im}; }
// conj(a) * b
__device__ __forceinline__ zv zcmul(zv a, zv b) { return zv{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }
__device__ __forceinline__ zv zfma(zv a, zv b, zv acc) {
  return zv{fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}
// acc + conj(a) * b
__device__ __forceinline__ zv zcfma(zv a, zv b, zv acc) {
  return zv{fma(a.re, b.re, fma(a.im, b.im, acc.re)), fma(a.re, b.im, fma(-a.im, b.re, acc.im))};
}

constexpr int BS = 16;        // diagonal block of the outer method
constexpr int PS = 2 * BS;    // pair subproblem order
constexpr int LDP = PS + 1;   // LDS row pitch (complex)
constexpr int NT = 256;
constexpr int NTP = 512;  // threads of the pair solve: one per (rotation, row or column)
// stats[0]: largest off-diagonal |S_uv| of the sweep (as ordered bits of a
// non-negative double), stats[1]: max_i |A_ii| at the sweep start.
constexpr int kStats = 2;

// Player at seat k of round r in the circle method over m (even) players:
// seat 0 keeps player 0, the others rotate one seat per round.
// (r in [0, m - 2], k in [0, m - 1], so k - 1 - r needs one correction.)
constexpr __device__ __host__ __forceinline__ int seat(int m, int r, int k) {
  const int x = k - 1 - r;
  return k == 0 ? 0 : 1 + (x < 0 ? x + (m - 1) : x);
}

// Global index of local index u (0..31) of pair (p, q).
__device__ __forceinline__ int64_t pidx(int p, int q, int u) {
  return u < BS ? (int64_t)p * BS + u : (int64_t)q * BS + (u - BS);
}

// 1 / sqrt(x) and 1 / x, x > 0 finite: the hardware estimate refined by two
// Newton steps (each squares the relative error; NaN propagates).
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  return y * fma(-x, y, 2.0);
}

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* a, double v) {
  // non-negative doubles order as their bit patterns; NaN (all exponent
  // bits set, any mantissa) orders above every finite value and is kept
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

__global__ __launch_bounds__(NT) void jac_init(const zv* G, int64_t ldg, int n, zv* A, zv* V, int npad) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= (int64_t)npad * npad) return;
  const int r = (int)(i % npad), c = (int)(i / npad);
  zv a{0.0, 0.0};
  if (r < n && c < n) a = r >= c ? G[r + c * ldg] : zconj(G[c + r * ldg]);
  if (r == c) a.im = 0.0;  // the quotient is Hermitian: its diagonal is real
  A[i] = a;
  V[i] = zv{r == c ? 1.0 : 0.0, 0.0};
}

// stats[1] = max |A_ii|, i < n; stats[0] = 0.
__global__ __launch_bounds__(NT) void jac_sweep_start(const zv* A, int n, int npad, unsigned long long* stats) {
  __shared__ double red[NT];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double d = A[i + (int64_t)i * npad].re;
    m = d == d ? fmax(m, fabs(d)) : INFINITY;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = 0ull;
    stats[1] = (unsigned long long)__double_as_longlong(red[0]);
  }
}

// One workgroup per pair of round r: one cyclic Jacobi sweep over S = A[P,
// P] (rotations below tol = u * max|A_ii| are skipped), write U (32 x 32,
// column-major) to Ubuf[pair] and rot[pair] = 1 if any rotation was made.
// A single sweep per visit: converging the 32 x 32 subproblem fully changes
// neither the number of outer sweeps nor the accuracy (the next visit of the
// pair continues from where this one stopped).  Each step applies 16
// rotations with disjoint indices to rows i, j and then columns i, j of S
// (writing the rotated 2 x 2 block exactly: diag(a', d'), zero coupling) and
// to columns i, j of U; the four lanes of a rotation compute its parameters
// from the same LDS words, read by one instruction before any is written.
__global__ __launch_bounds__(NTP) void jac_pair_solve(const zv* A, int npad, int nb, int r, zv* Ubuf, int* rot,
                                                     unsigned long long* stats) {
  __shared__ zv S[PS * LDP];
  __shared__ zv U[PS * LDP];
  __shared__ zv M[PS * LDP];
  __shared__ int rotflag[1];
  __shared__ double offmax[NTP / 64];
  const int t = threadIdx.x;
  const int pair = blockIdx.x;
  int p = seat(nb, r, pair), q = seat(nb, r, nb - 1 - pair);
  if (p > q) { const int x = p; p = q; q = x; }
  const double dmax = __longlong_as_double((long long)stats[1]);
  const double tol = 0x1p-53 * dmax, tol2 = tol * tol;

  // load S (row-major in LDS), U = I; largest off-diagonal entry
  double om = 0.0;
  for (int e = t; e < PS * PS; e += NTP) {
    const int u = e % PS, v = e / PS;
    zv a = A[pidx(p, q, u) + pidx(p, q, v) * (int64_t)npad];
    S[u * LDP + v] = a;
    U[u * LDP + v] = zv{u == v ? 1.0 : 0.0, 0.0};
    const double m = sqrt(a.re * a.re + a.im * a.im);
    if (!(m == m)) om = INFINITY;  // a non-finite entry reaches the host as an infinite maximum
    else if (u != v) om = fmax(om, m);
  }
  for (int off = 32; off > 0; off >>= 1) om = fmax(om, __shfl_down(om, off, 64));
  if ((t & 63) == 0) offmax[t >> 6] = om;
  if (t == 0) rotflag[0] = 0;
  __syncthreads();
  double pair_off = offmax[0];
  for (int w = 1; w < NTP / 64; ++w) pair_off = fmax(pair_off, offmax[w]);
  if (t == 0) atomic_max_nonneg(stats, pair_off);

  // The 32 threads t = 32 k + h of one wave half own rotation k of each
  // step: on column h of rows i, j, then, after a barrier, on row h of
  // columns i, j of S and U.  Rotations of one step touch disjoint rows and
  // columns, so two barriers per step suffice.
  const int kk = t >> 5, hq = t & 31;
  int rotated = 0;
  for (int step = 0; step < PS - 1 && !(pair_off <= tol); ++step) {
    int i = seat(PS, step, kk), j = seat(PS, step, PS - 1 - kk);
    if (i > j) { const int x = i; i = j; j = x; }
    const zv z = S[i * LDP + j];
    const double a = S[i * LDP + i].re, d = S[j * LDP + j].re;
    const double az2 = z.re * z.re + z.im * z.im;
    const bool go = az2 > tol2 || !(az2 == az2);
    double c = 1.0, an = a, dn = d;
    zv w{0.0, 0.0};
    if (go) {
      // tau = (d - a) / (2 |z|), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
      // c = 1 / sqrt(1 + t^2), s = t c, from hardware reciprocal (square
      // root) estimates with two Newton steps each: the rotation needs c^2 +
      // s^2 = 1 only to a few ulps (the Newton-Schulz step below restores
      // U's orthonormality), and the exact 2 x 2 values written below are
      // those of this very rotation
      const double inv_az = rsq_nr(az2);
      const double az = az2 * inv_az;
      const double tau = 0.5 * (d - a) * inv_az;
      const double at = fabs(tau);
      // |tau| above 2^500: t = 1 / (2 |tau|) to full precision, and tau^2 would overflow
      const double den = at > 0x1p500 ? 2.0 * at : at + (1.0 + at * at) * rsq_nr(1.0 + at * at);
      const double tt = (tau >= 0.0 ? 1.0 : -1.0) * rcp_nr(den);
      c = rsq_nr(1.0 + tt * tt);
      const double sn_az = tt * c * inv_az;
      w = zv{sn_az * z.re, sn_az * z.im};  // w = s e, e = z / |z|
      an = a - tt * az;
      dn = d + tt * az;
      rotated = 1;
      // rows i, j:  S_i <- c S_i - w S_j,  S_j <- conj(w) S_i + c S_j
      {
        const int col = hq;
        const zv si = S[i * LDP + col], sj = S[j * LDP + col];
        S[i * LDP + col] = zsub(zscale(c, si), zmul(w, sj));
        S[j * LDP + col] = zadd(zcmul(w, si), zscale(c, sj));
      }
    }
    __syncthreads();
    if (go) {
      // columns i, j of S and U:  X_i <- c X_i - conj(w) X_j,  X_j <- w X_i + c X_j
      {
        const int row = hq;
        const zv xi = S[row * LDP + i], xj = S[row * LDP + j];
        zv ni = zsub(zscale(c, xi), zcmul(w, xj)), nj = zadd(zmul(w, xi), zscale(c, xj));
        if (row == i) { ni = zv{an, 0.0}; nj = zv{0.0, 0.0}; }
        if (row == j) { ni = zv{0.0, 0.0}; nj = zv{dn, 0.0}; }
        S[row * LDP + i] = ni;
        S[row * LDP + j] = nj;
        const zv ui = U[row * LDP + i], uj = U[row * LDP + j];
        U[row * LDP + i] = zsub(zscale(c, ui), zcmul(w, uj));
        U[row * LDP + j] = zadd(zmul(w, ui), zscale(c, uj));
      }
    }
    __syncthreads();
  }
  if (rotated) rotflag[0] = 1;
  __syncthreads();
  const int any_total = rotflag[0];
  if (any_total) {
    // one Newton-Schulz step: U <- U (3 I - U^H U) / 2
    for (int e = t; e < PS * PS; e += NTP) {
      const int u = e % PS, v = e / PS;
      zv acc{0.0, 0.0};
#pragma unroll 4
      for (int l = 0; l < PS; ++l) acc = zcfma(U[l * LDP + u], U[l * LDP + v], acc);
      M[u * LDP + v] = zv{(u == v ? 3.0 : 0.0) - acc.re, -acc.im};
    }
    __syncthreads();
    for (int e = t; e < PS * PS; e += NTP) {
      const int u = e % PS, v = e / PS;
      zv acc{0.0, 0.0};
#pragma unroll 4
      for (int l = 0; l < PS; ++l) acc = zfma(U[u * LDP + l], M[l * LDP + v], acc);
      S[u * LDP + v] = zscale(0.5, acc);  // S is free now
    }
    __syncthreads();
  }
  zv* out = Ubuf + (int64_t)pair * PS * PS;
  for (int e = t; e < PS * PS; e += NTP) {
    const int u = e % PS, v = e / PS;
    out[u + v * PS] = any_total ? S[u * LDP + v] : U[u * LDP + v];
  }
  if (t == 0) rot[pair] = any_total;
}

// A <- J^H A J, V <- V J for the pairs of round r.  Work items: the tiles
// (a, c), a >= c, of A in pair coordinates (each written with its mirror),
// then the tiles (row block rb, pair c) of the first vrows rows of V (the
// rows below stay e_j, untouched).  Thread t computes the 2 x 2 outputs
// (u, u + 16) x (v, v + 16), u = t % 16, v = t / 16, of each 32 x 32 product.
__global__ __launch_bounds__(NT) void jac_apply(zv* A, zv* V, int npad, int nb, int r, int vblocks,
                                                const zv* Ubuf, const int* rot) {
  __shared__ zv X[PS * LDP];
  __shared__ zv T[PS * LDP];
  __shared__ zv W[PS * LDP];
  const int t = threadIdx.x;
  const int u = t & 15, v = t >> 4;
  const int k = nb / 2;
  const int64_t tilesA = (int64_t)k * (k + 1) / 2;
  const int64_t item = blockIdx.x;
  if (item < tilesA) {
    // (a, c) from the linear lower-triangle index
    int a = (int)((sqrt(8.0 * (double)item + 1.0) - 1.0) * 0.5);
    while ((int64_t)(a + 1) * (a + 2) / 2 <= item) ++a;
    while ((int64_t)a * (a + 1) / 2 > item) --a;
    const int c = (int)(item - (int64_t)a * (a + 1) / 2);
    if (!rot[a] && !rot[c]) return;
    int pa = seat(nb, r, a), qa = seat(nb, r, nb - 1 - a);
    if (pa > qa) { const int x = pa; pa = qa; qa = x; }
    int pc = seat(nb, r, c), qc = seat(nb, r, nb - 1 - c);
    if (pc > qc) { const int x = pc; pc = qc; qc = x; }
    const zv* Ua_g = Ubuf + (int64_t)a * PS * PS;
    const zv* Uc_g = Ubuf + (int64_t)c * PS * PS;
    for (int e = t; e < PS * PS; e += NT) {
      const int uu = e % PS, vv = e / PS;
      X[uu * LDP + vv] = A[pidx(pa, qa, uu) + pidx(pc, qc, vv) * (int64_t)npad];
      W[uu * LDP + vv] = Uc_g[uu + vv * PS];
    }
    __syncthreads();
    // T = X Uc
    zv t00{0, 0}, t01{0, 0}, t10{0, 0}, t11{0, 0};
#pragma unroll 4
    for (int l = 0; l < PS; ++l) {
      const zv x0 = X[u * LDP + l], x1 = X[(u + 16) * LDP + l];
      const zv w0 = W[l * LDP + v], w1 = W[l * LDP + v + 16];
      t00 = zfma(x0, w0, t00); t01 = zfma(x0, w1, t01);
      t10 = zfma(x1, w0, t10); t11 = zfma(x1, w1, t11);
    }
    T[u * LDP + v] = t00; T[u * LDP + v + 16] = t01;
    T[(u + 16) * LDP + v] = t10; T[(u + 16) * LDP + v + 16] = t11;
    __syncthreads();
    for (int e = t; e < PS * PS; e += NT) W[(e % PS) * LDP + e / PS] = Ua_g[e];  // W = Ua
    __syncthreads();
    // Y = Ua^H T
    zv y00{0, 0}, y01{0, 0}, y10{0, 0}, y11{0, 0};
#pragma unroll 4
    for (int l = 0; l < PS; ++l) {
      const zv a0 = W[l * LDP + u], a1 = W[l * LDP + u + 16];
      const zv b0 = T[l * LDP + v], b1 = T[l * LDP + v + 16];
      y00 = zcfma(a0, b0, y00); y01 = zcfma(a0, b1, y01);
      y10 = zcfma(a1, b0, y10); y11 = zcfma(a1, b1, y11);
    }
    X[u * LDP + v] = y00; X[u * LDP + v + 16] = y01;
    X[(u + 16) * LDP + v] = y10; X[(u + 16) * LDP + v + 16] = y11;
    __syncthreads();
    for (int e = t; e < PS * PS; e += NT) {
      const int uu = e % PS, vv = e / PS;
      zv y = X[uu * LDP + vv];
      if (a == c) {  // Hermitian diagonal tile: average with the mirror
        const zv m = X[vv * LDP + uu];
        y = zv{0.5 * (y.re + m.re), 0.5 * (y.im - m.im)};
        if (uu == vv) y.im = 0.0;
      }
      A[pidx(pa, qa, uu) + pidx(pc, qc, vv) * (int64_t)npad] = y;
    }
    if (a != c) {
      for (int e = t; e < PS * PS; e += NT) {
        const int vv = e % PS, uu = e / PS;  // row vv of the mirror tile runs along threads
        A[pidx(pc, qc, vv) + pidx(pa, qa, uu) * (int64_t)npad] = zconj(X[uu * LDP + vv]);
      }
    }
    return;
  }
  const int64_t vi = item - tilesA;
  if (vi >= (int64_t)vblocks * k) return;
  const int rb = (int)(vi / k), c = (int)(vi % k);
  if (!rot[c]) return;
  int pc = seat(nb, r, c), qc = seat(nb, r, nb - 1 - c);
  if (pc > qc) { const int x = pc; pc = qc; qc = x; }
  const zv* Uc_g = Ubuf + (int64_t)c * PS * PS;
  for (int e = t; e < PS * PS; e += NT) {
    const int uu = e % PS, vv = e / PS;
    X[uu * LDP + vv] = V[(int64_t)rb * PS + uu + pidx(pc, qc, vv) * (int64_t)npad];
    W[uu * LDP + vv] = Uc_g[uu + vv * PS];
  }
  __syncthreads();
  zv t00{0, 0}, t01{0, 0}, t10{0, 0}, t11{0, 0};
#pragma unroll 4
  for (int l = 0; l < PS; ++l) {
    const zv x0 = X[u * LDP + l], x1 = X[(u + 16) * LDP + l];
    const zv w0 = W[l * LDP + v], w1 = W[l * LDP + v + 16];
    t00 = zfma(x0, w0, t00); t01 = zfma(x0, w1, t01);
    t10 = zfma(x1, w0, t10); t11 = zfma(x1, w1, t11);
  }
  zv* Vc = V + (int64_t)rb * PS;
  Vc[u + pidx(pc, qc, v) * (int64_t)npad] = t00;
  Vc[u + pidx(pc, qc, v + 16) * (int64_t)npad] = t01;
  Vc[u + 16 + pidx(pc, qc, v) * (int64_t)npad] = t10;
  Vc[u + 16 + pidx(pc, qc, v + 16) * (int64_t)npad] = t11;
}

// Rank of each eigenvalue (ascending, ties by position) and theta in that order.
__global__ __launch_bounds__(NT) void jac_rank(const zv* A, int n, int npad, int* rank, double* theta) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double di = A[i + (int64_t)i * npad].re;
  int k = 0;
  for (int j = 0; j < n; ++j) {
    const double dj = A[j + (int64_t)j * npad].re;
    k += (dj < di) || (dj == di && j < i);
  }
  rank[i] = k;
  theta[k] = di;
}

// out[:, rank[i]] = V[0:n, i]
__global__ __launch_bounds__(NT) void jac_gather(const zv* V, int n, int npad, const int* rank, zv* out,
                                                 int64_t ldo) {
  const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int row = (int)(e % n), i = (int)(e / n);
  out[row + rank[i] * ldo] = V[row + (int64_t)i * npad];
}

struct Layout {
  int npad = 0, nb = 0;
  size_t offA = 0, offV = 0, offU = 0, offRot = 0, offRank = 0, offStats = 0, bytes = 0;
};

Layout layout(int64_t n) {
  Layout L;
  int nb = (int)cdiv(std::max<int64_t>(n, 1), BS);
  nb += nb & 1;
  L.nb = nb;
  L.npad = nb * BS;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t o = 0;
  L.offA = o; o = up(o + (size_t)L.npad * L.npad * 16);
  L.offV = o; o = up(o + (size_t)L.npad * L.npad * 16);
  L.offU = o; o = up(o + (size_t)(nb / 2) * PS * PS * 16);
  L.offRot = o; o = up(o + (size_t)(nb / 2) * 4);
  L.offRank = o; o = up(o + (size_t)L.npad * 4);
  L.offStats = o; o = up(o + kStats * 8);
  L.bytes = o;
  return L;
}

}  // namespace

int64_t heevj_workspace_bytes(int64_t n) { return (int64_t)layout(n).bytes; }

int heevj(z64* G, int64_t ldg, int64_t n, double* theta, void* ws, int* sweeps_out, hipStream_t s) {
  if (sweeps_out) *sweeps_out = 0;
  if (n <= 0) return kOk;
  if (!G || !theta || !ws || ldg < n) return -1;
  const Layout L = layout(n);
  char* base = static_cast<char*>(ws);
  zv* A = reinterpret_cast<zv*>(base + L.offA);
  zv* V = reinterpret_cast<zv*>(base + L.offV);
  zv* Ub = reinterpret_cast<zv*>(base + L.offU);
  int* rot = reinterpret_cast<int*>(base + L.offRot);
  int* rank = reinterpret_cast<int*>(base + L.offRank);
  unsigned long long* stats = reinterpret_cast<unsigned long long*>(base + L.offStats);
  const int npad = L.npad, nb = L.nb, k = nb / 2;
  const int64_t total = (int64_t)npad * npad;
  hipLaunchKernelGGL(jac_init, dim3((unsigned)cdiv(total, NT)), dim3(NT), 0, s, reinterpret_cast<const zv*>(G),
                     ldg, (int)n, A, V, npad);
  CHASE_CHK_LAUNCH();
  const int vblocks = (int)cdiv(n, PS);  // V's rows at and below n stay those of the identity
  const int64_t items = (int64_t)k * (k + 1) / 2 + (int64_t)vblocks * k;
  constexpr int kMaxSweeps = 40;
  unsigned long long host_stats[kStats];
  int sweep = 0;
  bool done = false;
  for (; sweep < kMaxSweeps && !done; ++sweep) {
    hipLaunchKernelGGL(jac_sweep_start, dim3(1), dim3(NT), 0, s, A, (int)n, npad, stats);
    CHASE_CHK_LAUNCH();
    for (int r = 0; r < nb - 1; ++r) {
      hipLaunchKernelGGL(jac_pair_solve, dim3((unsigned)k), dim3(NTP), 0, s, A, npad, nb, r, Ub, rot, stats);
      CHASE_CHK_LAUNCH();
      hipLaunchKernelGGL(jac_apply, dim3((unsigned)items), dim3(NT), 0, s, A, V, npad, nb, r, vblocks, Ub, rot);
      CHASE_CHK_LAUNCH();
    }
    CHASE_CHK(hipMemcpyAsync(host_stats, stats, sizeof(host_stats), hipMemcpyDeviceToHost, s));
    CHASE_CHK(hipStreamSynchronize(s));
    double off, dmax;
    std::memcpy(&off, &host_stats[0], 8);
    std::memcpy(&dmax, &host_stats[1], 8);
    if (!std::isfinite(off) || !std::isfinite(dmax)) return kBreakdown;
    // the sweep just made started from off-diagonal entries this small:
    // its quadratic convergence has taken them to rounding level
    done = off <= 1e-10 * dmax;
  }
  if (sweeps_out) *sweeps_out = sweep;
  if (!done) return kBreakdown;
  hipLaunchKernelGGL(jac_rank, dim3((unsigned)cdiv(n, NT)), dim3(NT), 0, s, A, (int)n, npad, rank, theta);
  CHASE_CHK_LAUNCH();
  hipLaunchKernelGGL(jac_gather, dim3((unsigned)cdiv(n * n, NT)), dim3(NT), 0, s, V, (int)n, npad, rank,
                     reinterpret_cast<zv*>(G), ldg);
  CHASE_CHK_LAUNCH();
  return kOk;
}

}  // namespace chase
