// Host driver of the ChASE hot path on one MI355X: the loop of Alg. 2 with a
// 1 x 1 grid (AllReduce = identity, B2 = C2), host scalar logic (bounds,
// degree optimisation, CondEst, locking decisions) and the C ABI.
//
// Device work all runs in the hand-written kernels of zgemm.hip, zfilter.hip,
// bfilter.hip, zgrad.hip, hhqr.hip, heevj.hip and small.hip; the library
// links no BLAS or LAPACK.  The n_e x n_e eigensolve of Rayleigh-Ritz is the
// block Jacobi of heevj.hip (the real quotient, with zero imaginary parts,
// gets real eigenvectors from it), and so are the level-2 trace's singular
// values (of the Householder R, through [[0, R], [R^H, 0]]).  The real type
// variant's Householder QR runs the complex hhqr.hip kernels on its block
// widened to complex128 with zero imaginary parts.
//
// Three element types share the loop: complex128 (chase_solve), real
// symmetric float64 (chase_solve_real: real columns read as complex row
// pairs, see Workspace) and complex64 (chase_solve_c64: every column on the
// FP32 rung, H in the caller's complex64 storage).
#include "../../include/chase_hip.h"
#include "common.hpp"
#include "kernels.hpp"


#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <functional>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

namespace chase {

static thread_local std::string g_last_error;

void set_last_error(const char* where, hipError_t err) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(err);
}
const char* last_error() { return g_last_error.c_str(); }

static void set_msg(const std::string& s) { g_last_error = s; }

// ---------------------------------------------------------------------------
// Host scalar logic (shared by the solve and the step entry points)
// ---------------------------------------------------------------------------

// rho(t) = max(|t - sqrt(t^2-1)|, |t + sqrt(t^2-1)|), complex square root.
static double rho_of(double t) {
  std::complex<double> s = std::sqrt(std::complex<double>(t * t - 1.0, 0.0));
  return std::max(std::abs(t - s), std::abs(t + s));
}

// Alg. 5.  The estimate reads the first column and the first active column
// of the block sorted by degree (ties in ascending Ritz value): the active
// column of smallest degree, and among those the smallest Ritz value, which
// is also the first column when nothing is locked.  Taking that column by
// search gives the same value for any order of the active columns, so the
// mixed-precision solve, whose block is sorted by rung first, gets the
// estimate of its degree-sorted view.
static double cond_est(const double* Lam, double c, double e, const int32_t* degs, int ne, int locked) {
  int js = locked;
  int d_max = degs[locked];
  for (int j = locked + 1; j < ne; ++j) {
    if (degs[j] < degs[js] || (degs[j] == degs[js] && Lam[j] < Lam[js])) js = j;
    d_max = std::max(d_max, (int)degs[j]);
  }
  const double t_first = ((locked > 0 ? Lam[0] : Lam[js]) - c) / e;
  const double t_active = (Lam[js] - c) / e;
  const int d = degs[js];
  return std::pow(rho_of(t_active), d) * std::pow(rho_of(t_first), d_max - d);
}

// Alg. 4's branch.
static int select_qr(double cond) {
  if (cond > 1e8) return CHASE_QR_SHIFTED;
  if (cond < 20.0) return CHASE_QR_CHOLQR1;
  return CHASE_QR_CHOLQR2;
}

// Degree optimisation: steps needed for resd to fall to tol_abs at the
// Chebyshev growth rate rho((lambda - c)/e), plus a margin; capped, even.
static int degree_opt(double resd, double lam, double c, double e, double tol_abs, int max_deg, int extra) {
  const double r = rho_of((lam - c) / e);
  int d;
  if (r <= 1.0 + 1e-12 || !std::isfinite(resd)) {
    d = max_deg;
  } else {
    const double ratio = resd / tol_abs;
    if (ratio <= 1.0) d = extra;
    else d = (int)std::ceil(std::log(ratio) / std::log(r)) + extra;
  }
  d = std::min(std::max(d, 2), max_deg);
  return d + (d % 2);
}

// Eigenpairs of a small real symmetric matrix by cyclic Jacobi rotations
// (k <= a few dozen: the Lanczos tridiagonals).  Ascending eigenvalues;
// Z column-major, column i the eigenvector of w[i].
static void jacobi_eig(int k, std::vector<double> a, std::vector<double>& w, std::vector<double>& Z) {
  Z.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) Z[i + (size_t)i * k] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[i + (size_t)j * k]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) {
        tot += A(i, j) * A(i, j);
        if (i != j) off += A(i, j) * A(i, j);
      }
    if (off <= 1e-34 * tot || off == 0.0) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A(p, q);
        if (apq == 0.0) continue;
        const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int r = 0; r < k; ++r) {  // columns p, q
          const double arp = A(r, p), arq = A(r, q);
          A(r, p) = cs * arp - sn * arq;
          A(r, q) = sn * arp + cs * arq;
        }
        for (int r = 0; r < k; ++r) {  // rows p, q
          const double apr = A(p, r), aqr = A(q, r);
          A(p, r) = cs * apr - sn * aqr;
          A(q, r) = sn * apr + cs * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double zrp = Z[r + (size_t)p * k], zrq = Z[r + (size_t)q * k];
          Z[r + (size_t)p * k] = cs * zrp - sn * zrq;
          Z[r + (size_t)q * k] = sn * zrp + cs * zrq;
        }
      }
  }
  std::vector<int> idx(k);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
  w.resize(k);
  std::vector<double> Zs((size_t)k * k);
  for (int i = 0; i < k; ++i) {
    w[i] = A(idx[i], idx[i]);
    for (int r = 0; r < k; ++r) Zs[r + (size_t)i * k] = Z[r + (size_t)idx[i] * k];
  }
  Z.swap(Zs);
}

// Spectral bounds from the Lanczos coefficients of `runs` runs (each
// alpha/beta row of length ksteps, truncated at the first zero beta).
static void bounds_from_lanczos(const std::vector<double>& alpha, const std::vector<double>& beta, int runs,
                                int ksteps, int64_t N, int ne, double out[4]) {
  double b_sup = -std::numeric_limits<double>::infinity();
  double mu_1 = std::numeric_limits<double>::infinity();
  double theta_max = -std::numeric_limits<double>::infinity();
  std::vector<double> nodes, weights;
  for (int r = 0; r < runs; ++r) {
    int k = 0;
    while (k < ksteps) {
      ++k;
      if (beta[(size_t)r * ksteps + k - 1] == 0.0) break;
    }
    std::vector<double> T((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) {
      T[i + (size_t)i * k] = alpha[(size_t)r * ksteps + i];
      if (i + 1 < k) {
        T[i + (size_t)(i + 1) * k] = beta[(size_t)r * ksteps + i];
        T[(i + 1) + (size_t)i * k] = beta[(size_t)r * ksteps + i];
      }
    }
    std::vector<double> w, Z;
    jacobi_eig(k, T, w, Z);
    b_sup = std::max(b_sup, w[k - 1] + beta[(size_t)r * ksteps + k - 1]);
    mu_1 = std::min(mu_1, w[0]);
    theta_max = std::max(theta_max, w[k - 1]);
    for (int i = 0; i < k; ++i) {
      nodes.push_back(w[i]);
      weights.push_back(Z[0 + (size_t)i * k] * Z[0 + (size_t)i * k]);
    }
  }
  std::vector<int> order(nodes.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nodes[x] < nodes[y]; });
  double cum = 0.0;
  size_t idx = order.size() - 1;
  for (size_t i = 0; i < order.size(); ++i) {
    cum += weights[order[i]];
    if ((double)N * cum / runs >= (double)ne) {
      idx = i;
      break;
    }
  }
  double mu_ne = nodes[order[idx]];
  mu_ne = std::min(std::max(mu_ne, mu_1), std::nextafter(b_sup, -std::numeric_limits<double>::infinity()));
  out[0] = b_sup;
  out[1] = mu_1;
  out[2] = mu_ne;
  out[3] = std::max(std::fabs(mu_1), std::fabs(theta_max));
}

// ---------------------------------------------------------------------------
// Device workspace
// ---------------------------------------------------------------------------

struct Workspace {
  int64_t N = 0;
  int ne = 0;
  int max_splits = 16;
  z64* C2 = nullptr;     // N x ne
  z64* B = nullptr;      // N x ne
  z64* G = nullptr;      // ne x ne (Gram / Rayleigh quotient / eigenvectors)
  z64* L = nullptr;      // ne x ne (Cholesky factor, then its inverse)
  z64* T = nullptr;      // ne x ne scratch
  z64* ws = nullptr;     // split-K partials
  z64* tau = nullptr;    // Householder scalars (ne)
  z64* hhV = nullptr;    // Householder QR scratch (hhqr.hip): N x panel
  z64* hhT = nullptr;    // panels x panel x panel
  z64* hhW = nullptr;    // 2 x panel x ne
  double* hhpart = nullptr;
  z64* hhrow = nullptr;
  double* theta = nullptr;
  double* resd = nullptr;
  double* shift = nullptr;
  int* info = nullptr;
  int* flag = nullptr;
  int* perm = nullptr;
  z64* lzV = nullptr;    // Lanczos: N x 8 each
  z64* lzVold = nullptr;
  z64* lzW = nullptr;
  z64* starts = nullptr; // N x 4 generated starts
  double* lz_alpha = nullptr;
  double* lz_beta = nullptr;
  // mixed precision
  c32* A32 = nullptr;
  c32* X32a = nullptr;
  c32* X32b = nullptr;
  uint16_t* P16 = nullptr;     // BF16x3 planes of conj(H) (4 x ldp x N)
  int64_t ldp = 0;
  uint16_t* XP16a = nullptr;   // BF16x3 planes of X32a / X32b (4 x ldp x ne each, k padding zero)
  uint16_t* XP16b = nullptr;
  void* tail_ws = nullptr;     // split-K tail of the big GEMMs
  int* tail_counters = nullptr;
  z64* tune_scratch = nullptr; // autotuner output sink (N x ne), allocated on first use
  void* jacws = nullptr;       // block-Jacobi eigensolver of the n_e x n_e quotient
  int jac_sweeps = 0;          // sweeps of its last call
  // Real symmetric problems run on the row-pair view: a real column of even
  // length 2 N is read as N complex values (rows 2 i, 2 i + 1 as Re, Im), so
  // every column operation, and every product whose real part is the wanted
  // real product, runs on the complex kernels unchanged.  N is then the
  // number of row pairs and `rows` the order; an odd order gets one zero row.
  bool real = false;
  int64_t rows = 0;
  z64* Cint = nullptr;         // N x ne: the caller's block in the row-pair layout
  double* Hpad = nullptr;      // 2N x 2N copy of H when its own layout does not fit
  const double* Hr = nullptr;  // this solve's H (real, order rows) for the Lanczos products
  int64_t ldhr = 0;
  // complex64 problems: H stays in the caller's complex64 storage; the filter
  // and the Rayleigh-Ritz H Q run on the FP32 kernels, the rest in FP64 on an
  // internal complex128 copy of the block (Cint).
  bool c64 = false;
  const c32* H32 = nullptr;    // this solve's H
  int64_t ldh32 = 0;
  std::vector<void*> owned;
  // Sizing mode: alloc adds up the bytes and allocates nothing; create()
  // then makes no device call either.
  bool counting = false;
  size_t counted = 0;

  template <class T>
  int alloc(T** p, size_t count) {
    void* q = nullptr;
    if (count == 0) count = 1;
    if (counting) {
      counted += count * sizeof(T);
      *p = nullptr;
      return kOk;
    }
    const hipError_t err = hipMalloc(&q, count * sizeof(T));
    if (err != hipSuccess) {
      (void)hipGetLastError();
      size_t free_b = 0, total_b = 0;
      (void)hipMemGetInfo(&free_b, &total_b);
      set_msg("hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed (" + hipGetErrorString(err) +
              "; " + std::to_string(free_b >> 20) + " of " + std::to_string(total_b >> 20) + " MiB free)");
      return kAllocFailed;
    }
    owned.push_back(q);
    *p = reinterpret_cast<T*>(q);
    return kOk;
  }

  int create(int64_t N_, int ne_, bool mixed, bool lanczos, bool bf16 = false) {
    N = N_;
    ne = ne_;
    const size_t nne = (size_t)N * ne, sq = (size_t)ne * ne;
    int st = kOk;
    st = st ? st : alloc(&C2, nne);
    st = st ? st : alloc(&B, nne);
    st = st ? st : alloc(&G, sq);
    st = st ? st : alloc(&L, sq);
    st = st ? st : alloc(&T, sq);
    st = st ? st : alloc(&ws, (size_t)zgemm_splitk_workspace(ne, ne, max_splits));
    st = st ? st : alloc(&tau, (size_t)ne);
    {
      const size_t hp = kHouseholderPanel, npan = (size_t)cdiv(ne, kHouseholderPanel);
      st = st ? st : alloc(&hhV, (size_t)N * hp);
      st = st ? st : alloc(&hhT, npan * hp * hp);
      st = st ? st : alloc(&hhW, 2 * hp * (size_t)ne);
      st = st ? st : alloc(&hhpart, (size_t)kHouseholderMaxWg * 2 * hp);
      st = st ? st : alloc(&hhrow, hp);
    }
    st = st ? st : alloc(reinterpret_cast<char**>(&jacws), (size_t)heevj_workspace_bytes(ne));
    st = st ? st : alloc(&theta, (size_t)ne);
    st = st ? st : alloc(&resd, (size_t)ne);
    st = st ? st : alloc(&shift, 1);
    st = st ? st : alloc(&info, 1);
    st = st ? st : alloc(&flag, 1);
    st = st ? st : alloc(&perm, (size_t)ne);
    st = st ? st : alloc(reinterpret_cast<char**>(&tail_ws), (size_t)tail_workspace_bytes());
    st = st ? st : alloc(&tail_counters, (size_t)kTailCounterInts);
    if (!st && !counting) st = tail_counters_init(tail_counters, nullptr);
    if (!st && !counting && hipDeviceSynchronize() != hipSuccess) st = kHipError;
    st = st ? st : alloc(&lz_alpha, 8 * 256);
    st = st ? st : alloc(&lz_beta, 8 * 256);
    if (lanczos) {
      st = st ? st : alloc(&lzV, (size_t)N * 8);
      st = st ? st : alloc(&lzVold, (size_t)N * 8);
      st = st ? st : alloc(&lzW, (size_t)N * 8);
      st = st ? st : alloc(&starts, (size_t)N * 4);
    }
    if (mixed) {
      st = st ? st : alloc(&A32, (size_t)N * N);
      st = st ? st : alloc(&X32a, nne);
      st = st ? st : alloc(&X32b, nne);
    }
    if (bf16) {
      ldp = bsplit_ld(N);
      st = st ? st : alloc(&P16, (size_t)4 * ldp * N);
      st = st ? st : alloc(&XP16a, (size_t)4 * ldp * ne);
      st = st ? st : alloc(&XP16b, (size_t)4 * ldp * ne);
      if (!st && !counting && (hipMemset(XP16a, 0, sizeof(uint16_t) * 4 * ldp * ne) != hipSuccess ||
                  hipMemset(XP16b, 0, sizeof(uint16_t) * 4 * ldp * ne) != hipSuccess)) {
        set_msg("hipMemset failed");
        st = kHipError;
      }
    }
    if (st) release();
    return st;
  }

  // Workspace of a real symmetric problem of order n_real (row-pair view).
  int create_real(int64_t n_real, int ne_) {
    int st = create((n_real + 1) / 2, ne_, false, true, false);
    if (st) return st;
    real = true;
    rows = n_real;
    st = st ? st : alloc(&Cint, (size_t)N * ne_);
    if (st) release();
    return st;
  }
  // Workspace of a complex64 problem: FP32 ping-pong blocks, no copy of H.
  int create_c64(int64_t n, int ne_) {
    int st = create(n, ne_, false, true, false);
    if (st) return st;
    c64 = true;
    const size_t nne = (size_t)N * ne_;
    st = st ? st : alloc(&X32a, nne);
    st = st ? st : alloc(&X32b, nne);
    st = st ? st : alloc(&Cint, nne);
    if (st) release();
    return st;
  }
  // Householder QR of a real block through the complex kernels (first use):
  // the widened block, its Q and one panel of reflectors, 2N rows each
  z64* hhXc = nullptr;
  z64* hhQc = nullptr;
  z64* hhVc = nullptr;
  int ensure_hh_real() {
    if (hhXc && hhQc && hhVc) return kOk;
    const size_t M = (size_t)(2 * N);
    int st = hhXc ? kOk : alloc(&hhXc, M * ne);
    st = st ? st : (hhQc ? kOk : alloc(&hhQc, M * ne));
    st = st ? st : (hhVc ? kOk : alloc(&hhVc, M * kHouseholderPanel));
    if (st) {  // free what this call allocated: the next use retries from scratch
      for (z64** p : {&hhXc, &hhQc, &hhVc}) free_one(reinterpret_cast<void**>(p));
    }
    return st;
  }
  void free_one(void** p) {
    if (!*p) return;
    if (!counting) (void)hipFree(*p);
    owned.erase(std::remove(owned.begin(), owned.end(), *p), owned.end());
    *p = nullptr;
  }
  // Trace level 2 (first use): a copy of the block to factor, its R, the
  // augmented 2 n_e x 2 n_e Hermitian matrix of R and its eigensolver's
  // workspace and eigenvalues
  z64* trX = nullptr;
  z64* trR = nullptr;
  z64* trAug = nullptr;
  void* trJac = nullptr;
  double* trTheta = nullptr;
  int ensure_trace() {
    if (trX && trR && trAug && trJac && trTheta) return kOk;
    const size_t n2 = 2 * (size_t)ne;
    int st = trX ? kOk : alloc(&trX, (size_t)N * ne);
    st = st ? st : (trR ? kOk : alloc(&trR, (size_t)ne * ne));
    st = st ? st : (trAug ? kOk : alloc(&trAug, n2 * n2));
    st = st ? st : (trJac ? kOk : alloc(reinterpret_cast<char**>(&trJac), (size_t)heevj_workspace_bytes((int64_t)n2)));
    st = st ? st : (trTheta ? kOk : alloc(&trTheta, n2));
    if (st) {
      for (void** q : {reinterpret_cast<void**>(&trX), reinterpret_cast<void**>(&trR), reinterpret_cast<void**>(&trAug),
                       &trJac, reinterpret_cast<void**>(&trTheta)})
        free_one(q);
    }
    return st;
  }
  int ensure_hpad() {
    return Hpad ? kOk : alloc(&Hpad, (size_t)(2 * N) * (size_t)(2 * N));
  }

  void release() {
    for (void* p : owned) (void)hipFree(p);
    owned.clear();
  }
};

// ---------------------------------------------------------------------------
// Steps
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Tile-shape autotuner for the filter GEMM.  A size class is (order M, active
// columns in steps of 32); the first time a class is seen the candidate
// launches (tile configuration x tail policy) are timed on the real operands
// with the output redirected to scratch, and the fastest is kept for the
// life of the process.
// ---------------------------------------------------------------------------
struct FilterTuner {
  std::mutex mu;
  std::map<std::pair<int64_t, int64_t>, int> best;
};
static FilterTuner& filter_tuner() {
  static FilterTuner t;
  return t;
}

static int time_launches(const std::function<int()>& launch, hipStream_t s, float* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  CHASE_CHK(hipEventCreate(&a));
  CHASE_CHK(hipEventCreate(&b));
  int st = launch();  // warm-up
  if (!st) {
    (void)hipEventRecord(a, s);
    for (int r = 0; r < 2 && !st; ++r) st = launch();
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    (void)hipEventElapsedTime(ms, a, b);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

static int tuned_choice(Workspace& w, const GemmArgs& g, hipStream_t s, int* choice) {
  FilterTuner& T = filter_tuner();
  const std::pair<int64_t, int64_t> key(g.M, (g.N + 31) / 32);
  std::lock_guard<std::mutex> lock(T.mu);
  auto it = T.best.find(key);
  if (it != T.best.end()) {
    *choice = it->second;
    return kOk;
  }
  if (!w.tune_scratch) {
    int st = w.alloc(&w.tune_scratch, (size_t)w.N * w.ne);
    if (st) return st;
    CHASE_CHK(hipMemsetAsync(w.tune_scratch, 0, sizeof(z64) * (size_t)w.N * w.ne, s));
  }
  GemmArgs t = g;
  t.Y = w.tune_scratch;
  t.ldy = g.M;
  int bestc = kChoiceT0Tail;
  float best_ms = 1e30f;
  for (int c = 0; c < kNumChoices; ++c) {
    float ms = 1e30f;
    int st = time_launches([&]() { return zgemm_nn_big_launch(t, s, true, w.tail_ws, w.tail_counters, c); }, s, &ms);
    if (st) return st;
    if (ms < best_ms) {
      best_ms = ms;
      bestc = c;
    }
  }
  T.best[key] = bestc;
  *choice = bestc;
  return kOk;
}

// Filter (Eq. 1 with the scaled Chebyshev coefficients): the GEMM of every
// degree step.  V: N x n (the final iterate of an even degree lands back in
// V), W: its ping-pong partner; degs ascending.  Step k computes X_{k+1} for
// the columns whose degree exceeds k, a suffix of the block.
static std::vector<GemmArgs> plan_filter(const z64* A, int64_t lda, z64* V, int64_t ldv, z64* W, int64_t ldw,
                                         int64_t N, int64_t n, const int32_t* degs, double c, double e,
                                         double mu1) {
  std::vector<GemmArgs> steps;
  if (n <= 0) return steps;
  const int dmax = degs[n - 1];
  const double sigma1 = e / (mu1 - c);
  double sigma = sigma1;
  int64_t s0 = 0;
  for (int k = 0; k < dmax; ++k) {
    while (s0 < n && degs[s0] < k + 1) ++s0;
    const int64_t cols = n - s0;
    if (cols <= 0) break;
    double alpha, beta;
    if (k == 0) {
      alpha = sigma1 / e;
      beta = 0.0;
    } else {
      const double sigma_next = 1.0 / (2.0 / sigma1 - sigma);
      alpha = 2.0 * sigma_next / e;
      beta = -sigma * sigma_next;
      sigma = sigma_next;
    }
    // X_k lives in V for even k, in W for odd k; X_{k+1} overwrites X_{k-1}.
    const bool cur_in_v = (k % 2 == 0);
    const z64* cur = cur_in_v ? V : W;
    const int64_t ldc = cur_in_v ? ldv : ldw;
    z64* out = cur_in_v ? W : V;
    const int64_t ldo = cur_in_v ? ldw : ldv;
    GemmArgs g;
    g.M = N; g.N = cols; g.K = N;
    g.A = A; g.lda = lda;
    g.B = cur + s0 * ldc; g.ldb = ldc;
    g.Y = out + s0 * ldo; g.ldy = ldo;
    g.Z = cur + s0 * ldc; g.ldz = ldc;
    g.alpha = alpha; g.beta = beta; g.gamma = -alpha * c;
    steps.push_back(g);
  }
  return steps;
}

// The steps of plan_filter on the row-pair view of a real problem (N pairs):
// the B operand is the same memory read as a real block of 2 N rows.
static void as_real_steps(std::vector<GemmArgs>& steps) {
  for (GemmArgs& g : steps) {
    g.K = 2 * g.M;
    g.ldb *= 2;
  }
}

static int run_filter(const z64* A, int64_t lda, z64* V, int64_t ldv, z64* W, int64_t ldw, int64_t N,
                      int64_t n, const int32_t* degs, double c, double e, double mu1, int64_t* matvecs,
                      int64_t* launches, hipStream_t s, void* tail_ws, int* tail_counters, bool real = false,
                      int max_segments = kTailMaxSegments) {
  std::vector<GemmArgs> steps = plan_filter(A, lda, V, ldv, W, ldw, N, n, degs, c, e, mu1);
  if (real) as_real_steps(steps);
  int64_t mv = 0;
  for (const GemmArgs& g : steps) {
    int st = real ? dfilter_big_launch(g, s, tail_ws, tail_counters)
                  : zgemm_nn_big_launch(g, s, true, tail_ws, tail_counters, kChoiceT0Tail, max_segments);
    if (st) return st;
    mv += g.N;
  }
  if (matvecs) *matvecs = mv;
  if (launches) *launches = (int64_t)steps.size();
  return kOk;
}

// log T_k(tau) for tau >= 1, where T_k(tau) = (r^k + r^-k) / 2 with
// r = tau + sqrt(tau^2 - 1); 0 for tau < 1 (|T_k| <= 1 there).  Written so
// that neither r^k nor tau^2 is formed.
static double log_cheb(int k, double tau) {
  if (!(tau > 1.0)) return 0.0;
  const double q = 1.0 / tau;
  const double lr = std::log(tau) + std::log1p(std::sqrt((1.0 - q) * (1.0 + q)));
  return k * lr + std::log1p(std::exp(-2.0 * k * lr)) - std::log(2.0);
}

// Power-of-two range guard of the low-precision recurrence.  The filter is
// normalised at mu1, but mu1 is the smallest Ritz value of the last
// iteration, so eigenvalues below it grow like T_k(t(lambda)) / T_k(t(mu1)),
// which can pass the FP32 range (about 2^128) long before the FP64 one when
// the Ritz values are still far from the spectrum (tiny orders, poor
// starts).  Step k stores 2^-m[k] X_k instead of X_k, with m[k] chosen from
// the bound T_k(t(lam_lo)) / T_k(t(mu1)) so that the stored iterate stays
// below 2^90; the recurrence is linear and homogeneous in (X_k, X_{k-1}), so
// the scalars of each step absorb the ratios and the widening conversion
// multiplies the finished column by 2^m[d] in FP64.  m is zero whenever the
// bound stays below 2^90, which leaves every scalar and value unchanged.
static std::vector<int> lowp_range_exponents(int dmax, double c, double e, double mu1, double lam_lo) {
  std::vector<int> m((size_t)dmax + 1, 0);
  const double tau_lo = std::fabs((lam_lo - c) / e), tau_mu = std::fabs((mu1 - c) / e);
  if (!std::isfinite(tau_lo) || !std::isfinite(tau_mu)) return m;
  for (int k = 1; k <= dmax; ++k) {
    const double log2_growth = (log_cheb(k, tau_lo) - log_cheb(k, tau_mu)) / std::log(2.0);
    m[k] = std::max(0, (int)std::ceil(log2_growth - 90.0));
  }
  return m;
}

// Low-precision filter for the columns still on an FP32 or BF16x3 rung: the
// same recurrence and scalars as plan_filter, on complex64 copies of the
// columns (X0/X1 ping-pong), converted back to complex128 as each column
// reaches its degree.  `launch` runs one step's GEMM; it is told which buffer
// the step reads and the step's first column.  lam_lo: a lower estimate of
// the spectrum for the range guard above.
static int run_filter_lowp(int64_t N, z64* V, int64_t ldv, c32* X0, c32* X1, int64_t n, const int32_t* degs,
                           double c, double e, double mu1, double lam_lo, int64_t* matvecs, int64_t* launches,
                           hipStream_t s, const std::function<int(const CGemmArgs&, bool, int64_t)>& launch) {
  if (n <= 0) return kOk;
  int st = convert_z_to_c(V, ldv, X0, N, N, n, s);
  if (st) return st;
  const int dmax = degs[n - 1];
  const std::vector<int> m = lowp_range_exponents(dmax, c, e, mu1, lam_lo);
  int64_t mv = 0, nl = 0;
  const double sigma1 = e / (mu1 - c);
  double sigma = sigma1;
  int64_t done = 0;  // columns [0, done) already converted back
  for (int k = 0; k < dmax; ++k) {
    int64_t s0 = 0;
    while (s0 < n && degs[s0] < k + 1) ++s0;
    // columns that finished after step k (degree == k, even) sit in X0
    if (s0 > done) {
      st = convert_c_to_z(X0 + done * N, N, V + done * ldv, ldv, N, s0 - done, s, std::ldexp(1.0, m[k]));
      if (st) return st;
      done = s0;
    }
    const int64_t cols = n - s0;
    if (cols <= 0) break;
    double alpha, beta;
    if (k == 0) {
      alpha = sigma1 / e;
      beta = 0.0;
    } else {
      const double sigma_next = 1.0 / (2.0 / sigma1 - sigma);
      alpha = 2.0 * sigma_next / e;
      beta = -sigma * sigma_next;
      sigma = sigma_next;
    }
    // stored iterates carry 2^-m[k]: X_{k+1} from X_k scales by 2^(m[k]-m[k+1]),
    // the X_{k-1} term by 2^(m[k-1]-m[k+1])
    alpha = std::ldexp(alpha, m[k] - m[k + 1]);
    if (k > 0) beta = std::ldexp(beta, m[k - 1] - m[k + 1]);
    const bool cur0 = (k % 2 == 0);
    c32* cur = cur0 ? X0 : X1;
    c32* out = cur0 ? X1 : X0;
    CGemmArgs g;
    g.M = N; g.N = cols; g.K = N;
    g.B = cur + s0 * N; g.ldb = N;
    g.Y = out + s0 * N; g.ldy = N;
    g.Z = cur + s0 * N; g.ldz = N;
    g.alpha = (float)alpha; g.beta = (float)beta; g.gamma = (float)(-alpha * c);
    st = launch(g, cur0, s0);  // cur0: the step reads X0; s0: its first column
    if (st) return st;
    mv += cols;
    ++nl;
  }
  if (n > done) {
    st = convert_c_to_z(X0 + done * N, N, V + done * ldv, ldv, N, n - done, s, std::ldexp(1.0, m[dmax]));
    if (st) return st;
  }
  if (matvecs) *matvecs = mv;
  if (launches) *launches = nl;
  return kOk;
}

// The BF16x3 rung: columns V[:, 0:n) (degrees ascending) through the
// split-product step on the bfloat16 planes of conj(H) in w.P16, with the
// complex64 ping-pong blocks w.X32a / w.X32b and their planes w.XP16a /
// w.XP16b (each step's epilogue writes the planes of the block it produces).
static int filter_rung_bf16(Workspace& w, z64* V, int64_t ldv, int64_t n, const int32_t* degs, double c, double e,
                            double mu1, double lam_lo, int64_t* mv, int64_t* nl, hipStream_t s) {
  const int64_t N = w.N, ldp = w.ldp, xps = w.ldp * w.ne;
  uint16_t* const XP[2] = {w.XP16a, w.XP16b};
  bool first = true;
  auto launch = [&](const CGemmArgs& a, bool cur0, int64_t s0) {
    int r;
    if (first) {  // planes of the starting block (step 0 reads X0 from column 0)
      first = false;
      if ((r = bsplit_block(a.B, a.ldb, a.K, a.N, XP[0], ldp, xps, s))) return r;
    }
    BGemmArgs b;
    b.M = a.M; b.N = a.N; b.K = a.K;
    b.P = w.P16; b.ldp = ldp; b.plane_stride = ldp * N;
    b.X = a.B; b.ldx = a.ldb;
    b.Y = a.Y; b.ldy = a.ldy;
    b.Z = a.Z; b.ldz = a.ldz;
    b.alpha = a.alpha; b.beta = a.beta; b.gamma = a.gamma;
    b.Xp = XP[cur0 ? 0 : 1] + s0 * ldp; b.ldxp = ldp; b.xps = xps;
    b.Yp = XP[cur0 ? 1 : 0] + s0 * ldp; b.ldyp = ldp; b.yps = xps;
    return bfilter_launch(b, s, w.tail_ws, w.tail_counters);
  };
  return run_filter_lowp(N, V, ldv, w.X32a, w.X32b, n, degs, c, e, mu1, lam_lo, mv, nl, s, launch);
}

// The FP32 rung: the same on complex64 H (H32, leading dimension ld32).
static int filter_rung_fp32(Workspace& w, const c32* H32, int64_t ld32, z64* V, int64_t ldv, int64_t n,
                            const int32_t* degs, double c, double e, double mu1, double lam_lo, int64_t* mv,
                            int64_t* nl, hipStream_t s) {
  auto launch = [&](const CGemmArgs& a, bool, int64_t) {
    CGemmArgs b = a;
    b.A = H32;
    b.lda = ld32;
    return cfilter_big_launch(b, s, w.tail_ws, w.tail_counters);
  };
  return run_filter_lowp(w.N, V, ldv, w.X32a, w.X32b, n, degs, c, e, mu1, lam_lo, mv, nl, s, launch);
}

// Gram matrix G = X^H X (Hermitised), X: N x n.
static int gram(Workspace& w, const z64* X, int64_t ldx, int64_t n, hipStream_t s) {
  GemmArgs g;
  g.M = n; g.N = n; g.K = w.N;
  g.A = X; g.lda = ldx;
  g.B = X; g.ldb = ldx;
  g.Y = w.G; g.ldy = n;
  g.real_out = w.real;  // row-pair view: X^T X is the real part
  // lower triangle only: the Cholesky factorisation and the shift read nothing else
  const int splits = choose_splits(n, n, w.N, w.max_splits, true);
  return zgemm_splitk(1, 0, g, w.ws, splits, w.real ? 3 : 2, s);
}

// X <- X R^{-1} with R = L^H from G = L L^H.  Returns 1 in *failed when the
// Cholesky factorisation breaks down (X untouched).
static int chol_apply(Workspace& w, z64* X, int64_t ldx, int64_t n, bool shifted, int* failed,
                      hipStream_t s) {
  int st = kOk;
  if (shifted) {
    st = add_cholqr_shift(w.G, n, n, w.real ? w.rows : w.N, w.shift, s);
    if (st) return st;
  }
  st = potrf_lower(w.G, n, n, w.info, nullptr, s);
  if (st) return st;
  int info = 0;
  CHASE_CHK(hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, s));
  CHASE_CHK(hipStreamSynchronize(s));
  if (info != 0) {
    *failed = 1;
    return kOk;
  }
  *failed = 0;
  st = trtri_lower(w.G, n, w.L, n, n, w.T, s);
  if (st) return st;
  GemmArgs g;  // B = X L^{-H}
  g.M = w.N; g.N = n; g.K = n;
  g.A = X; g.lda = ldx;
  g.B = w.L; g.ldb = n;
  g.Y = w.B; g.ldy = w.N;
  g.upper_b = 1;
  g.real_b = w.real;  // L^{-H} of a real Gram matrix is real-valued
  st = zgemm_launch(0, 1, g, s);
  if (st) return st;
  return copy_columns(w.B, w.N, X, ldx, w.N, n, s);
}

static int cholqr_pass(Workspace& w, z64* X, int64_t ldx, int64_t n, bool shifted, int* failed,
                       hipStream_t s) {
  int st = gram(w, X, ldx, n, s);
  if (st) return st;
  return chol_apply(w, X, ldx, n, shifted, failed, s);
}

static int householder(Workspace& w, z64* X, int64_t ldx, int64_t n, hipStream_t s, z64* R_out = nullptr) {
  HouseholderWs h;
  h.V = w.hhV;
  h.T = w.hhT;
  h.W1 = w.hhW;
  h.W2 = w.hhW + (int64_t)kHouseholderPanel * w.ne;
  h.part = w.hhpart;
  h.rowj = w.hhrow;
  h.tau = w.tau;
  h.Q = w.B;
  h.splitk = w.ws;
  h.R = R_out;
  if (!w.real) return householder_qr(X, ldx, w.N, n, h, s);
  // The real block (2N rows; a zero padding row stays zero) through the same
  // kernels, widened with zero imaginary parts: every norm, reflector, tau and
  // product of real operands then has an exactly zero imaginary part, so Q is
  // the real Householder Q in LAPACK's conventions.
  int st = w.ensure_hh_real();
  if (st) return st;
  const int64_t M = 2 * w.N;
  double* Xr = reinterpret_cast<double*>(X);
  if ((st = widen_real_block(Xr, 2 * ldx, w.hhXc, M, M, n, s))) return st;
  h.V = w.hhVc;
  h.Q = w.hhQc;
  if ((st = householder_qr(w.hhXc, M, M, n, h, s))) return st;
  return real_part_block(w.hhXc, M, Xr, 2 * ldx, M, n, s);
}

// Alg. 4 with escalation on Cholesky failure.
static int caqr(Workspace& w, z64* X, int64_t ldx, int64_t n, double cond, int force, int* variant,
                hipStream_t s) {
  int v = force >= 0 ? force : select_qr(cond);
  int failed = 0, st = kOk;
  while (true) {
    if (v == CHASE_QR_CHOLQR1 || v == CHASE_QR_CHOLQR2) {
      const int passes = v == CHASE_QR_CHOLQR1 ? 1 : 2;
      for (int p = 0; p < passes; ++p) {
        st = cholqr_pass(w, X, ldx, n, false, &failed, s);
        if (st) return st;
        if (failed) break;
      }
      if (!failed) break;
      v = CHASE_QR_SHIFTED;
      continue;
    }
    if (v == CHASE_QR_SHIFTED) {
      st = cholqr_pass(w, X, ldx, n, true, &failed, s);
      if (st) return st;
      for (int p = 0; p < 2 && !failed; ++p) {
        st = cholqr_pass(w, X, ldx, n, false, &failed, s);
        if (st) return st;
      }
      if (!failed) break;
      v = CHASE_QR_HOUSEHOLDER;
      continue;
    }
    st = householder(w, X, ldx, n, s);
    if (st) return st;
    v = CHASE_QR_HOUSEHOLDER;
    break;
  }
  *variant = v;
  return kOk;
}

// Rayleigh-Ritz on the active block plus residuals.  Q (= C2_a on entry,
// orthonormal, N x n) and V (= C_a): on return V holds the Ritz vectors, Q a
// copy of them, theta/resd (device) the Ritz values and residual norms.
// HC = H Q is computed once (Alg. 2's H C); the residual's H V is formed as
// (H Q) W, the same product reassociated.
// The three parts of rayleigh_ritz: the projection (B = H Q, G = Q^H B),
// the n x n eigensolve (W into G, theta) and the rest.
static int rr_project(Workspace& w, const z64* A, int64_t lda, z64* Q, int64_t ldq, int64_t n, hipStream_t s) {
  if (n <= 0) return kOk;
  const int64_t N = w.N;
  GemmArgs g;  // B = H Q
  g.M = N; g.N = n; g.K = N;
  g.A = A; g.lda = lda;
  g.B = Q; g.ldb = ldq;
  g.Y = w.B; g.ldy = N;
  int st;
  if (w.c64) {  // H Q in FP32 from the complex64 H, back to FP64
    if ((st = convert_z_to_c(Q, ldq, w.X32a, N, N, n, s))) return st;
    CGemmArgs c;
    c.M = N; c.N = n; c.K = N;
    c.A = w.H32; c.lda = w.ldh32;
    c.B = w.X32a; c.ldb = N;
    c.Y = w.X32b; c.ldy = N;
    c.Z = w.X32b; c.ldz = N;
    c.alpha = 1.0f; c.beta = 0.0f; c.gamma = 0.0f;
    if ((st = cfilter_big_launch(c, s, w.tail_ws, w.tail_counters))) return st;
    st = convert_c_to_z(w.X32b, N, w.B, N, N, n, s);
  } else if (w.real) {
    g.K = 2 * N;
    g.ldb = 2 * ldq;
    st = dfilter_big_launch(g, s, w.tail_ws, w.tail_counters);
  } else {
    st = zgemm_nn_big_launch(g, s, false, w.tail_ws, w.tail_counters);
  }
  if (st) return st;
  GemmArgs q;  // G = Q^H B, lower triangle (the eigensolver reads nothing else)
  q.M = n; q.N = n; q.K = N;
  q.A = Q; q.lda = ldq;
  q.B = w.B; q.ldb = N;
  q.Y = w.G; q.ldy = n;
  q.real_out = w.real;
  return zgemm_splitk(1, 0, q, w.ws, choose_splits(n, n, N, w.max_splits, true), w.real ? 3 : 2, s);
}

// The quotient's eigensolve (Alg. 2): ascending Ritz values into w.theta and
// the eigenvectors over w.G, by the block-Jacobi kernels of heevj.hip.  The
// real variant's quotient has zero imaginary parts, which the complex plane
// rotations keep at zero, so its eigenvectors come out real.
static int rr_eigensolve(Workspace& w, int64_t n, hipStream_t s) {
  if (n <= 0) return kOk;
  return heevj(w.G, n, n, w.theta, w.jacws, &w.jac_sweeps, s);
}

static int rr_finish(Workspace& w, z64* Q, int64_t ldq, z64* V, int64_t ldv, int64_t n, hipStream_t s) {
  if (n <= 0) return kOk;
  const int64_t N = w.N;
  int st;
  GemmArgs b;  // V = Q W
  b.M = N; b.N = n; b.K = n;
  b.A = Q; b.lda = ldq;
  b.B = w.G; b.ldb = n;
  b.Y = V; b.ldy = ldv;
  b.real_b = w.real;  // eigenvectors of the real quotient
  st = zgemm_launch(0, 0, b, s);
  if (st) return st;
  GemmArgs hv;  // Q <- (H Q) W = H V
  hv.M = N; hv.N = n; hv.K = n;
  hv.A = w.B; hv.lda = N;
  hv.B = w.G; hv.ldb = n;
  hv.Y = Q; hv.ldy = ldq;
  hv.real_b = w.real;
  st = zgemm_launch(0, 0, hv, s);
  if (st) return st;
  st = residual_norms(Q, ldq, V, ldv, w.theta, N, n, w.resd, s);
  if (st) return st;
  return copy_columns(V, ldv, Q, ldq, N, n, s);
}

static int rayleigh_ritz(Workspace& w, const z64* A, int64_t lda, z64* Q, int64_t ldq, z64* V, int64_t ldv,
                         int64_t n, hipStream_t s) {
  int st;
  if ((st = rr_project(w, A, lda, Q, ldq, n, s)) || (st = rr_eigensolve(w, n, s))) return st;
  return rr_finish(w, Q, ldq, V, ldv, n, s);
}

static int lanczos(Workspace& w, const z64* A, int64_t lda, const z64* starts, int64_t lds, int nstarts,
                   int ksteps, int ne, double out[4], hipStream_t s) {
  const int64_t N = w.N;
  const int64_t order = w.real ? w.rows : N;
  ksteps = (int)std::min<int64_t>(ksteps, order);
  if (nstarts < 1 || nstarts > 8 || ksteps < 1 || ksteps > 256) return -1;
  int st = lanczos_init(starts, lds, w.lzV, w.lzVold, N, nstarts, s);
  if (st) return st;
  for (int j = 0; j < ksteps; ++j) {
    if (w.real)
      st = symv_block(w.Hr, w.ldhr, reinterpret_cast<const double*>(w.lzV), 2 * N, reinterpret_cast<double*>(w.lzW),
                      2 * N, w.rows, 2 * N, nstarts, s);
    else if (w.c64)
      st = hemv_block_c64(w.H32, w.ldh32, w.lzV, N, w.lzW, N, N, nstarts, s);
    else
      st = hemv_block(A, lda, w.lzV, N, w.lzW, N, N, nstarts, s);
    if (st) return st;
    st = lanczos_step(w.lzV, w.lzVold, w.lzW, N, nstarts, j, ksteps, w.lz_alpha, w.lz_beta, s);
    if (st) return st;
  }
  std::vector<double> al((size_t)nstarts * ksteps), be((size_t)nstarts * ksteps);
  CHASE_CHK(hipMemcpyAsync(al.data(), w.lz_alpha, al.size() * 8, hipMemcpyDeviceToHost, s));
  CHASE_CHK(hipMemcpyAsync(be.data(), w.lz_beta, be.size() * 8, hipMemcpyDeviceToHost, s));
  CHASE_CHK(hipStreamSynchronize(s));
  for (double x : al)
    if (!std::isfinite(x)) return kBreakdown;
  bounds_from_lanczos(al, be, nstarts, ksteps, order, ne, out);
  return kOk;
}

static int apply_perm(Workspace& w, z64* X, int64_t ldx, const std::vector<int>& perm, bool also_c2,
                      int64_t c2_off, hipStream_t s) {
  const int64_t n = (int64_t)perm.size();
  if (n == 0) return kOk;
  CHASE_CHK(hipMemcpyAsync(w.perm, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  int st = gather_columns(X, ldx, w.B, w.N, w.perm, w.N, n, s);
  if (st) return st;
  st = copy_columns(w.B, w.N, X, ldx, w.N, n, s);
  if (st) return st;
  if (also_c2) st = copy_columns(w.B, w.N, w.C2 + c2_off * w.N, w.N, w.N, n, s);
  // the host vector must outlive the async copy
  CHASE_CHK(hipStreamSynchronize(s));
  return st;
}

struct PhaseTimer {
  hipEvent_t a = nullptr, b = nullptr;
  double acc = 0.0;
  bool pending = false;
  int init() {
    CHASE_CHK(hipEventCreate(&a));
    CHASE_CHK(hipEventCreate(&b));
    return kOk;
  }
  void start(hipStream_t s) { (void)hipEventRecord(a, s); }
  void stop(hipStream_t s) {
    (void)hipEventRecord(b, s);
    pending = true;
  }
  void collect() {  // after a synchronisation point
    if (!pending) return;
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) == hipSuccess) acc += ms * 1e-3;
    pending = false;
  }
  void destroy() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

static bool valid_params(const chase_params_t* p) {
  if (!p) return false;
  if (p->nev < 1 || p->nex < 0) return false;
  if (p->deg < 2 || p->deg % 2 || p->max_deg < 2 || p->max_deg % 2) return false;
  if (!(p->tol > 0)) return false;
  if (p->max_iter < 1 || p->lanczos_steps < 1 || p->lanczos_steps > 256) return false;
  if (p->precision != CHASE_FP64 && p->precision != CHASE_FP32_MIXED && p->precision != CHASE_BF16X3_MIXED)
    return false;
  if (p->force_qr < -1 || p->force_qr > 3) return false;
  return true;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Exact condition number sigma_max / sigma_min of the N x n block X (trace
// level 2): X (or X with unit columns) is copied and factored by Householder
// QR; the singular values of R are the non-negative eigenvalues of the
// Hermitian [[0, R], [R^H, 0]], found by the block-Jacobi eigensolver (to
// within a few ulps of sigma_max, as an SVD's).  w.theta and w.resd serve as
// scratch for the column norms; w.B holds Q.
static int kappa_of_block(Workspace& w, const z64* X, int64_t ldx, int64_t n, bool equilibrate, hipStream_t s,
                          double* kappa) {
  int st = kOk;
  if (n <= 0) {
    *kappa = std::nan("");
    return kOk;
  }
  if ((st = w.ensure_trace())) return st;
  if (equilibrate) {
    std::vector<double> g(n, 0.0);
    CHASE_CHK(hipMemcpyAsync(w.theta, g.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    if ((st = residual_norms(X, ldx, X, ldx, w.theta, w.N, n, w.resd, s))) return st;  // ||x_j - 0 x_j||
    CHASE_CHK(hipMemcpyAsync(g.data(), w.resd, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    CHASE_CHK(hipStreamSynchronize(s));
    for (double& v : g) v = v > 0 ? 1.0 / v : 0.0;
    CHASE_CHK(hipMemcpyAsync(w.theta, g.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    if ((st = scale_columns(X, ldx, w.theta, w.trX, w.N, w.N, n, s))) return st;
    CHASE_CHK(hipStreamSynchronize(s));  // g is read by the copy before it goes
  } else if ((st = copy_columns(X, ldx, w.trX, w.N, w.N, n, s))) {
    return st;
  }
  if ((st = householder(w, w.trX, w.N, n, s, w.trR))) return st;
  if ((st = augment_hermitian(w.trR, n, w.trAug, s))) return st;
  int sweeps = 0;
  if ((st = heevj(w.trAug, 2 * n, 2 * n, w.trTheta, w.trJac, &sweeps, s))) return st;
  std::vector<double> ev(2 * n);
  CHASE_CHK(hipMemcpyAsync(ev.data(), w.trTheta, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s));
  CHASE_CHK(hipStreamSynchronize(s));
  // ascending: -sigma_1 .. -sigma_n, sigma_n .. sigma_1
  const double hi = ev[2 * n - 1], lo = std::fabs(ev[n]);
  *kappa = lo > 0 ? hi / lo : std::numeric_limits<double>::infinity();
  return kOk;
}

// State of one problem's ChASE loop (Alg. 2).  The single solve and the
// batched solve drive the same steps; only the filter launch differs.
// CHASE_LOG=1 in the environment (read once): one line per outer iteration
// on stderr.
static bool chase_log_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("CHASE_LOG");
    return v != nullptr && v[0] != '\0' && v[0] != '0';
  }();
  return on;
}

struct ProblemState {
  Workspace* w = nullptr;
  chase_params_t P{};
  const z64* A = nullptr;
  int64_t lda = 0;
  z64* V = nullptr;
  int64_t ldv = 0;
  int64_t N = 0;
  int nev = 0, ne = 0;
  bool mixed = false;
  std::vector<int32_t> degs;
  std::vector<double> Lam, resd, prev_resd, th_h, rs_h;
  std::vector<char> low;  // precision rung of each column: 2 BF16x3, 1 FP32, 0 FP64
  // Rayleigh-Ritz returns the active pairs in ascending Ritz value.  origin[j]
  // is that rank for the pair in column j (its column index before the first
  // iteration); it moves with the column through every permutation.
  std::vector<int> origin;
  std::vector<int> sort_order;  // the permutation prepare() applied this iteration (empty: none)
  int locked = 0, it = 1;
  double bnd[4] = {0, 0, 0, 0};
  double b_sup = 0, mu_ne = 0, c = 0, e = 1, mu1_cur = 0, tol_abs = 0, sw_abs = 0, sw16_abs = 0;
  bool breakdown = false;
  chase_stats_t S{};
  int64_t total_mv = 0;
  PhaseTimer t_lz, t_f, t_qr, t_rr;
  int trace_level = 0;
  std::vector<chase_trace_t>* trace = nullptr;
  std::vector<chase_trace_column_t>* trace_cols = nullptr;  // per traced iteration, its active columns
  std::vector<int64_t>* trace_col_off = nullptr;            // start of each iteration's columns
  chase_trace_t rec{};  // the iteration being traced
  const c32* A32 = nullptr;  // H for the FP32 rung: the library's copy, or a complex64 caller's own
  int64_t lda32 = 0;

  int init_timers() {
    int st;
    for (PhaseTimer* t : {&t_lz, &t_f, &t_qr, &t_rr})
      if ((st = t->init())) return st;
    return kOk;
  }
  void destroy_timers() {
    for (PhaseTimer* t : {&t_lz, &t_f, &t_qr, &t_rr}) t->destroy();
  }
  void collect_timers() {
    for (PhaseTimer* t : {&t_lz, &t_f, &t_qr, &t_rr}) t->collect();
  }
  bool active() const { return !breakdown && locked < nev && it <= P.max_iter; }
  int na() const { return ne - locked; }

  template <class T>
  void permute_active(std::vector<T>& arr, const std::vector<int>& order) {
    std::vector<T> tmp(arr.begin() + locked, arr.end());
    for (int j = 0; j < na(); ++j) arr[locked + j] = tmp[order[j]];
  }
  template <class T>
  void unpermute_active(std::vector<T>& arr, const std::vector<int>& order) {
    std::vector<T> tmp(arr.begin() + locked, arr.end());
    for (int j = 0; j < na(); ++j) arr[locked + order[j]] = tmp[j];
  }
  void permute_state(const std::vector<int>& order) {
    permute_active(Lam, order);
    permute_active(resd, order);
    permute_active(degs, order);
    permute_active(low, order);
    permute_active(prev_resd, order);
    permute_active(origin, order);
  }
  void unpermute_state(const std::vector<int>& order) {
    unpermute_active(Lam, order);
    unpermute_active(resd, order);
    unpermute_active(degs, order);
    unpermute_active(low, order);
    unpermute_active(prev_resd, order);
    unpermute_active(origin, order);
  }

  // Initial block, Lanczos bounds (Alg. 2 first line), FP32 copy of H.
  int setup(int use_v0, const z64* starts, int64_t lds, int nstarts, hipStream_t s) {
    int st = kOk;
    N = w->N;
    nev = P.nev;
    ne = P.nev + P.nex;
    mixed = P.precision != CHASE_FP64 || w->c64;
    // degree-optimisation margin: a negative value asks for the measured
    // default of the ladder (4 with every column in FP64, 2 with FP32 or
    // BF16x3 rungs)
    if (P.deg_extra < 0) P.deg_extra = mixed ? 2 : 4;
    std::memset(&S, 0, sizeof(S));
    if (!use_v0 && (st = fill_gaussian(V, ldv, N, ne, P.seed, s))) return st;
    if (!use_v0 && (st = zero_pad_row(V, ldv, ne, s))) return st;
    if (P.bounds_given) {
      bnd[0] = P.b_sup;
      bnd[1] = P.mu_1;
      bnd[2] = P.mu_ne;
      bnd[3] = P.norm_est;
    } else {
      int64_t ld = lds;
      int ns = nstarts;
      if (!starts) {
        if ((st = fill_gaussian(w->starts, N, N, 4, P.seed ^ 0x5DEECE66Dull, s))) return st;
        if ((st = zero_pad_row(w->starts, N, 4, s))) return st;
        starts = w->starts;
        ld = N;
        ns = 4;
      }
      t_lz.start(s);
      if ((st = lanczos(*w, A, lda, starts, ld, ns, P.lanczos_steps, ne, bnd, s))) return st;
      t_lz.stop(s);
      total_mv += (int64_t)ns * std::min<int64_t>(P.lanczos_steps, w->real ? w->rows : N);
    }
    b_sup = bnd[0];
    mu1_cur = bnd[1];
    mu_ne = bnd[2];
    tol_abs = P.tol * bnd[3];
    sw_abs = P.mixed_switch * bnd[3];
    sw16_abs = P.bf16_switch * bnd[3];
    c = 0.5 * (b_sup + mu_ne);
    e = 0.5 * (b_sup - mu_ne);
    if (w->c64) {
      A32 = w->H32;
      lda32 = w->ldh32;
    } else if (mixed) {
      A32 = w->A32;
      lda32 = N;
      if ((st = convert_z_to_c(A, lda, w->A32, N, N, N, s))) return st;
    }
    if (P.precision == CHASE_BF16X3_MIXED && (st = bsplit_planes(A, lda, N, w->P16, s))) return st;
    degs.assign(ne, P.deg);
    Lam.assign(ne, 0.0);
    resd.assign(ne, std::numeric_limits<double>::infinity());
    prev_resd = resd;
    low.assign(ne, w->c64 ? (char)1 : (char)P.precision);  // complex64: every column on the FP32 rung
    // With nex = 0 the largest Ritz value is a wanted one, and from the second
    // iteration on it is the lower end of the damped interval [mu_ne, b_sup]:
    // the filter then no longer separates that pair from the eigenvalues above
    // it, so the rounding a low rung leaves in it could never be filtered out.
    // Its column (the largest Ritz value after the first Rayleigh-Ritz) runs in
    // FP64 from the start.
    if (mixed && !w->c64 && P.nex == 0) low[ne - 1] = 0;
    origin.resize(ne);
    std::iota(origin.begin(), origin.end(), 0);
    sort_order.clear();
    th_h.assign(ne, 0.0);
    rs_h.assign(ne, 0.0);
    return copy_columns(V, ldv, w->C2, N, N, ne, s);
  }

  // Iteration prologue (iterations after the first): new bounds, degree
  // optimisation and the stable sort of the active columns by degree.
  int prepare(hipStream_t s) {
    if (it == 1) return kOk;
    mu1_cur = *std::min_element(Lam.begin(), Lam.end());
    mu_ne = *std::max_element(Lam.begin(), Lam.end());
    c = 0.5 * (b_sup + mu_ne);
    e = 0.5 * (b_sup - mu_ne);
    if (P.opt)
      for (int j = locked; j < ne; ++j) degs[j] = degree_opt(resd[j], Lam[j], c, e, tol_abs, P.max_deg, P.deg_extra);
    std::vector<int> order(na());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      if (mixed && low[locked + x] != low[locked + y]) return low[locked + x] > low[locked + y];
      return degs[locked + x] < degs[locked + y];
    });
    bool ident = true;
    for (int j = 0; j < na(); ++j) ident = ident && order[j] == j;
    sort_order.clear();
    if (ident) return kOk;
    int st = apply_perm(*w, V + (int64_t)locked * ldv, ldv, order, false, 0, s);
    if (st) return st;
    permute_state(order);
    sort_order = order;
    return kOk;
  }

  // Real problems: the padding row of an odd order (the last real row of
  // the row-pair layout) is kept at zero.
  int zero_pad_row(z64* X, int64_t ldx, int64_t n, hipStream_t s) {
    if (!w->real || w->rows % 2 == 0) return kOk;
    double* Xr = reinterpret_cast<double*>(X);
    return dcopy_pad(Xr, 2 * ldx, w->rows, n, Xr, 2 * ldx, 2 * N, n, s);
  }

  // active columns on rung r (contiguous: the sort puts higher rungs first)
  int n_rung(int r) const {
    int k = 0;
    for (int j = 0; j < na(); ++j) k += (low[locked + j] == r);
    return k;
  }
  int n_low() const { return n_rung(1) + n_rung(2); }

  // Lower estimate of the spectrum for the low-precision range guard: the
  // smaller of the Lanczos estimate and the current mu1, less 1% of the span.
  double lam_lo() const {
    const double lo = std::min(bnd[1], mu1_cur);
    return lo - 0.01 * std::fabs(b_sup - lo);
  }

  // FP64 filter GEMMs of this iteration (the columns not in FP32).
  std::vector<GemmArgs> plan() {
    const int nl = mixed ? n_low() : 0;
    std::vector<GemmArgs> steps = plan_filter(A, lda, V + (int64_t)(locked + nl) * ldv, ldv,
                                              w->B + (int64_t)(locked + nl) * N, N, N, na() - nl,
                                              degs.data() + locked + nl, c, e, mu1_cur);
    if (w->real) as_real_steps(steps);
    return steps;
  }

  // Filter launched eagerly on `s` (single-problem solve).
  int filter_eager(hipStream_t s) {
    t_f.start(s);
    int st = kOk;
    int64_t mv = 0, nl = 0;
    const int n16 = mixed ? n_rung(2) : 0, n32 = mixed ? n_rung(1) : 0;
    if (n16 > 0) {
      int64_t mv16 = 0, nl16 = 0;
      if ((st = filter_rung_bf16(*w, V + (int64_t)locked * ldv, ldv, n16, degs.data() + locked, c, e, mu1_cur,
                                 lam_lo(), &mv16, &nl16, s)))
        return st;
      S.filter_matvecs_bf16 += mv16;
      mv += mv16;
      nl += nl16;
    }
    if (n32 > 0) {
      int64_t mv32 = 0, nl32 = 0;
      if ((st = filter_rung_fp32(*w, A32, lda32, V + (int64_t)(locked + n16) * ldv, ldv, n32,
                                 degs.data() + locked + n16, c, e, mu1_cur, lam_lo(), &mv32, &nl32, s)))
        return st;
      S.filter_matvecs_fp32 += mv32;
      mv += mv32;
      nl += nl32;
    }
    for (const GemmArgs& g : plan()) {
      if (w->real) {
        if ((st = dfilter_big_launch(g, s, w->tail_ws, w->tail_counters))) return st;
        mv += g.N;
        ++nl;
        continue;
      }
      int choice = kChoiceT0Tail;
      if (P.autotune && (st = tuned_choice(*w, g, s, &choice))) return st;
      if ((st = zgemm_nn_big_launch(g, s, true, w->tail_ws, w->tail_counters, choice))) return st;
      mv += g.N;
      ++nl;
    }
    t_f.stop(s);
    S.filter_matvecs += mv;
    S.filter_launches += nl;
    total_mv += mv;
    return kOk;
  }

  // CondEst, 1D-CAQR, restore/save, Rayleigh-Ritz, residuals, locking.
  int post_filter(hipStream_t s) {
    int st;
    if ((st = post_filter_a(s)) || (st = rr_eigensolve(*w, na(), s))) return st;
    S.eig_sweeps += w->jac_sweeps;
    rec.eig_sweeps = w->jac_sweeps;
    return post_filter_b(s);
  }

  // The part of post_filter up to the Rayleigh-Ritz projection (the n_a x n_a
  // quotient in w->G), and the part after its eigensolve.
  double acc0[3] = {0, 0, 0};  // phase timers when the iteration's trace record began
  double log_cond = 0;          // this iteration's CondEst and filter degree range (CHASE_LOG)
  int log_dmin = 0, log_dmax = 0;
  int post_filter_a(hipStream_t s) {
    int st = kOk;
    std::vector<double> Lam_est = Lam;
    if (it == 1) std::fill(Lam_est.begin(), Lam_est.end(), mu1_cur);
    const double cond = cond_est(Lam_est.data(), c, e, degs.data(), ne, locked);
    log_cond = cond;
    log_dmin = log_dmax = 0;
    if (na() > 0) {
      log_dmin = *std::min_element(degs.begin() + locked, degs.end());
      log_dmax = *std::max_element(degs.begin() + locked, degs.end());
    }
    acc0[0] = t_f.acc;
    acc0[1] = t_qr.acc;
    acc0[2] = t_rr.acc;
    if (trace_level > 0) {
      rec = chase_trace_t{};
      rec.iteration = it;
      rec.locked = locked;
      rec.n_active = na();
      for (int j = locked; j < ne; ++j) rec.filter_matvecs += degs[j];
      rec.kappa_est = cond;
      rec.kappa_com = rec.kappa_com_active = rec.kappa_com_equil = std::nan("");
      if (trace_cols && trace_col_off && trace->size() < CHASE_TRACE_MAX) {
        trace_col_off->push_back((int64_t)trace_cols->size());
        for (int j = locked; j < ne; ++j) {
          chase_trace_column_t col{};
          col.origin = origin[j];
          col.rung = mixed ? low[j] : 0;
          col.degree = degs[j];
          col.ritz = Lam[j];
          col.resid = resd[j];
          trace_cols->push_back(col);
        }
      }
      if (trace_level > 1) {
        if ((st = kappa_of_block(*w, V, ldv, ne, false, s, &rec.kappa_com))) return st;
        if ((st = kappa_of_block(*w, V + (int64_t)locked * ldv, ldv, na(), false, s, &rec.kappa_com_active)))
          return st;
        if ((st = kappa_of_block(*w, V, ldv, ne, true, s, &rec.kappa_com_equil))) return st;
      }
    }
    t_qr.start(s);
    int variant = 0;
    if ((st = caqr(*w, V, ldv, ne, cond, P.force_qr, &variant, s))) return st;
    t_qr.stop(s);
    S.qr_count[variant] += 1;
    rec.qr_variant = variant;

    // restore the locked columns, save the new active ones
    if (locked > 0 && (st = copy_columns(w->C2, N, V, ldv, N, locked, s))) return st;
    if ((st = copy_columns(V + (int64_t)locked * ldv, ldv, w->C2 + (int64_t)locked * N, N, N, na(), s))) return st;

    t_rr.start(s);
    return rr_project(*w, A, lda, w->C2 + (int64_t)locked * N, N, na(), s);
  }

  int post_filter_b(hipStream_t s) {
    int st;
    if ((st = rr_finish(*w, w->C2 + (int64_t)locked * N, N, V + (int64_t)locked * ldv, ldv, na(), s))) return st;
    t_rr.stop(s);
    total_mv += 2 * (int64_t)na();
    CHASE_CHK(hipMemcpyAsync(th_h.data(), w->theta, na() * sizeof(double), hipMemcpyDeviceToHost, s));
    CHASE_CHK(hipMemcpyAsync(rs_h.data(), w->resd, na() * sizeof(double), hipMemcpyDeviceToHost, s));
    CHASE_CHK(hipStreamSynchronize(s));
    collect_timers();
    if (trace_level > 0 && trace && trace->size() < CHASE_TRACE_MAX) {
      rec.t_filter = t_f.acc - acc0[0];  // the filter's events are collected here
      rec.t_qr = t_qr.acc - acc0[1];
      rec.t_rr = t_rr.acc - acc0[2];
      trace->push_back(rec);
    }
    // Rayleigh-Ritz returned the pairs in ascending Ritz value, the order the
    // active columns had before prepare() sorted them: undo that sort on the
    // per-pair state, so that each pair keeps its own rung and residual.
    if (!sort_order.empty()) {
      unpermute_state(sort_order);
      sort_order.clear();
    }
    for (int j = 0; j < na(); ++j) {
      Lam[locked + j] = th_h[j];
      prev_resd[locked + j] = resd[locked + j];
      resd[locked + j] = rs_h[j];
      origin[locked + j] = j;
      if (!std::isfinite(th_h[j]) || !std::isfinite(rs_h[j])) breakdown = true;
    }
    if (breakdown) return kOk;
    if (mixed && !w->c64)
      for (int j = locked; j < ne; ++j) {
        // one rung down once the pair stops improving (residual above half
        // the previous one); below a rung's floor it leaves that rung at once
        int r = low[j];
        if (r > 0 && resd[j] > 0.5 * prev_resd[j]) --r;
        if (r == 2 && resd[j] <= sw16_abs) r = 1;
        if (r == 1 && resd[j] <= sw_abs) r = 0;
        low[j] = (char)r;
      }

    // Deflation and locking
    std::vector<int> order;
    std::vector<char> taken(na(), 0);
    int n_new = 0;
    for (int j = 0; j < std::min(nev - locked, na()); ++j)
      if (resd[locked + j] <= tol_abs) {
        order.push_back(j);
        taken[j] = 1;
        ++n_new;
      }
    for (int j = 0; j < na(); ++j)
      if (!taken[j]) order.push_back(j);
    if (n_new > 0) {
      bool ident = true;
      for (int j = 0; j < na(); ++j) ident = ident && order[j] == j;
      if (!ident) {
        if ((st = apply_perm(*w, V + (int64_t)locked * ldv, ldv, order, true, locked, s))) return st;
        permute_state(order);
      }
    }
    if (chase_log_enabled()) {
      static const char* const kQr[4] = {"CholQR", "CholQR2", "sCholQR2", "HHQR"};
      double rmin = INFINITY, rmax = 0.0;
      for (int j = locked; j < ne; ++j) {
        rmin = std::min(rmin, resd[j]);
        rmax = std::max(rmax, resd[j]);
      }
      std::fprintf(stderr,
                   "[chase] N=%lld nev=%d it %d: locked %d (+%d) of %d, CondEst %.3g -> %s, resid %.2e..%.2e "
                   "(tol %.2e), degrees %d..%d, Jacobi sweeps %d\n",
                   (long long)N, nev, it, locked + n_new, n_new, nev, log_cond,
                   kQr[rec.qr_variant & 3], rmin, rmax, tol_abs, log_dmin, log_dmax, w->jac_sweeps);
    }
    locked += n_new;
    ++it;
    return kOk;
  }

  // Output: the nev lowest pairs, ascending, in V[:, 0:nev].
  int finish(double* ritzv, double* resid, hipStream_t s) {
    const bool converged = locked >= nev;
    std::vector<int> idx(converged ? locked : ne);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return Lam[x] < Lam[y]; });
    idx.resize(nev);
    int st = apply_perm(*w, V, ldv, idx, false, 0, s);
    if (st) return st;
    for (int j = 0; j < nev; ++j) {
      ritzv[j] = Lam[idx[j]];
      resid[j] = resd[idx[j]];
    }
    collect_timers();
    S.status = breakdown ? kBreakdown : (converged ? kOk : kNotConverged);
    S.iterations = it - 1;
    S.locked = locked;
    S.total_matvecs = total_mv;
    S.filter_flops = w->real ? 2.0 * (double)w->rows * (double)w->rows * (double)S.filter_matvecs
                             : 8.0 * (double)N * (double)N * (double)S.filter_matvecs;
    S.t_lanczos = t_lz.acc;
    S.t_filter += t_f.acc;
    S.t_qr = t_qr.acc;
    S.t_rr = t_rr.acc;
    S.t_resid = 0.0;  // inside the Rayleigh-Ritz phase: the residual reuses H C2
    for (int i = 0; i < 4; ++i) S.bounds[i] = bnd[i];
    return kOk;
  }
};

static int check_solve_args(int64_t N, const void* A, int64_t lda, const void* V, int64_t ldv, const void* starts,
                            int64_t ld_starts, int32_t nstarts, const double* ritzv, const double* resid) {
  if (!A || !aligned16(A)) return -2;
  if (lda < N) return -3;
  if (!V || !aligned16(V)) return -4;
  if (ldv < N) return -5;
  if (starts && !aligned16(starts)) return -7;
  if (starts && ld_starts < N) return -8;
  if (starts && (nstarts < 1 || nstarts > 8)) return -9;
  if (!ritzv) return -10;
  if (!resid) return -11;
  return kOk;
}

// Argument checks of chase_filter (and of its allocation-free variant).
int filter_check_args(const void* A, int64_t lda, const void* V, int64_t ldv, const void* W, int64_t ldw, int64_t N,
                      int64_t n, const int32_t* degs, double e) {
  if (!A || !aligned16(A)) return -1;
  if (lda < N) return -2;
  if (!V || !aligned16(V)) return -3;
  if (ldv < N) return -4;
  if (!W || !aligned16(W)) return -5;
  if (ldw < N) return -6;
  if (N < 1) return -7;
  if (n < 0) return -8;
  if (n > 0 && !degs) return -9;
  // even degrees >= 2, ascending: every column's last iterate lands in V
  for (int64_t j = 0; j < n; ++j)
    if (degs[j] < 2 || degs[j] % 2 || (j > 0 && degs[j] < degs[j - 1])) return -9;
  if (!(e > 0)) return -11;
  return kOk;
}

// The complex filter on caller-owned tail scratch (max_segments partial tiles
// at tail_ws, kTailCounterInts counters), enqueued on s without waiting.  The
// counters are cleared by a fill kernel first.
int filter_on_scratch(const void* A, int64_t lda, void* V, int64_t ldv, void* W, int64_t ldw, int64_t N, int64_t n,
                      const int32_t* degs, double c, double e, double mu_1, int64_t* matvecs, void* tail_ws,
                      int* tail_counters, int max_segments, hipStream_t s) {
  int st = tail_counters_init(tail_counters, s);
  int64_t mv = 0, nl = 0;
  if (!st)
    st = run_filter(reinterpret_cast<const z64*>(A), lda, reinterpret_cast<z64*>(V), ldv,
                    reinterpret_cast<z64*>(W), ldw, N, n, degs, c, e, mu_1, &mv, &nl, s, tail_ws, tail_counters,
                    false, max_segments);
  if (st < 0) {  // a launch refused a split larger than the scratch (the planner keeps to the cap)
    set_msg("chase_filter_noalloc: a step's split-K tail needs more partial tiles than the scratch holds");
    return -12;
  }
  if (!st && matvecs) *matvecs = mv;
  return st;
}

}  // namespace chase

using namespace chase;

struct chase_handle_s {
  Workspace w;
  chase_params_t p;
  bool real = false;  // created by chase_create_real
  bool c64 = false;   // created by chase_create_c64
  int trace_level = 0;
  std::vector<chase_trace_t> trace;  // of the last solve
  std::vector<chase_trace_column_t> trace_cols;  // its active columns, iteration after iteration
  std::vector<int64_t> trace_col_off;            // where each iteration's columns start
};

extern "C" {

int chase_default_params(chase_params_t* p) {
  if (!p) return -1;
  std::memset(p, 0, sizeof(*p));
  p->nev = 1;
  p->nex = 0;
  p->deg = 20;
  p->max_deg = 36;
  p->deg_extra = -1;
  p->max_iter = 25;
  p->opt = 1;
  p->precision = CHASE_FP64;
  p->lanczos_steps = 25;
  p->force_qr = CHASE_QR_AUTO;
  p->bounds_given = 0;
  p->tol = 1e-10;
  p->mixed_switch = 5e-6;
  p->bf16_switch = 5e-5;
  p->seed = 2309;
  return 0;
}

int chase_create(int64_t N, const chase_params_t* p, chase_handle_t* h) {
  if (N < 2) return -1;
  if (!valid_params(p) || (int64_t)p->nev + p->nex >= N) return -2;
  if (!h) return -3;
  auto* hh = new chase_handle_s();
  hh->p = *p;
  int st = hh->w.create(N, p->nev + p->nex, p->precision != CHASE_FP64, true,
                        p->precision == CHASE_BF16X3_MIXED);
  if (st) {
    delete hh;
    *h = nullptr;
    return st;
  }
  *h = hh;
  return kOk;
}

int chase_workspace_bytes(int64_t N, const chase_params_t* p, int32_t variant, int64_t* bytes) {
  if (N < 2) return -1;
  if (!valid_params(p) || (int64_t)p->nev + p->nex >= N) return -2;
  if (variant < 0 || variant > 2) return -3;
  if (!bytes) return -4;
  if (variant == 1 && p->precision != CHASE_FP64) return -2;
  if (variant == 2 && p->precision == CHASE_BF16X3_MIXED) return -2;
  Workspace w;
  w.counting = true;
  const int ne = p->nev + p->nex;
  int st;
  if (variant == 0) {
    st = w.create(N, ne, p->precision != CHASE_FP64, true, p->precision == CHASE_BF16X3_MIXED);
  } else if (variant == 1) {
    st = w.create_real(N, ne);
    if (!st && N % 2 != 0) st = w.ensure_hpad();  // an odd order always solves on a padded copy of H
  } else {
    st = w.create_c64(N, ne);
  }
  if (st) return st;
  *bytes = (int64_t)w.counted;
  return kOk;
}

int chase_destroy(chase_handle_t h) {
  if (!h) return -1;
  h->w.release();
  delete h;
  return kOk;
}

int chase_solve(chase_handle_t h, const void* A_, int64_t lda, void* V_, int64_t ldv, int32_t use_v0,
                const void* starts_, int64_t ld_starts, int32_t nstarts, double* ritzv, double* resid,
                chase_stats_t* stats, chase_stream_t stream_) {
  if (!h || h->real || h->c64) return -1;
  int st = check_solve_args(h->w.N, A_, lda, V_, ldv, starts_, ld_starts, nstarts, ritzv, resid);
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
  ProblemState ps;
  ps.w = &h->w;
  ps.P = h->p;
  ps.trace_level = h->trace_level;
  ps.trace = &h->trace;
  ps.trace_cols = &h->trace_cols;
  ps.trace_col_off = &h->trace_col_off;
  h->trace.clear();
  h->trace_cols.clear();
  h->trace_col_off.clear();
  ps.A = reinterpret_cast<const z64*>(A_);
  ps.lda = lda;
  ps.V = reinterpret_cast<z64*>(V_);
  ps.ldv = ldv;
  PhaseTimer t_all;
  if ((st = t_all.init()) || (st = ps.init_timers())) {
    t_all.destroy();
    ps.destroy_timers();
    return st;
  }
  auto run = [&]() -> int {
    int r;
    t_all.start(s);
    if ((r = ps.setup(use_v0, reinterpret_cast<const z64*>(starts_), ld_starts, nstarts, s))) return r;
    while (ps.active()) {
      if ((r = ps.prepare(s))) return r;
      if ((r = ps.filter_eager(s))) return r;
      if ((r = ps.post_filter(s))) return r;
    }
    if ((r = ps.finish(ritzv, resid, s))) return r;
    t_all.stop(s);
    CHASE_CHK(hipStreamSynchronize(s));
    t_all.collect();
    return kOk;
  };
  st = run();
  ps.S.t_total = t_all.acc;
  t_all.destroy();
  ps.destroy_timers();
  if (st) return st;
  if (stats) *stats = ps.S;
  return ps.S.status;
}

int chase_create_real(int64_t N, const chase_params_t* p, chase_handle_t* h) {
  if (N < 2) return -1;
  if (!valid_params(p) || (int64_t)p->nev + p->nex >= N || p->precision != CHASE_FP64) return -2;
  if (!h) return -3;
  auto* hh = new chase_handle_s();
  hh->p = *p;
  hh->real = true;
  int st = hh->w.create_real(N, p->nev + p->nex);
  if (st) {
    delete hh;
    *h = nullptr;
    return st;
  }
  *h = hh;
  return kOk;
}

int chase_solve_real(chase_handle_t h, const double* A, int64_t lda, double* V, int64_t ldv, int32_t use_v0,
                     const double* starts, int64_t ld_starts, int32_t nstarts, double* ritzv, double* resid,
                     chase_stats_t* stats, chase_stream_t stream_) {
  if (!h || !h->real) return -1;
  Workspace& w = h->w;
  const int64_t n_real = w.rows, np = w.N;  // order, row pairs
  int st = check_solve_args(n_real, A, lda, V, ldv, starts, ld_starts, nstarts, ritzv, resid);
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
  const int ne = h->p.nev + h->p.nex;
  // H in the row-pair layout: the caller's storage when the order and the
  // leading dimension are even (and H 16-byte aligned), else a zero-padded copy
  const z64* Apair = reinterpret_cast<const z64*>(A);
  int64_t ldpair = lda / 2;
  if (n_real % 2 != 0 || lda % 2 != 0) {
    if ((st = w.ensure_hpad())) return st;
    if ((st = dcopy_pad(A, lda, n_real, n_real, w.Hpad, 2 * np, 2 * np, 2 * np, s))) return st;
    Apair = reinterpret_cast<const z64*>(w.Hpad);
    ldpair = np;
  }
  w.Hr = A;
  w.ldhr = lda;
  // the block and the Lanczos starts in the row-pair layout
  double* Cr = reinterpret_cast<double*>(w.Cint);
  if (use_v0 && (st = dcopy_pad(V, ldv, n_real, ne, Cr, 2 * np, 2 * np, ne, s))) return st;
  const z64* starts_pair = nullptr;
  int64_t lds_pair = 0;
  if (starts) {
    if ((st = dcopy_pad(starts, ld_starts, n_real, nstarts, reinterpret_cast<double*>(w.lzW), 2 * np, 2 * np,
                        nstarts, s)))
      return st;
    starts_pair = w.lzW;
    lds_pair = np;
  }
  ProblemState ps;
  ps.w = &w;
  ps.P = h->p;
  ps.trace_level = h->trace_level;
  ps.trace = &h->trace;
  ps.trace_cols = &h->trace_cols;
  ps.trace_col_off = &h->trace_col_off;
  h->trace.clear();
  h->trace_cols.clear();
  h->trace_col_off.clear();
  ps.A = Apair;
  ps.lda = ldpair;
  ps.V = w.Cint;
  ps.ldv = np;
  PhaseTimer t_all;
  if ((st = t_all.init()) || (st = ps.init_timers())) {
    t_all.destroy();
    ps.destroy_timers();
    return st;
  }
  auto run = [&]() -> int {
    int r;
    t_all.start(s);
    if ((r = ps.setup(use_v0, starts_pair, lds_pair, nstarts, s))) return r;
    while (ps.active()) {
      if ((r = ps.prepare(s))) return r;
      if ((r = ps.filter_eager(s))) return r;
      if ((r = ps.post_filter(s))) return r;
    }
    if ((r = ps.finish(ritzv, resid, s))) return r;
    if ((r = dcopy_pad(Cr, 2 * np, n_real, ne, V, ldv, n_real, ne, s))) return r;
    t_all.stop(s);
    CHASE_CHK(hipStreamSynchronize(s));
    t_all.collect();
    return kOk;
  };
  st = run();
  ps.S.t_total = t_all.acc;
  t_all.destroy();
  ps.destroy_timers();
  w.Hr = nullptr;
  if (st) return st;
  if (stats) *stats = ps.S;
  return ps.S.status;
}

int chase_create_c64(int64_t N, const chase_params_t* p, chase_handle_t* h) {
  if (N < 2) return -1;
  if (!valid_params(p) || (int64_t)p->nev + p->nex >= N || p->precision == CHASE_BF16X3_MIXED) return -2;
  if (!h) return -3;
  auto* hh = new chase_handle_s();
  hh->p = *p;
  hh->c64 = true;
  int st = hh->w.create_c64(N, p->nev + p->nex);
  if (st) {
    delete hh;
    *h = nullptr;
    return st;
  }
  *h = hh;
  return kOk;
}

int chase_solve_c64(chase_handle_t h, const void* A, int64_t lda, void* V, int64_t ldv, int32_t use_v0,
                    const void* starts, int64_t ld_starts, int32_t nstarts, double* ritzv, double* resid,
                    chase_stats_t* stats, chase_stream_t stream_) {
  if (!h || !h->c64) return -1;
  Workspace& w = h->w;
  const int64_t N = w.N;
  int st = check_solve_args(N, A, lda, V, ldv, starts, ld_starts, nstarts, ritzv, resid);
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
  const int ne = h->p.nev + h->p.nex;
  w.H32 = reinterpret_cast<const c32*>(A);
  w.ldh32 = lda;
  if (use_v0 && (st = convert_c_to_z(reinterpret_cast<const c32*>(V), ldv, w.Cint, N, N, ne, s))) return st;
  const z64* starts64 = nullptr;
  if (starts) {
    if ((st = convert_c_to_z(reinterpret_cast<const c32*>(starts), ld_starts, w.lzW, N, N, nstarts, s))) return st;
    starts64 = w.lzW;
  }
  ProblemState ps;
  ps.w = &w;
  ps.P = h->p;
  ps.trace_level = h->trace_level;
  ps.trace = &h->trace;
  ps.trace_cols = &h->trace_cols;
  ps.trace_col_off = &h->trace_col_off;
  h->trace.clear();
  h->trace_cols.clear();
  h->trace_col_off.clear();
  ps.A = nullptr;  // every product with H goes through the FP32 kernels
  ps.lda = 0;
  ps.V = w.Cint;
  ps.ldv = N;
  PhaseTimer t_all;
  if ((st = t_all.init()) || (st = ps.init_timers())) {
    t_all.destroy();
    ps.destroy_timers();
    return st;
  }
  auto run = [&]() -> int {
    int r;
    t_all.start(s);
    if ((r = ps.setup(use_v0, starts64, N, nstarts, s))) return r;
    while (ps.active()) {
      if ((r = ps.prepare(s))) return r;
      if ((r = ps.filter_eager(s))) return r;
      if ((r = ps.post_filter(s))) return r;
    }
    if ((r = ps.finish(ritzv, resid, s))) return r;
    if ((r = convert_z_to_c(w.Cint, N, reinterpret_cast<c32*>(V), ldv, N, ne, s))) return r;
    t_all.stop(s);
    CHASE_CHK(hipStreamSynchronize(s));
    t_all.collect();
    return kOk;
  };
  st = run();
  ps.S.t_total = t_all.acc;
  t_all.destroy();
  ps.destroy_timers();
  w.H32 = nullptr;
  if (st) return st;
  if (stats) *stats = ps.S;
  return ps.S.status;
}

int chase_filter_real(const double* A, int64_t lda, double* V, int64_t ldv, double* W, int64_t ldw, int64_t N,
                      int64_t n, const int32_t* degs, double c, double e, double mu_1, int64_t* matvecs,
                      chase_stream_t stream) {
  if (!A || !aligned16(A)) return -1;
  if (lda < N || lda % 2) return -2;
  if (!V || !aligned16(V)) return -3;
  if (ldv < N || ldv % 2) return -4;
  if (!W || !aligned16(W)) return -5;
  if (ldw < N || ldw % 2) return -6;
  if (N < 2 || N % 2) return -7;
  if (n < 0) return -8;
  if (n > 0 && !degs) return -9;
  for (int64_t j = 0; j < n; ++j)
    if (degs[j] < 2 || degs[j] % 2 || (j > 0 && degs[j] < degs[j - 1])) return -9;
  if (!(e > 0)) return -11;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void* tws = nullptr;
  int* tcnt = nullptr;
  if (hipMalloc(&tws, (size_t)tail_workspace_bytes()) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&tcnt), sizeof(int) * kTailCounterInts) != hipSuccess) {
    (void)hipGetLastError();
    if (tws) (void)hipFree(tws);
    return kAllocFailed;
  }
  int64_t mv = 0, nl = 0;
  int st = tail_counters_init(tcnt, s);
  if (!st)
    st = run_filter(reinterpret_cast<const z64*>(A), lda / 2, reinterpret_cast<z64*>(V), ldv / 2,
                    reinterpret_cast<z64*>(W), ldw / 2, N / 2, n, degs, c, e, mu_1, &mv, &nl, s, tws, tcnt, true);
  hipError_t err = hipStreamSynchronize(s);
  (void)hipFree(tws);
  (void)hipFree(tcnt);
  if (st) return st;
  if (err != hipSuccess) {
    set_last_error("chase_filter_real", err);
    return kHipError;
  }
  if (matvecs) *matvecs = mv;
  return kOk;
}

int chase_set_trace(chase_handle_t h, int32_t level) {
  if (!h) return -1;
  if (level < 0 || level > 2) return -2;
  h->trace_level = level;
  return kOk;
}

int chase_get_trace(chase_handle_t h, chase_trace_t* out, int32_t cap, int32_t* count) {
  if (!h) return -1;
  if (cap < 0 || (cap > 0 && !out)) return -3;
  const int32_t n = std::min<int32_t>(cap, (int32_t)h->trace.size());
  for (int32_t i = 0; i < n; ++i) out[i] = h->trace[(size_t)i];
  if (count) *count = n;
  return kOk;
}

int chase_get_trace_columns(chase_handle_t h, int32_t iteration, chase_trace_column_t* out, int32_t cap,
                            int32_t* count) {
  if (!h) return -1;
  if (iteration < 1 || iteration > (int32_t)h->trace_col_off.size()) return -2;
  if (cap < 0 || (cap > 0 && !out)) return -4;
  const size_t i = (size_t)iteration - 1;
  const int64_t b = h->trace_col_off[i];
  const int64_t e = i + 1 < h->trace_col_off.size() ? h->trace_col_off[i + 1] : (int64_t)h->trace_cols.size();
  const int32_t n = (int32_t)std::min<int64_t>(cap, e - b);
  for (int32_t j = 0; j < n; ++j) out[j] = h->trace_cols[(size_t)(b + j)];
  if (count) *count = n;
  return kOk;
}

int chase_solve_batched(int32_t count, const int64_t* Ns, const void* const* As, const int64_t* ldas,
                        void* const* Vs, const int64_t* ldvs, const int32_t* use_v0, const void* const* starts,
                        const int64_t* ld_starts, const int32_t* nstarts, const chase_params_t* params,
                        double* const* ritzv, double* const* resid, chase_stats_t* stats, chase_stream_t stream_) {
  if (count < 1) return -1;
  if (!Ns) return -2;
  if (!As) return -3;
  if (!ldas) return -4;
  if (!Vs) return -5;
  if (!ldvs) return -6;
  if (!params) return -11;
  if (!ritzv) return -12;
  if (!resid) return -13;
  for (int i = 0; i < count; ++i) {
    if (Ns[i] < 2) return -2;
    if (!valid_params(&params[i]) || (int64_t)params[i].nev + params[i].nex >= Ns[i]) return -11;
    if (params[i].precision != CHASE_FP64) return -11;  // grouped filter is FP64
    const void* st_i = starts ? starts[i] : nullptr;
    const int64_t lds_i = (st_i && ld_starts) ? ld_starts[i] : 0;
    const int32_t ns_i = (st_i && nstarts) ? nstarts[i] : 0;
    int a = check_solve_args(Ns[i], As[i], ldas[i], Vs[i], ldvs[i], st_i, lds_i, ns_i, ritzv[i], resid[i]);
    if (a) {
      const int map[] = {0, 0, -3, -4, -5, -6, 0, -8, -9, -10, -12, -13};
      return map[-a] ? map[-a] : a;
    }
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
  std::vector<Workspace> ws(count);
  std::vector<ProblemState> ps(count);
  GroupEntry* h_table = nullptr;
  GroupEntry* d_table = nullptr;
  int* d_queue = nullptr;  // work queue of the grouped filter launches
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  PhaseTimer t_all, t_f;
  const int nw = std::min(count, 8);   // worker threads / streams for the per-problem steps
  std::vector<hipStream_t> wstreams(nw, nullptr);
  hipEvent_t filtered = nullptr;
  int dev = 0;
  int max_deg = 2;
  for (int i = 0; i < count; ++i) max_deg = std::max(max_deg, (int)std::max(params[i].max_deg, params[i].deg));

  auto run = [&]() -> int {
    int st;
    if ((st = t_all.init()) || (st = t_f.init())) return st;
    for (int i = 0; i < count; ++i) {
      if ((st = ws[i].create(Ns[i], params[i].nev + params[i].nex, false, true))) return st;
      ps[i].w = &ws[i];
      ps[i].P = params[i];
      ps[i].A = reinterpret_cast<const z64*>(As[i]);
      ps[i].lda = ldas[i];
      ps[i].V = reinterpret_cast<z64*>(Vs[i]);
      ps[i].ldv = ldvs[i];
      if ((st = ps[i].init_timers())) return st;
    }
    // Descriptor table: max_deg steps x count problems, pinned on the host.
    const size_t tbytes = sizeof(GroupEntry) * (size_t)max_deg * count;
    CHASE_CHK(hipHostMalloc(reinterpret_cast<void**>(&h_table), tbytes, hipHostMallocDefault));
    CHASE_CHK(hipMalloc(reinterpret_cast<void**>(&d_table), tbytes));
    CHASE_CHK(hipMalloc(reinterpret_cast<void**>(&d_queue), sizeof(int) * kQueueInts));
    if ((st = queue_counters_init(d_queue, s))) return st;
    CHASE_CHK(hipGetDevice(&dev));
    for (int wk = 0; wk < nw; ++wk) CHASE_CHK(hipStreamCreate(&wstreams[wk]));
    CHASE_CHK(hipEventCreateWithFlags(&filtered, hipEventDisableTiming));

    t_all.start(s);
    for (int i = 0; i < count; ++i) {
      const void* st_i = starts ? starts[i] : nullptr;
      if ((st = ps[i].setup(use_v0 ? use_v0[i] : 1, reinterpret_cast<const z64*>(st_i),
                            st_i && ld_starts ? ld_starts[i] : 0, st_i && nstarts ? nstarts[i] : 0, s)))
        return st;
    }
    // Fill the table with this iteration's filter GEMMs (plans) for tile
    // configuration cfg, with the running tile count of every step.
    // Problems enter each step's row longest first (largest order: its tiles
    // have the longest K loop), for the grouped kernel's rotation over XCDs.
    std::vector<std::vector<GemmArgs>> plans(count);
    std::vector<int> slot_of(count);
    {
      std::vector<int> by_len(count);
      std::iota(by_len.begin(), by_len.end(), 0);
      std::stable_sort(by_len.begin(), by_len.end(), [&](int x, int y) { return Ns[x] > Ns[y]; });
      for (int j = 0; j < count; ++j) slot_of[by_len[j]] = j;
    }
    auto build_table = [&](int cfg) -> int {
      std::memset(h_table, 0, tbytes);
      for (int i = 0; i < count; ++i) {
        if (plans[i].size() > (size_t)max_deg) return -11;
        for (size_t k = 0; k < plans[i].size(); ++k) {
          GroupEntry& e = h_table[k * count + slot_of[i]];
          e.g = plans[i][k];
          zfilter_tiles(e.g.M, e.g.N, &e.tiles_n, cfg);
        }
      }
      for (int k = 0; k < max_deg; ++k) {
        int64_t acc = 0;
        for (int i = 0; i < count; ++i) {
          GroupEntry& e = h_table[(size_t)k * count + i];
          acc += zfilter_tiles(e.g.M, e.g.N, nullptr, cfg);
          e.tile_end = acc;
        }
      }
      return kOk;
    };
    auto make_plans = [&]() -> int {
      for (int i = 0; i < count; ++i) {
        plans[i].clear();
        if (!ps[i].active()) continue;
        int r = ps[i].prepare(s);
        if (r) return r;
        plans[i] = ps[i].plan();
      }
      return kOk;
    };
    if ((st = make_plans())) return st;

    // Tile shape: with autotuning, time degree step 0 of the real batch in
    // both configurations (step 0 only writes the ping-pong buffers, so the
    // trial launches change nothing) and keep the faster one.
    int cfg = 0;
    bool tune = false;
    for (int i = 0; i < count; ++i) tune = tune || params[i].autotune;
    if (tune) {
      float best_ms = 1e30f;
      for (int c = 0; c < 2; ++c) {
        if ((st = build_table(c))) return st;
        CHASE_CHK(hipMemcpyAsync(d_table, h_table, tbytes, hipMemcpyHostToDevice, s));
        float ms = 1e30f;
        if ((st = time_launches([&]() { return zfilter_grouped_launch(d_table, count, 0, grouped_grid(c), s, c, d_queue); },
                                s, &ms)))
          return st;
        if (ms < best_ms) {
          best_ms = ms;
          cfg = c;
        }
      }
    }
    // One captured graph holds every degree step of the grouped filter; its
    // kernels read all parameters from d_table, so it is replayed unchanged.
    const int grid = grouped_grid(cfg);
    CHASE_CHK(hipStreamCreate(&cs));
    CHASE_CHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < max_deg; ++k) {
      if ((st = zfilter_grouped_launch(d_table, count, k, grid, cs, cfg, d_queue))) {
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(cs, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        return st;
      }
    }
    CHASE_CHK(hipStreamEndCapture(cs, &graph));
    CHASE_CHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));

    bool first = true;
    while (true) {
      bool any = false;
      for (int i = 0; i < count; ++i) any = any || ps[i].active();
      if (!any) break;
      if (!first && (st = make_plans())) return st;
      first = false;
      if ((st = build_table(cfg))) return st;
      for (int i = 0; i < count; ++i) {
        int64_t mv = 0;
        for (const GemmArgs& g : plans[i]) mv += g.N;
        ps[i].S.filter_matvecs += mv;
        ps[i].S.filter_launches += (int64_t)plans[i].size();
        ps[i].total_mv += mv;
      }
      CHASE_CHK(hipMemcpyAsync(d_table, h_table, tbytes, hipMemcpyHostToDevice, s));
      t_f.start(s);
      CHASE_CHK(hipGraphLaunch(exec, s));
      t_f.stop(s);
      CHASE_CHK(hipEventRecord(filtered, s));
      // The rest of the iteration is per problem and latency-bound (small
      // kernels, the eigensolve, host decisions): overlap problems on worker
      // threads, each with its own stream after the grouped filter.  Workers
      // take the active problems from a shared queue, largest first, so that
      // uneven orders spread evenly over the workers.
      std::vector<int> order;
      for (int i = 0; i < count; ++i)
        if (ps[i].active()) order.push_back(i);
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ps[x].N * ps[x].na() > ps[y].N * ps[y].na(); });
      std::atomic<size_t> next{0};
      std::vector<int> wst(nw, kOk);
      std::vector<std::thread> pool;
      for (int wk = 0; wk < nw; ++wk)
        pool.emplace_back([&, wk]() {
          if (hipSetDevice(dev) != hipSuccess || hipStreamWaitEvent(wstreams[wk], filtered, 0) != hipSuccess) {
            wst[wk] = kHipError;
            return;
          }
          for (size_t q; (q = next.fetch_add(1)) < order.size();)
            if ((wst[wk] = ps[order[q]].post_filter(wstreams[wk]))) return;
        });
      for (auto& th : pool) th.join();
      for (int wk = 0; wk < nw; ++wk)
        if (wst[wk]) return wst[wk];
      for (int wk = 0; wk < nw; ++wk) CHASE_CHK(hipStreamSynchronize(wstreams[wk]));
      t_f.collect();
    }
    for (int i = 0; i < count; ++i)
      if ((st = ps[i].finish(ritzv[i], resid[i], s))) return st;
    t_all.stop(s);
    CHASE_CHK(hipStreamSynchronize(s));
    t_all.collect();
    return kOk;
  };
  int st = run();
  (void)hipStreamSynchronize(s);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (cs) (void)hipStreamDestroy(cs);
  for (hipStream_t w : wstreams)
    if (w) (void)hipStreamDestroy(w);
  if (filtered) (void)hipEventDestroy(filtered);
  if (d_table) (void)hipFree(d_table);
  if (d_queue) (void)hipFree(d_queue);
  if (h_table) (void)hipHostFree(h_table);
  int worst = kOk;
  for (int i = 0; i < count; ++i) {
    if (!st && stats) {
      stats[i] = ps[i].S;
      stats[i].t_total = t_all.acc;
      stats[i].t_filter = t_f.acc;  // the grouped filter is shared by all problems
    }
    if (!st && ps[i].S.status > worst) worst = ps[i].S.status;
    ps[i].destroy_timers();
    ws[i].release();
  }
  t_all.destroy();
  t_f.destroy();
  return st ? st : worst;
}

int chase_eigval_grad(int64_t N, int32_t nev, const void* X, int64_t ldx, const double* g, void* G, int64_t ldg,
                      int32_t fill, chase_stream_t stream) {
  if (N < 1) return -1;
  if (nev < 1 || nev > N) return -2;
  if (!X || !aligned16(X)) return -3;
  if (ldx < N) return -4;
  if (!g) return -5;
  if (!G || !aligned16(G)) return -6;
  if (ldg < N) return -7;
  if (fill != 0 && fill != 1) return -8;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  GemmArgs a;  // G = X (diag(g) X^H): the scale is applied to the B operand's K index
  a.M = N; a.N = N; a.K = nev;
  a.A = reinterpret_cast<const z64*>(X); a.lda = ldx;
  a.B = reinterpret_cast<const z64*>(X); a.ldb = ldx;
  a.bscale = g;
  a.Y = reinterpret_cast<z64*>(G); a.ldy = ldg;
  a.lower_only = fill == 1 ? 1 : 0;
  return zgrad_launch(a, s);
}

// ---- step entry points -------------------------------------------------------

int chase_filter(const void* A, int64_t lda, void* V, int64_t ldv, void* W, int64_t ldw, int64_t N, int64_t n,
                 const int32_t* degs, double c, double e, double mu_1, int64_t* matvecs, chase_stream_t stream) {
  if (int bad = filter_check_args(A, lda, V, ldv, W, ldw, N, n, degs, e)) return bad;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void* tws = nullptr;
  int* tcnt = nullptr;
  if (hipMalloc(&tws, (size_t)tail_workspace_bytes()) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&tcnt), sizeof(int) * kTailCounterInts) != hipSuccess) {
    (void)hipGetLastError();
    if (tws) (void)hipFree(tws);
    return kAllocFailed;
  }
  int64_t mv = 0, nl = 0;
  int st = tail_counters_init(tcnt, s);
  if (!st)
    st = run_filter(reinterpret_cast<const z64*>(A), lda, reinterpret_cast<z64*>(V), ldv,
                    reinterpret_cast<z64*>(W), ldw, N, n, degs, c, e, mu_1, &mv, &nl, s, tws, tcnt);
  hipError_t err = hipStreamSynchronize(s);
  (void)hipFree(tws);
  (void)hipFree(tcnt);
  if (st) return st;
  if (err != hipSuccess) {
    set_last_error("chase_filter", err);
    return kHipError;
  }
  if (matvecs) *matvecs = mv;
  return kOk;
}

int chase_caqr(void* V, int64_t ldv, int64_t N, int64_t n, double cond, int32_t force, int32_t* variant,
               chase_stream_t stream) {
  if (!V || !aligned16(V)) return -1;
  if (ldv < N) return -2;
  if (N < 1) return -3;
  if (n < 1 || n > N) return -4;
  if (force < -1 || force > 3) return -6;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace w;
  int st = w.create(N, (int)n, false, false);
  if (st) return st;
  int v = 0;
  st = caqr(w, reinterpret_cast<z64*>(V), ldv, n, cond, force, &v, s);
  if (!st) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_last_error("chase_caqr", e);
      st = kHipError;
    }
  }
  w.release();
  if (!st && variant) *variant = v;
  return st;
}

int chase_caqr_real(double* V, int64_t ldv, int64_t N, int64_t n, double cond, int32_t force, int32_t* variant,
                    chase_stream_t stream) {
  if (!V || !aligned16(V)) return -1;
  if (ldv < N) return -2;
  if (N < 2) return -3;
  if (n < 1 || n > N) return -4;
  if (force < -1 || force > 3) return -6;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace w;
  int st = w.create_real(N, (int)n);
  if (st) return st;
  // the block in the row-pair layout of the real solve (an odd order gets a
  // zero row), through the same 1D-CAQR, and back
  const int64_t np = w.N;
  double* Cr = reinterpret_cast<double*>(w.Cint);
  int v = 0;
  st = dcopy_pad(V, ldv, N, n, Cr, 2 * np, 2 * np, n, s);
  if (!st) st = caqr(w, w.Cint, np, n, cond, force, &v, s);
  if (!st) st = dcopy_pad(Cr, 2 * np, N, n, V, ldv, N, n, s);
  if (!st) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_last_error("chase_caqr_real", e);
      st = kHipError;
    }
  }
  w.release();
  if (!st && variant) *variant = v;
  return st;
}

int chase_filter_lowp(const void* A, int64_t lda, void* V, int64_t ldv, int64_t N, int64_t n, const int32_t* degs,
                      double c, double e, double mu_1, int32_t precision, int64_t* matvecs, chase_stream_t stream) {
  if (!A || !aligned16(A)) return -1;
  if (lda < N) return -2;
  if (!V || !aligned16(V)) return -3;
  if (ldv < N) return -4;
  if (N < 2) return -5;
  if (n < 0 || n > N) return -6;
  if (n > 0 && !degs) return -7;
  for (int64_t j = 0; j < n; ++j)
    if (degs[j] < 2 || degs[j] % 2 || (j > 0 && degs[j] < degs[j - 1])) return -7;
  if (!(e > 0)) return -9;
  if (precision != CHASE_FP32_MIXED && precision != CHASE_BF16X3_MIXED) return -11;
  if (n == 0) {  // no columns: nothing to filter, nothing allocated
    if (matvecs) *matvecs = 0;
    return kOk;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool bf16 = precision == CHASE_BF16X3_MIXED;
  Workspace w;
  int st = w.create(N, (int)n, true, false, bf16);
  if (st) return st;
  const z64* H = reinterpret_cast<const z64*>(A);
  z64* X = reinterpret_cast<z64*>(V);
  // the range guard's lower estimate of the spectrum, as in the solve: mu_1
  // less 1 % of its distance to the upper bound c + e
  const double lam_lo = mu_1 - 0.01 * std::fabs(c + e - mu_1);
  int64_t mv = 0, nl = 0;
  if (bf16) {
    st = bsplit_planes(H, lda, N, w.P16, s);
    if (!st) st = filter_rung_bf16(w, X, ldv, n, degs, c, e, mu_1, lam_lo, &mv, &nl, s);
  } else {
    st = convert_z_to_c(H, lda, w.A32, N, N, N, s);
    if (!st) st = filter_rung_fp32(w, w.A32, N, X, ldv, n, degs, c, e, mu_1, lam_lo, &mv, &nl, s);
  }
  if (!st) {
    hipError_t err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
      set_last_error("chase_filter_lowp", err);
      st = kHipError;
    }
  }
  w.release();
  if (!st && matvecs) *matvecs = mv;
  return st;
}

int chase_rayleigh_ritz(const void* A, int64_t lda, void* Q, int64_t ldq, int64_t N, int64_t n, double* theta,
                        double* resid, chase_stream_t stream) {
  if (!A || !aligned16(A)) return -1;
  if (lda < N) return -2;
  if (!Q || !aligned16(Q)) return -3;
  if (ldq < N) return -4;
  if (N < 1) return -5;
  if (n < 1 || n > N) return -6;
  if (!theta) return -7;
  if (!resid) return -8;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace w;
  int st = w.create(N, (int)n, false, false);
  if (st) return st;
  // Q doubles as C2_a: copy it to the workspace's C2 and write Ritz vectors to Q.
  st = copy_columns(reinterpret_cast<const z64*>(Q), ldq, w.C2, N, N, n, s);
  if (!st)
    st = rayleigh_ritz(w, reinterpret_cast<const z64*>(A), lda, w.C2, N, reinterpret_cast<z64*>(Q), ldq, n, s);
  if (!st) {
    if (hipMemcpyAsync(theta, w.theta, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(resid, w.resd, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_msg("chase_rayleigh_ritz: copy-out failed");
      st = kHipError;
    }
  }
  w.release();
  return st;
}

int chase_heev(void* G, int64_t ldg, int64_t n, double* theta, int32_t* sweeps, chase_stream_t stream) {
  if (!G || !aligned16(G)) return -1;
  if (ldg < n) return -2;
  if (n < 1 || n > 65536) return -3;
  if (!theta) return -4;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void* ws = nullptr;
  double* th = nullptr;
  if (hipMalloc(&ws, (size_t)heevj_workspace_bytes(n)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&th), sizeof(double) * (size_t)n) != hipSuccess) {
    (void)hipGetLastError();
    if (ws) (void)hipFree(ws);
    set_msg("chase_heev: hipMalloc failed");
    return kAllocFailed;
  }
  int sw = 0;
  int st = heevj(reinterpret_cast<z64*>(G), ldg, n, th, ws, &sw, s);
  if (!st && (hipMemcpyAsync(theta, th, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess)) {
    set_msg("chase_heev: copy-out failed");
    st = kHipError;
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(ws);
  (void)hipFree(th);
  if (sweeps) *sweeps = sw;
  return st;
}

int chase_lanczos(const void* A, int64_t lda, int64_t N, const void* starts, int64_t ld_starts, int32_t nstarts,
                  int32_t ksteps, int32_t ne, double* out, chase_stream_t stream) {
  if (!A || !aligned16(A)) return -1;
  if (lda < N) return -2;
  if (N < 2) return -3;
  if (!starts || !aligned16(starts)) return -4;
  if (ld_starts < N) return -5;
  if (nstarts < 1 || nstarts > 8) return -6;
  if (ksteps < 1 || ksteps > 256) return -7;
  if (ne < 1 || ne >= N) return -8;
  if (!out) return -9;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace w;
  int st = w.create(N, ne, false, true);
  if (st) return st;
  st = lanczos(w, reinterpret_cast<const z64*>(A), lda, reinterpret_cast<const z64*>(starts), ld_starts, nstarts,
               ksteps, ne, out, s);
  w.release();
  return st;
}

double chase_cond_est(const double* lam, double c, double e, const int32_t* degs, int32_t ne, int32_t locked) {
  if (!lam || !degs || ne < 1 || locked < 0 || locked >= ne || !(e > 0)) return std::nan("");
  return cond_est(lam, c, e, degs, ne, locked);
}

int chase_degree_opt(const double* resd, const double* lam, int32_t n, double c, double e, double tol_abs,
                     int32_t max_deg, int32_t extra, int32_t* degs) {
  if (n < 0) return -3;
  if (n > 0 && (!resd || !lam || !degs)) return -1;
  if (!(e > 0) || !(tol_abs > 0)) return -5;
  if (max_deg < 2 || max_deg % 2 || extra < 0) return -7;
  for (int32_t j = 0; j < n; ++j) degs[j] = degree_opt(resd[j], lam[j], c, e, tol_abs, max_deg, extra);
  return kOk;
}

const char* chase_status_string(int status) {
  switch (status) {
    case 0: return "ok";
    case 1: return "not converged within max_iter";
    case 2: return "device allocation failed";
    case 3: return "HIP runtime error";
    case 4: return "numerical breakdown";
    default: return status < 0 ? "invalid argument" : "unknown status";
  }
}

const char* chase_last_error(void) { return chase::last_error(); }

}  // extern "C"
