/* A plain C99 caller of the library: no Python, no torch.  Builds a Hermitian
 * matrix of known spectrum on the host, H = P diag(lambda) P with the
 * Householder reflector P = I - 2 v v^H (||v|| = 1), so that
 *   H_ij = lambda_i delta_ij - 2 v_i conj(v_j) (lambda_i + lambda_j - 2 s),
 *   s = sum_k lambda_k |v_k|^2,
 * copies it to the device and solves for the nev lowest pairs of each
 * variant's kind of matrix through the C ABI (complex128; float64 with a real
 * v).  Exit status 0 when every eigenvalue is within 1e-10 ||H|| of lambda
 * and every residual within tol ||H||.
 *
 * Build: gcc -std=c99 -O2 -I include -I /opt/rocm/include -D__HIP_PLATFORM_AMD__
 *        c_abi_solve.c -L <dir of libchase_hip.so> -lchase_hip -L /opt/rocm/lib -lamdhip64 -lm
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "chase_hip.h"

static uint64_t lcg = 0x2309155952309ULL;
static double uniform(void) { /* (0, 1) */
  lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
  return ((double)(lcg >> 11) + 0.5) / 9007199254740992.0;
}

static int check(const char* what, int n, const double* ritz, const double* resid, const double* lam,
                 double norm, double tol) {
  double err = 0.0, res = 0.0;
  for (int i = 0; i < n; ++i) {
    err = fmax(err, fabs(ritz[i] - lam[i]));
    res = fmax(res, resid[i]);
  }
  printf("%s: max |ritz - lambda| / ||H|| = %.2e, max resid / ||H|| = %.2e\n", what, err / norm, res / norm);
  return err <= 1e-10 * norm && res <= 1.01 * tol * norm ? 0 : 1;
}

int main(void) {
  const int64_t N = 600;
  const int nev = 24, nex = 12, ne = nev + nex;
  double* lam = (double*)malloc(sizeof(double) * N);
  double* v = (double*)malloc(sizeof(double) * 2 * N); /* complex (re, im) */
  for (int64_t i = 0; i < N; ++i) lam[i] = -1.0 + 2.0 * (double)i / (double)(N - 1);
  double nv = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    v[2 * i] = uniform() - 0.5;
    v[2 * i + 1] = uniform() - 0.5;
    nv += v[2 * i] * v[2 * i] + v[2 * i + 1] * v[2 * i + 1];
  }
  nv = sqrt(nv);
  double s = 0.0;
  for (int64_t i = 0; i < 2 * N; ++i) v[i] /= nv;
  for (int64_t i = 0; i < N; ++i) s += lam[i] * (v[2 * i] * v[2 * i] + v[2 * i + 1] * v[2 * i + 1]);

  /* complex128, column-major: element (i, j) at 2 (i + j N) */
  double* H = (double*)malloc(sizeof(double) * 2 * N * N);
  for (int64_t j = 0; j < N; ++j)
    for (int64_t i = 0; i < N; ++i) {
      const double f = -2.0 * (lam[i] + lam[j] - 2.0 * s);
      /* v_i conj(v_j) */
      const double re = v[2 * i] * v[2 * j] + v[2 * i + 1] * v[2 * j + 1];
      const double im = v[2 * i + 1] * v[2 * j] - v[2 * i] * v[2 * j + 1];
      H[2 * (i + j * N)] = f * re + (i == j ? lam[i] : 0.0);
      H[2 * (i + j * N) + 1] = f * im;
    }

  void *dA = NULL, *dV = NULL;
  if (hipMalloc(&dA, sizeof(double) * 2 * N * N) != hipSuccess ||
      hipMalloc(&dV, sizeof(double) * 2 * N * ne) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 2;
  }
  if (hipMemcpy(dA, H, sizeof(double) * 2 * N * N, hipMemcpyHostToDevice) != hipSuccess) return 2;

  chase_params_t p;
  chase_default_params(&p);
  p.nev = nev;
  p.nex = nex;
  int64_t bytes = 0;
  if (chase_workspace_bytes(N, &p, 0, &bytes) != 0) return 3;
  printf("complex128 workspace: %lld bytes\n", (long long)bytes);
  chase_handle_t h = NULL;
  int st = chase_create(N, &p, &h);
  if (st != 0) {
    fprintf(stderr, "chase_create: %s\n", chase_status_string(st));
    return 3;
  }
  double ritz[64], resid[64];
  chase_stats_t stats;
  /* use_v0 = 0: the initial block and the Lanczos starts come from p.seed */
  st = chase_solve(h, dA, N, dV, N, 0, NULL, 0, 0, ritz, resid, &stats, NULL);
  chase_destroy(h);
  if (st != 0) {
    fprintf(stderr, "chase_solve: %s (%s)\n", chase_status_string(st), chase_last_error());
    return 4;
  }
  printf("complex128: %d iterations, %lld filter MatVecs\n", stats.iterations, (long long)stats.filter_matvecs);
  int bad = check("complex128", nev, ritz, resid, lam, 1.0, p.tol);

  /* float64 real symmetric: the same construction with a real v */
  double* Hr = (double*)malloc(sizeof(double) * N * N);
  double* vr = (double*)malloc(sizeof(double) * N);
  nv = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    vr[i] = uniform() - 0.5;
    nv += vr[i] * vr[i];
  }
  nv = sqrt(nv);
  s = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    vr[i] /= nv;
    s += lam[i] * vr[i] * vr[i];
  }
  for (int64_t j = 0; j < N; ++j)
    for (int64_t i = 0; i < N; ++i)
      Hr[i + j * N] = -2.0 * vr[i] * vr[j] * (lam[i] + lam[j] - 2.0 * s) + (i == j ? lam[i] : 0.0);
  if (hipMemcpy(dA, Hr, sizeof(double) * N * N, hipMemcpyHostToDevice) != hipSuccess) return 2;
  st = chase_create_real(N, &p, &h);
  if (st != 0) return 3;
  st = chase_solve_real(h, (const double*)dA, N, (double*)dV, N, 0, NULL, 0, 0, ritz, resid, &stats, NULL);
  chase_destroy(h);
  if (st != 0) {
    fprintf(stderr, "chase_solve_real: %s (%s)\n", chase_status_string(st), chase_last_error());
    return 4;
  }
  bad |= check("float64", nev, ritz, resid, lam, 1.0, p.tol);

  hipFree(dA);
  hipFree(dV);
  free(H);
  free(Hr);
  free(v);
  free(vr);
  free(lam);
  printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}
