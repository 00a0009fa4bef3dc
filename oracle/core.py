"""Plain FP64 CPU ChASE: the oracle the GPU library is checked against.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg import this module; the GPU library never does,
and the two share no code.  Everything runs in complex128/float64 with numpy
and scipy, one library call per step of the method, with no blocking, fusion
or reordering beyond what the paper states.

Source: Wu & Di Napoli, "Advancing the distributed Multi-GPU ChASE library
through algorithm optimization and NCCL library" (arXiv 2309.15595).
  * Alg. 1 (ChASE algorithm) and Alg. 2 (ChASE with distributed QR) give the
    loop; Alg. 2 is followed with a 1 x 1 process grid, where every AllReduce
    is the identity and B2 is C2.
  * Eq. (1) is the Chebyshev three-term recurrence of the filter.
  * Alg. 3 (1D-CholeskyQR), Alg. 4 (1D-CAQR variant selection) and Alg. 5
    (condition-number estimate) give the QR step.

The paper leaves several details open.  The readings taken here (and by the
GPU library) are:
  R1 Eq. (1)'s alpha, beta, gamma: the scaled Chebyshev filter of Zhou et al.
     (cited by the paper for the filter): gamma = c, alpha_k = 2 sigma_{k+1}/e,
     beta_k = -sigma_k sigma_{k+1}, sigma_1 = e/(mu_1 - c), first step
     X_1 = (sigma_1/e)(A - cI) X_0.  Column j is p_{d_j}(A) x_j with
     p_m(x) = T_m((x-c)/e) / T_m((mu_1-c)/e).
  R2 Alg. 2's Filter(H, C, degs, c) also needs e and mu_1: Alg. 1's argument
     list is used.
  R3 Lanczos: k = min(25, N) steps from each of R supplied start vectors,
     no reorthogonalisation; b_sup = max over runs of (largest Ritz value +
     last beta); mu_1 = smallest Ritz value; mu_ne from the density of
     states: the smallest pooled Ritz value at which N * (cumulative
     quadrature weight)/R reaches n_e, clamped to [mu_1, b_sup).
  R4 CondEst at the first iteration, where Lambda is still zero: Lambda[1]
     and Lambda[locked+1] are taken as mu_1.
  R5 degreeOpt: d_j = ceil(ln(resd_j/tol_abs) / ln rho(t_j)) + deg_extra
     with t_j = (Lambda_j - c)/e; rho <= 1 + 1e-12 gives max_deg; clamped to
     [2, max_deg] and rounded up to even (the paper enforces even degrees and
     caps them at 36).  The margin is not given in the paper; deg_extra = 4
     is the FP64 solve's (the GPU's measured optimum at N = 20000).
  R6 tol is relative: a pair is converged when resd <= tol * ||A||_lo with
     ||A||_lo the largest |Ritz value| of the Lanczos runs.  Ritz values lie
     in [lambda_1, lambda_N], so ||A||_lo <= ||A||_2 and a converged pair has
     ||A x - lambda x|| <= tol ||A||_2.
  R7 Locking: every converged pair among the first nev - locked active pairs
     is locked; they are moved, in their current order, to the front of the
     active block.
  R8 Sort by degree: stable, ascending, applied to the active columns with
     their Ritz values, residuals and degrees.
  R9 CAQR thresholds: cond > 1e8 -> shifted CholeskyQR2; cond < 20 ->
     CholeskyQR; otherwise CholeskyQR2.
  R10 Shift of s-CholeskyQR2: u = 2^-53 and the squared Frobenius norm, as
     printed.
  R11 A failed Cholesky in CholeskyQR/CholeskyQR2 escalates to shifted
     CholeskyQR2 on the same input, and a failed shifted Cholesky to
     Householder QR.
  R12 Householder QR (ScaLAPACK in the paper) is LAPACK's reduced QR.
  R14 The Rayleigh quotient is Hermitised, (G + G^H)/2, before HEEVD.
  R17 MaxIter defaults to 25.
  R19 The residual recomputes H C as Alg. 2 does.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

U_ROUNDOFF = 2.0 ** -53          # unit round-off of IEEE binary64
COND_SHIFTED = 1e8               # Alg. 4: above this, s-CholeskyQR2
COND_CHOLQR1 = 20.0              # Alg. 4: below this, one CholeskyQR pass

QR_CHOLQR1, QR_CHOLQR2, QR_SHIFTED, QR_HOUSEHOLDER = 0, 1, 2, 3
QR_NAMES = ("cholqr1", "cholqr2", "shifted_cholqr2", "householder")


@dataclasses.dataclass
class Params:
    """Alg. 2's inputs (nev, nex, deg, tol, MaxIter, opt) plus the readings."""
    nev: int
    nex: int
    deg: int = 20               # initial degree (experiments use 20)
    max_deg: int = 36           # maximal degree allowed (experiments use 36)
    deg_extra: int = 4          # R5 margin (FP64)
    max_iter: int = 25          # R17
    opt: bool = True            # degree optimisation on
    tol: float = 1e-10          # residual threshold (all experiments)
    lanczos_steps: int = 25     # R3
    force_qr: Optional[int] = None   # testing: bypass CondEst's choice

    @property
    def ne(self) -> int:
        return self.nev + self.nex


# --------------------------------------------------------------------------
# Chebyshev filter: Eq. (1) with the scaled coefficients of R1
# --------------------------------------------------------------------------

def filter_coefficients(c: float, e: float, mu1: float, m: int):
    """Per-step (alpha, gamma, beta) of Eq. (1) for steps 1..m (R1).

    Step 1 maps X_0 to X_1, step k+1 maps (X_k, X_{k-1}) to X_{k+1}:
        X_{k+1} = alpha_k (A - gamma I) X_k + beta_k X_{k-1}.
    """
    sigma1 = e / (mu1 - c)
    coeffs = [(sigma1 / e, c, 0.0)]
    sigma = sigma1
    for _ in range(1, m):
        sigma_next = 1.0 / (2.0 / sigma1 - sigma)
        coeffs.append((2.0 * sigma_next / e, c, -sigma * sigma_next))
        sigma = sigma_next
    return coeffs


def chebyshev_filter(A: np.ndarray, V: np.ndarray, degs, c: float, e: float,
                     mu1: float):
    """Apply p_{d_j}(A) to column j of V via the recurrence of Eq. (1).

    Returns (filtered block, MatVecs) with MatVecs = sum_j d_j: column j
    takes part in steps 1..d_j only.
    """
    degs = np.asarray(degs, dtype=np.int64)
    n = V.shape[1]
    if n == 0:
        return V.copy(), 0
    if degs.shape != (n,) or np.any(degs < 1):
        raise ValueError("one degree >= 1 per column")
    m = int(degs.max())
    coeffs = filter_coefficients(c, e, mu1, m)
    out = np.array(V, dtype=np.complex128, copy=True)
    x_prev = np.zeros_like(out)
    x_cur = out.copy()
    for k, (alpha, gamma, beta) in enumerate(coeffs, start=1):
        x_next = alpha * (A @ x_cur - gamma * x_cur) + beta * x_prev
        x_prev, x_cur = x_cur, x_next
        done = degs == k
        out[:, done] = x_cur[:, done]
    return out, int(degs.sum())


def chebyshev_scalar(x, m: int, c: float, e: float, mu1: float):
    """p_m(x) = T_m((x-c)/e) / T_m((mu1-c)/e) by the same recurrence."""
    x = np.asarray(x, dtype=np.float64)
    coeffs = filter_coefficients(c, e, mu1, m)
    y_prev = np.zeros_like(x)
    y_cur = np.ones_like(x)
    for alpha, gamma, beta in coeffs:
        y_prev, y_cur = y_cur, alpha * (x - gamma) * y_cur + beta * y_prev
    return y_cur


# --------------------------------------------------------------------------
# Lanczos spectral bounds (Alg. 1 / Alg. 2 first line; reading R3)
# --------------------------------------------------------------------------

def lanczos_run(A: np.ndarray, start: np.ndarray, k: int):
    """k plain Lanczos steps from ``start``; returns (alpha, beta) arrays.

    beta has the same length as alpha; beta[-1] is the norm of the last
    residual, used by the upper-bound estimate.  Stops early on breakdown.
    """
    v = start / np.linalg.norm(start)
    v_old = np.zeros_like(v)
    beta_old = 0.0
    alphas, betas = [], []
    for _ in range(k):
        w = A @ v - beta_old * v_old
        alpha = float(np.real(np.vdot(v, w)))
        w = w - alpha * v
        beta = float(np.linalg.norm(w))
        alphas.append(alpha)
        betas.append(beta)
        if beta == 0.0:
            break
        v_old, v = v, w / beta
        beta_old = beta
    return np.array(alphas), np.array(betas)


def tridiagonal_eig(alpha: np.ndarray, beta: np.ndarray):
    """Eigenpairs of the symmetric tridiagonal T(alpha, beta[:-1])."""
    k = alpha.shape[0]
    T = np.diag(alpha)
    if k > 1:
        T += np.diag(beta[: k - 1], 1) + np.diag(beta[: k - 1], -1)
    theta, Z = np.linalg.eigh(T)
    return theta, Z


def lanczos_bounds(A: np.ndarray, starts: np.ndarray, ne: int, k: int = 25):
    """(b_sup, mu_1, mu_ne, norm_lo) from len(starts) Lanczos runs (R3, R6).

    norm_lo = max |Ritz value| is a lower bound of ||A||_2.
    """
    N = A.shape[0]
    k = min(k, N)
    R = starts.shape[1]
    b_sup = -np.inf
    mu_1 = np.inf
    theta_max = -np.inf
    nodes, weights = [], []
    for r in range(R):
        alpha, beta = lanczos_run(A, starts[:, r], k)
        theta, Z = tridiagonal_eig(alpha, beta)
        b_sup = max(b_sup, theta[-1] + beta[-1])
        mu_1 = min(mu_1, theta[0])
        theta_max = max(theta_max, theta[-1])
        nodes.append(theta)
        weights.append(np.abs(Z[0, :]) ** 2)
    nodes = np.concatenate(nodes)
    weights = np.concatenate(weights)
    order = np.argsort(nodes, kind="stable")
    count = N * np.cumsum(weights[order]) / R
    idx = int(np.searchsorted(count, ne, side="left"))
    idx = min(idx, nodes.shape[0] - 1)
    mu_ne = float(nodes[order][idx])
    mu_ne = min(max(mu_ne, mu_1), np.nextafter(b_sup, -np.inf))
    norm_lo = max(abs(mu_1), abs(theta_max))
    return float(b_sup), float(mu_1), mu_ne, float(norm_lo)


# --------------------------------------------------------------------------
# Condition-number estimate (Alg. 5) and QR variants (Alg. 3, Alg. 4)
# --------------------------------------------------------------------------

def rho(t: float) -> float:
    """max(|t - sqrt(t^2-1)|, |t + sqrt(t^2-1)|) with a complex square root."""
    s = np.sqrt(complex(t) ** 2 - 1.0)
    return float(max(abs(t - s), abs(t + s)))


def cond_est(Lam: np.ndarray, c: float, e: float, degs: np.ndarray,
             locked: int) -> float:
    """Alg. 5: |rho|^d |rho'|^(d_M - d) from Lambda[1], Lambda[locked+1]."""
    t_first = (Lam[0] - c) / e
    t_active = (Lam[locked] - c) / e
    d = int(degs[locked])
    d_max = int(np.max(degs[locked:]))
    # IEEE product: an estimate beyond the double range is +inf, which takes
    # the same branch of Alg. 4 as any other estimate above its threshold.
    with np.errstate(over="ignore"):
        est = np.float64(rho(t_active)) ** d * np.float64(rho(t_first)) ** (d_max - d)
    return float(est)


def select_qr(cond: float) -> int:
    """Alg. 4's branch for an estimated condition number (R9)."""
    if cond > COND_SHIFTED:
        return QR_SHIFTED
    if cond < COND_CHOLQR1:
        return QR_CHOLQR1
    return QR_CHOLQR2


class CholeskyFailure(Exception):
    pass


def _upper_cholesky(G: np.ndarray) -> np.ndarray:
    """R upper triangular with R^H R = G; CholeskyFailure when not SPD."""
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError as exc:
        raise CholeskyFailure(str(exc)) from exc
    if not np.all(np.isfinite(L)):
        raise CholeskyFailure("non-finite factor")
    return L.conj().T


def _right_solve_upper(X: np.ndarray, R: np.ndarray) -> np.ndarray:
    """X R^{-1} for upper triangular R (TRSM): R^T Y^T = X^T."""
    return sla.solve_triangular(R.T, X.T, lower=True).T


def gram(X: np.ndarray) -> np.ndarray:
    """X^H X, Hermitised (SYRK/HERK)."""
    G = X.conj().T @ X
    return 0.5 * (G + G.conj().T)


def cholesky_qr(X: np.ndarray, passes: int) -> np.ndarray:
    """Alg. 3 with cholDegree = passes on a 1 x 1 grid."""
    for _ in range(passes):
        R = _upper_cholesky(gram(X))
        X = _right_solve_upper(X, R)
    return X


def shifted_shift(m: int, n: int, fro2: float) -> float:
    """Alg. 4's shift s = 11 (m n + n (n + 1)) u ||X||_F^2."""
    return 11.0 * (m * n + n * (n + 1)) * U_ROUNDOFF * fro2


def shifted_cholesky_qr2(X: np.ndarray) -> np.ndarray:
    """Alg. 4's s-CholeskyQR2 branch without the Householder fallback."""
    m, n = X.shape
    G = gram(X)
    fro2 = float(np.sum(np.abs(X) ** 2))
    s = shifted_shift(m, n, fro2)
    R = _upper_cholesky(G + s * np.eye(n))
    X = _right_solve_upper(X, R)
    return cholesky_qr(X, 2)


def householder_qr(X: np.ndarray) -> np.ndarray:
    """Reduced Householder QR (LAPACK geqrf/ungqr), Q only (R12)."""
    Q, _ = np.linalg.qr(X, mode="reduced")
    return Q


def caqr(X: np.ndarray, cond: float, force: Optional[int] = None):
    """Alg. 4 with the escalation of R11.  Returns (Q, variant used)."""
    variant = select_qr(cond) if force is None else force
    while True:
        try:
            if variant == QR_CHOLQR1:
                return cholesky_qr(X, 1), variant
            if variant == QR_CHOLQR2:
                return cholesky_qr(X, 2), variant
            if variant == QR_SHIFTED:
                return shifted_cholesky_qr2(X), variant
            return householder_qr(X), QR_HOUSEHOLDER
        except CholeskyFailure:
            variant = QR_SHIFTED if variant < QR_SHIFTED else QR_HOUSEHOLDER


# --------------------------------------------------------------------------
# Rayleigh-Ritz, residual, degree optimisation, locking
# --------------------------------------------------------------------------

def rayleigh_ritz(A: np.ndarray, Q: np.ndarray):
    """Alg. 2's RR: B = H Q, G = Q^H B (Hermitised, R14), eigh, Q W."""
    B = A @ Q
    G = Q.conj().T @ B
    G = 0.5 * (G + G.conj().T)
    theta, W = np.linalg.eigh(G)
    return theta, Q @ W


def residual_norms(A: np.ndarray, X: np.ndarray, theta: np.ndarray):
    """||H x_j - theta_j x_j||_2 per column (Alg. 2 residual, R19)."""
    B = A @ X - X * theta[None, :]
    return np.sqrt(np.sum(np.abs(B) ** 2, axis=0))


def degree_opt(resd: np.ndarray, Lam: np.ndarray, c: float, e: float,
               tol_abs: float, max_deg: int, deg_extra: int) -> np.ndarray:
    """R5: degrees from the Chebyshev growth rate rho((Lambda_j - c)/e)."""
    out = np.empty(resd.shape[0], dtype=np.int64)
    for j in range(resd.shape[0]):
        r = rho((Lam[j] - c) / e)
        if r <= 1.0 + 1e-12 or not np.isfinite(resd[j]):
            d = max_deg
        else:
            ratio = resd[j] / tol_abs
            if ratio <= 1.0:
                d = deg_extra
            else:
                d = int(math.ceil(math.log(ratio) / math.log(r))) + deg_extra
        d = min(max(d, 2), max_deg)
        out[j] = d + d % 2          # max_deg is even, so this stays <= max_deg
    return out


def degree_order(degs: np.ndarray) -> np.ndarray:
    """R8 (Alg. 1's sort by degree): the stable ascending permutation of the
    active columns by degree, equal degrees keeping their current order."""
    return np.argsort(degs, kind="stable")


def lock_order(resd_active: np.ndarray, n_lockable: int, tol_abs: float):
    """R7: permutation of the active block moving converged pairs first."""
    n = resd_active.shape[0]
    conv = [j for j in range(min(n_lockable, n)) if resd_active[j] <= tol_abs]
    taken = set(conv)
    rest = [j for j in range(n) if j not in taken]
    return np.array(conv + rest, dtype=np.int64), len(conv)


# --------------------------------------------------------------------------
# The loop of Alg. 2
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    evals: np.ndarray
    evecs: np.ndarray
    resid: np.ndarray
    converged: bool
    iterations: int
    locked: int
    filter_matvecs: int
    total_matvecs: int
    bounds: tuple
    history: List[dict]


def chase(A: np.ndarray, params: Params, V0: Optional[np.ndarray] = None,
          starts: Optional[np.ndarray] = None, bounds: Optional[tuple] = None,
          rng_seed: int = 0) -> Result:
    """Lowest nev eigenpairs of Hermitian A by Alg. 2 on a 1 x 1 grid."""
    A = np.asarray(A)
    N = A.shape[0]
    nev, nex = params.nev, params.nex
    ne = nev + nex
    if nev < 1 or nex < 0 or ne >= N:
        raise ValueError("need 1 <= nev, 0 <= nex, nev + nex < N")
    if params.deg < 2 or params.deg % 2 or params.max_deg % 2:
        raise ValueError("degrees must be even and >= 2")
    if not params.tol > 0:
        raise ValueError("tol must be positive")

    if V0 is None:
        rng = np.random.default_rng(rng_seed)
        V0 = (rng.standard_normal((N, ne)) + 1j * rng.standard_normal((N, ne))) / np.sqrt(2)
    C = np.array(V0, dtype=np.complex128, copy=True)
    C2 = C.copy()

    if bounds is None:
        if starts is None:
            rng = np.random.default_rng(rng_seed + 1)
            starts = (rng.standard_normal((N, 4)) + 1j * rng.standard_normal((N, 4))) / np.sqrt(2)
        b_sup, mu_1, mu_ne, norm_lo = lanczos_bounds(A, starts, ne, params.lanczos_steps)
        lanczos_matvecs = starts.shape[1] * min(params.lanczos_steps, N)
    else:
        b_sup, mu_1, mu_ne, norm_lo = bounds
        lanczos_matvecs = 0
    tol_abs = params.tol * norm_lo

    degs = np.full(ne, params.deg, dtype=np.int64)
    Lam = np.zeros(ne)
    resd = np.full(ne, np.inf)
    locked = 0
    it = 1
    c = 0.5 * (b_sup + mu_ne)
    e = 0.5 * (b_sup - mu_ne)
    mu1_cur = mu_1
    filter_mv = 0
    total_mv = lanczos_matvecs
    history = []

    while locked < nev and it <= params.max_iter:
        if it != 1:
            mu1_cur = float(np.min(Lam))
            mu_ne = float(np.max(Lam))
            c = 0.5 * (b_sup + mu_ne)
            e = 0.5 * (b_sup - mu_ne)
            if params.opt:
                degs[locked:] = degree_opt(resd[locked:], Lam[locked:], c, e, tol_abs,
                                           params.max_deg, params.deg_extra)
            order = degree_order(degs[locked:])
            sl = slice(locked, ne)
            C[:, sl] = C[:, sl][:, order]
            Lam[sl] = Lam[sl][order]
            resd[sl] = resd[sl][order]
            degs[sl] = degs[sl][order]

        # Filter on the active columns
        C[:, locked:], mv = chebyshev_filter(A, C[:, locked:], degs[locked:], c, e, mu1_cur)
        filter_mv += mv
        total_mv += mv

        # CondEst (R4 at the first iteration) and 1D-CAQR on all columns
        Lam_est = Lam if it != 1 else np.full(ne, mu1_cur)
        cond = cond_est(Lam_est, c, e, degs, locked)
        C, variant = caqr(C, cond, params.force_qr)

        # restore the locked columns, save the new active ones
        C[:, :locked] = C2[:, :locked]
        C2[:, locked:] = C[:, locked:]

        # Rayleigh-Ritz on the active block
        theta, Ca = rayleigh_ritz(A, C2[:, locked:])
        C[:, locked:] = Ca
        C2[:, locked:] = Ca
        Lam[locked:] = theta
        total_mv += ne - locked

        # Residuals
        resd[locked:] = residual_norms(A, C[:, locked:], theta)
        total_mv += ne - locked

        # Deflation and locking
        order, n_new = lock_order(resd[locked:], nev - locked, tol_abs)
        sl = slice(locked, ne)
        C[:, sl] = C[:, sl][:, order]
        C2[:, sl] = C2[:, sl][:, order]
        Lam[sl] = Lam[sl][order]
        resd[sl] = resd[sl][order]
        degs[sl] = degs[sl][order]
        history.append(dict(iteration=it, locked_before=locked, new_locked=n_new,
                            cond=cond, qr=variant, c=c, e=e, mu1=mu1_cur,
                            degs=degs.copy(), matvecs=mv))
        locked += n_new
        it += 1

    converged = locked >= nev
    if converged:
        idx = np.argsort(Lam[:locked], kind="stable")[:nev]
    else:
        idx = np.argsort(Lam, kind="stable")[:nev]
    return Result(evals=Lam[idx].copy(), evecs=C[:, idx].copy(), resid=resd[idx].copy(),
                  converged=converged, iterations=it - 1, locked=locked,
                  filter_matvecs=filter_mv, total_matvecs=total_mv,
                  bounds=(b_sup, mu_1, mu_ne, norm_lo), history=history)


# --------------------------------------------------------------------------
# Eigenvalue gradient (Hellmann-Feynman)
# --------------------------------------------------------------------------

def eigval_grad(X: np.ndarray, g: np.ndarray) -> np.ndarray:
    """dL/dA for L = sum_i g_i lambda_i: X diag(g) X^H (d lambda = x^H dA x)."""
    return (X * np.asarray(g)[None, :]) @ X.conj().T
