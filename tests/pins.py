"""Checks that tie the CPU oracle to the paper and to the mathematics.

Each check takes the oracle module and raises AssertionError when the oracle
disagrees with a closed form, an invariant, a brute-force computation or a
value printed in (or derived by hand from) the paper.  The planted-mistake
tests re-run these checks against a deliberately broken copy of the oracle.
"""
import json
import math
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def chebyshev_closed_form(t, m):
    """T_m(t) from cos/cosh, independent of any recurrence."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(m * np.arccos(t[inside]))
    ti = t[~inside]
    out[~inside] = np.sign(ti) ** m * np.cosh(m * np.arccosh(np.abs(ti)))
    return out


# ----------------------------------------------------------------- filter

def check_filter_golden(oc):
    d = _golden("chebyshev_values.json")
    for case in d["cases"]:
        got = float(oc.chebyshev_scalar(np.array([case["x"]]), case["m"], d["c"], d["e"], d["mu1"])[0])
        assert abs(got - case["expected"]) <= 1e-14 * max(1.0, abs(case["expected"])) + 1e-15, (case, got)


def check_filter_diagonal(oc, seed=5):
    """On A = diag(lam), column j of the output is p_{d_j}(lam) * v_j."""
    rng = np.random.default_rng(seed)
    lam = np.concatenate([np.linspace(-1.3, -0.9, 7), np.linspace(-0.85, 2.0, 33)])
    N = lam.shape[0]
    A = np.diag(lam).astype(np.complex128)
    degs = np.array([1, 2, 3, 4, 7, 10, 20, 36])
    V = synth.complex_gaussian(rng, (N, degs.shape[0]))
    c, e, mu1 = 0.55, 1.45, -1.3
    out, mv = oc.chebyshev_filter(A, V, degs, c, e, mu1)
    assert mv == int(degs.sum())
    for j, m in enumerate(degs):
        p = chebyshev_closed_form((lam - c) / e, m) / chebyshev_closed_form(np.array([(mu1 - c) / e]), m)[0]
        ref = p * V[:, j]
        err = np.max(np.abs(out[:, j] - ref)) / np.max(np.abs(ref))
        assert err <= 1e-12, (m, err)


def check_filter_rotated(oc, seed=6):
    """On A = Q diag(lam) Q^H the filter equals Q diag(p(lam)) Q^H V."""
    rng = np.random.default_rng(seed)
    N = 60
    lam = np.linspace(-1.0, 3.0, N)
    Q = synth.gaussian_unitary(N, rng)
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    V = synth.complex_gaussian(rng, (N, 5))
    degs = np.array([2, 4, 6, 12, 20])
    c, e, mu1 = 1.6, 1.4, -1.0
    out, _ = oc.chebyshev_filter(A, V, degs, c, e, mu1)
    for j, m in enumerate(degs):
        p = chebyshev_closed_form((lam - c) / e, m) / chebyshev_closed_form(np.array([(mu1 - c) / e]), m)[0]
        ref = (Q * p) @ (Q.conj().T @ V[:, j])
        err = np.linalg.norm(out[:, j] - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, (m, err)


def check_filter_unit_at_mu1(oc):
    for m in (1, 2, 5, 20, 36):
        for (c, e, mu1) in ((0.3, 0.9, -1.0), (5.0, 4.0, -0.99)):
            v = float(oc.chebyshev_scalar(np.array([mu1]), m, c, e, mu1)[0])
            assert abs(v - 1.0) <= 1e-13 * m, (m, v)


# ----------------------------------------------------------------- Lanczos

def check_lanczos_bounds(oc, seed=7):
    rng = np.random.default_rng(seed)
    N = 300
    lam = np.linspace(-2.0, 1.5, N)
    A = synth.hermitian_from_spectrum(lam, "gaussian", seed=seed)
    starts = synth.complex_gaussian(rng, (N, 4))
    b_sup, mu_1, mu_ne, norm_lo = oc.lanczos_bounds(A, starts, ne=20, k=25)
    assert norm_lo <= np.max(np.abs(lam)) + 1e-12 and norm_lo >= 0.9 * np.max(np.abs(lam))
    assert b_sup >= lam[-1] - 1e-12, (b_sup, lam[-1])
    assert mu_1 >= lam[0] - 1e-12 and mu_1 <= lam[-1]
    assert mu_1 <= mu_ne < b_sup


def check_lanczos_full_spectrum(oc, seed=8):
    """With k = N steps the tridiagonal T has A's eigenvalues (small N)."""
    rng = np.random.default_rng(seed)
    N = 8
    lam = np.array([-3.0, -1.0, -0.5, 0.0, 0.7, 1.5, 2.0, 6.0])
    A = synth.hermitian_from_spectrum(lam, "gaussian", seed=seed)
    alpha, beta = oc.lanczos_run(A, synth.complex_gaussian(rng, N), N)
    theta, Z = oc.tridiagonal_eig(alpha, beta)
    assert np.max(np.abs(theta - lam)) <= 1e-10, theta
    # the quadrature weights are a probability distribution
    assert abs(np.sum(np.abs(Z[0]) ** 2) - 1.0) <= 1e-12


def dos_problem(N, seed):
    """Hermitian A = Q diag(lam) Q^H and a Lanczos start whose squared
    weights on the eigenvectors are 1.5/N, 1/N, ..., 1/N, 0.5/N (ascending
    eigenvalues): N times the cumulative weight is j + 1.5 after the j-th
    eigenvalue, so it first reaches any integer n_e at eigenvalue n_e, half a
    step clear of rounding."""
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(-2.0, 3.0, N))
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    w = np.full(N, 1.0 / N)
    w[0], w[-1] = 1.5 / N, 0.5 / N
    return lam, A, (Q @ np.sqrt(w))[:, None]


def check_dos_closed_form(oc):
    """The spectral-density estimate of mu_ne: with k = N Lanczos steps the
    Ritz values are the eigenvalues and the quadrature weights the start's
    squared components, so for the start of dos_problem mu_ne is exactly
    the n_e-th eigenvalue; mu_1 the smallest, b_sup the largest."""
    for seed in range(3):
        for N in (10, 12):
            lam, A, start = dos_problem(N, seed)
            for ne in range(1, N - 1):
                b_sup, mu_1, mu_ne, _ = oc.lanczos_bounds(A, start, ne, N)
                assert abs(mu_ne - lam[ne - 1]) <= 1e-9, (seed, N, ne, mu_ne, lam[ne - 1])
                assert abs(mu_1 - lam[0]) <= 1e-9 and abs(b_sup - lam[-1]) <= 1e-6


# ----------------------------------------------------------------- CondEst

def check_condest_golden(oc):
    d = _golden("condest_cases.json")
    for case in d["cases"]:
        ne = 5
        Lam = np.full(ne, 9.0)
        Lam[0] = case["lam_first"]
        locked = 2
        Lam[locked] = case["lam_active"]
        degs = np.full(ne, case["d"], dtype=np.int64)
        degs[locked] = case["d"]
        degs[-1] = case["d_max"]
        got = oc.cond_est(Lam, case["c"], case["e"], degs, locked)
        assert abs(got - case["expected"]) <= 1e-12 * case["expected"], (case, got)


def check_condest_overflow(oc):
    """Alg. 5 far outside the damped interval: the growth factor
    |t| + sqrt(t^2 - 1) for t = -2000 raised to d = 80 is finite (about 1e288,
    checked in logarithms); to d = 200 it passes the double range and the
    estimate is +inf, which still selects the shifted CholeskyQR of Alg. 4."""
    ne = 3
    Lam = np.array([-1.0, 0.0, 0.5])
    c, e = 1.0, 1e-3                      # t = (lambda_1 - c) / e = -2000
    g = 2000.0 + np.sqrt(2000.0 ** 2 - 1.0)
    got = oc.cond_est(Lam, c, e, np.full(ne, 80, dtype=np.int64), 0)
    assert np.isfinite(got)
    assert abs(np.log(got) - 80 * np.log(g)) <= 1e-12 * 80 * np.log(g)
    big = oc.cond_est(Lam, c, e, np.full(ne, 200, dtype=np.int64), 0)
    assert big == np.inf
    assert oc.select_qr(big) == oc.QR_SHIFTED


def _growth(t):
    """Growth rate of T_k at |t| >= 1 in closed form: |t| + sqrt(t^2 - 1)."""
    a = abs(t)
    return a + np.sqrt(a * a - 1.0)


def check_degree_opt(oc):
    """Per-vector degrees of Alg. 2: even, within [2, max_deg]; outside the
    damped interval d - extra is the smallest exponent (up to the even
    round-up) with resd * g^-(d - extra) <= tol, g the growth rate at
    t = (lambda - c) / e; inside it, or for a non-finite residual, the cap;
    an already converged residual takes the margin alone."""
    c, e, tol, max_deg, extra = 0.5, 0.5, 1e-10, 36, 2
    lam = np.array([-0.1, -0.3, -0.05, -0.8, 0.2, -0.02, -0.2])
    resd = np.array([1e-3, 1e-6, 1e-8, 1e-2, 1e-3, np.inf, 5e-11])
    d = oc.degree_opt(resd, lam, c, e, tol, max_deg, extra)
    assert np.all(d % 2 == 0) and np.all((d >= 2) & (d <= max_deg)), d
    checked = 0
    for j in range(lam.shape[0]):
        t = (lam[j] - c) / e
        if abs(t) <= 1.0 or not np.isfinite(resd[j]):
            assert d[j] == max_deg, (j, d[j])
            continue
        if resd[j] <= tol:
            assert d[j] == max(2, extra + extra % 2), (j, d[j])
            continue
        g, k = _growth(t), int(d[j]) - extra
        assert d[j] < max_deg
        assert resd[j] * g ** (-k) <= tol * (1 + 1e-12), (j, d[j])
        assert resd[j] * g ** (-(k - 2)) > tol, (j, d[j])
        checked += 1
    assert checked == 4


def check_degree_order(oc):
    """Alg. 1's sort of the active columns by degree (R8: stable, ascending).
    Brute force over every pair of output positions: a permutation, with
    degrees non-decreasing and equal degrees in their input order.  Then in a
    solve: every filter call from the second iteration on sees non-decreasing
    degrees, and columns of equal degree in ascending Rayleigh quotient (the
    Ritz order they left Rayleigh-Ritz and locking in)."""
    rng = np.random.default_rng(8)
    for n in (1, 2, 7, 40):
        degs = rng.choice(np.arange(2, 38, 2), n)
        p = [int(x) for x in oc.degree_order(degs)]
        assert sorted(p) == list(range(n)), p
        for a in range(n):
            for b in range(a + 1, n):
                assert degs[p[a]] < degs[p[b]] or (degs[p[a]] == degs[p[b]] and p[a] < p[b]), (degs, p)

    N, nev, nex = 150, 12, 6
    lam = np.concatenate([np.linspace(-1.0, -0.9, 20), np.linspace(-0.5, 4.0, N - 20)])
    Q, _ = np.linalg.qr(synth.complex_gaussian(np.random.default_rng(81), (N, N)))
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    calls = []
    real_filter = oc.chebyshev_filter

    def spy(A_, V, degs, c, e, mu1):
        rq = np.real(np.sum(V.conj() * (A_ @ V), axis=0)) / np.real(np.sum(V.conj() * V, axis=0))
        calls.append((np.array(degs), rq))
        return real_filter(A_, V, degs, c, e, mu1)

    oc.chebyshev_filter = spy
    try:
        r = oc.chase(A, oc.Params(nev=nev, nex=nex, deg=8), rng_seed=3)
    finally:
        oc.chebyshev_filter = real_filter
    assert r.converged and len(calls) >= 3
    ties = 0
    for degs, rq in calls[1:]:
        assert np.all(np.diff(degs) >= 0), degs
        for j in range(degs.shape[0] - 1):
            if degs[j] == degs[j + 1]:
                ties += 1
                assert rq[j] <= rq[j + 1] + 1e-12 * np.max(np.abs(lam)), (degs, rq)
    assert ties > 0


def check_lock_order(oc):
    """Locking in Alg. 2: among the first n_lockable active pairs, those
    with resd <= tol move to the front in their order; the rest keep their
    relative order; a converged pair past n_lockable does not lock."""
    resd = np.array([5e-11, 2e-10, 1e-12, 3e-11, 1e-13, 1e-9])
    perm, k = oc.lock_order(resd, 4, 1e-10)
    assert k == 3
    assert list(perm) == [0, 2, 3, 1, 4, 5]


def check_qr_selection(oc):
    consts = _golden("paper_constants.json")
    hi = consts["cond_shifted_threshold"]["value"]
    lo = consts["cond_cholqr1_threshold"]["value"]
    assert oc.select_qr(hi * (1 + 1e-12)) == oc.QR_SHIFTED
    assert oc.select_qr(hi) == oc.QR_CHOLQR2
    assert oc.select_qr(lo) == oc.QR_CHOLQR2
    assert oc.select_qr(lo * (1 - 1e-12)) == oc.QR_CHOLQR1
    assert oc.select_qr(1.0) == oc.QR_CHOLQR1


def check_shift_formula(oc):
    # s = 11 (m n + n (n + 1)) u ||X||_F^2 with m = 1000, n = 10, ||X||_F^2 = 10:
    # 11 * 10110 * 10 = 1112100 units of 2^-53.
    assert oc.shifted_shift(1000, 10, 10.0) == 1112100 * 2.0 ** -53


# ----------------------------------------------------------------- CAQR

def matrix_with_cond(m, n, kappa, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(synth.complex_gaussian(rng, (m, n)))
    W, _ = np.linalg.qr(synth.complex_gaussian(rng, (n, n)))
    s = np.logspace(0, -math.log10(kappa), n)
    return (U * s) @ W.conj().T


def _orth(Q):
    return np.linalg.norm(Q.conj().T @ Q - np.eye(Q.shape[1]), 2)


def check_caqr_orthogonality(oc):
    m, n = 400, 24
    cases = [(10.0, oc.QR_CHOLQR1, 1e-12), (1e5, oc.QR_CHOLQR2, 1e-13),
             (1e7, oc.QR_CHOLQR2, 1e-13), (1e12, oc.QR_SHIFTED, 1e-13),
             (1e14, oc.QR_SHIFTED, 1e-13)]
    for i, (kappa, variant, bound) in enumerate(cases):
        X = matrix_with_cond(m, n, kappa, seed=100 + i)
        Q, used = oc.caqr(X, cond=kappa, force=variant)
        assert used == variant
        assert _orth(Q) <= bound, (kappa, _orth(Q))
        # span(Q) = span(X): X is reproduced by its projection on Q
        R = Q.conj().T @ X
        assert np.linalg.norm(Q @ R - X) <= 1e-12 * np.linalg.norm(X), kappa
        # R is upper triangular with |R| equal to LAPACK's up to a diagonal phase
        assert np.max(np.abs(np.tril(R, -1))) <= 1e-11 * np.max(np.abs(R))
        _, R_ref = np.linalg.qr(X)
        if kappa <= 1e7:
            rel = np.max(np.abs(np.abs(np.triu(R)) - np.abs(R_ref))) / np.max(np.abs(R_ref))
            assert rel <= 1e-10, (kappa, rel)


def check_caqr_fallback(oc):
    X = matrix_with_cond(200, 12, 10.0, seed=7)
    X[:, 5] = 0.0                        # rank deficient: every Cholesky route fails
    Q, used = oc.caqr(X, cond=1e3)
    assert used == oc.QR_HOUSEHOLDER
    assert _orth(Q) <= 1e-13
    X2 = matrix_with_cond(200, 12, 10.0, seed=8)
    X2[:, 3] = X2[:, 2]                  # duplicated column: Gram singular
    Q2, used2 = oc.caqr(X2, cond=10.0)
    assert used2 in (oc.QR_SHIFTED, oc.QR_HOUSEHOLDER)
    assert _orth(Q2) <= 1e-12


# ----------------------------------------------------------------- RR / residual

def check_rr_invariant_subspace(oc, seed=9):
    rng = np.random.default_rng(seed)
    N = 90
    lam = np.linspace(-2.0, 2.0, N)
    Q = synth.gaussian_unitary(N, rng)
    A = 0.5 * ((Q * lam) @ Q.conj().T + ((Q * lam) @ Q.conj().T).conj().T)
    idx = np.arange(3, 15)
    mix, _ = np.linalg.qr(synth.complex_gaussian(rng, (idx.size, idx.size)))
    C = Q[:, idx] @ mix
    theta, X = oc.rayleigh_ritz(A, C)
    assert np.max(np.abs(theta - lam[idx])) <= 1e-13 * 2.0, theta - lam[idx]
    r = oc.residual_norms(A, X, theta)
    assert np.max(r) <= 1e-13 * 2.0 * 10


def check_rr_interlacing(oc, seed=10):
    rng = np.random.default_rng(seed)
    N, n = 80, 10
    lam = np.sort(rng.uniform(-1, 1, N))
    A = synth.hermitian_from_spectrum(lam, "gaussian", seed=seed)
    C, _ = np.linalg.qr(synth.complex_gaussian(rng, (N, n)))
    theta, X = oc.rayleigh_ritz(A, C)
    assert np.all(np.diff(theta) >= 0)
    for j in range(n):
        assert lam[j] - 1e-13 <= theta[j] <= lam[N - n + j] + 1e-13
    # Ritz vectors are orthonormal and X^H A X = diag(theta)
    assert _orth(X) <= 1e-13
    assert np.max(np.abs(X.conj().T @ A @ X - np.diag(theta))) <= 1e-13


def check_residual_bruteforce(oc, seed=11):
    rng = np.random.default_rng(seed)
    N, n = 50, 7
    A = synth.hermitian_from_spectrum(rng.uniform(-1, 1, N), "gaussian", seed=seed)
    X = synth.complex_gaussian(rng, (N, n))
    theta = rng.uniform(-1, 1, n)
    got = oc.residual_norms(A, X, theta)
    for j in range(n):
        acc = 0.0
        for i in range(N):
            s = 0.0 + 0.0j
            for k in range(N):
                s += A[i, k] * X[k, j]
            s -= theta[j] * X[i, j]
            acc += s.real ** 2 + s.imag ** 2
        assert abs(got[j] - math.sqrt(acc)) <= 1e-13 * math.sqrt(acc)


# ----------------------------------------------------------------- whole solve

def check_solve_bruteforce(oc, N=120, nev=10, nex=6, seed=12, spectrum=None):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(-1, 1, N)) if spectrum is None else spectrum
    A = synth.hermitian_from_spectrum(lam, "gaussian", seed=seed)
    V0 = synth.complex_gaussian(rng, (N, nev + nex))
    starts = synth.complex_gaussian(rng, (N, 4))
    res = oc.chase(A, oc.Params(nev=nev, nex=nex), V0=V0, starts=starts)
    ref = np.linalg.eigvalsh(A)[:nev]
    normA = np.max(np.abs(lam))
    assert res.converged
    assert np.max(np.abs(res.evals - ref)) <= 1e-10 * normA, np.max(np.abs(res.evals - ref))
    X = res.evecs
    r = np.linalg.norm(A @ X - X * res.evals, axis=0)
    assert np.max(r) <= 1e-10 * normA
    assert _orth(X) <= 1e-12
    return res


def check_eigval_grad(oc, seed=13):
    """Hellmann-Feynman: finite differences of sum_i w_i lambda_i(A + hE)."""
    rng = np.random.default_rng(seed)
    N, nev = 40, 6
    lam = np.sort(rng.uniform(-1, 1, N))
    A = synth.hermitian_from_spectrum(lam, "gaussian", seed=seed)
    w = rng.uniform(0, 1, nev)
    evals, evecs = np.linalg.eigh(A)
    G = oc.eigval_grad(evecs[:, :nev], w)
    E = synth.complex_gaussian(rng, (N, N))
    E = 0.5 * (E + E.conj().T)
    h = 1e-6

    def loss(M):
        return float(np.dot(w, np.linalg.eigvalsh(M)[:nev]))

    fd = (loss(A + h * E) - loss(A - h * E)) / (2 * h)
    an = float(np.real(np.vdot(G, E)))
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)
    assert np.max(np.abs(G - G.conj().T)) <= 1e-15 * N
