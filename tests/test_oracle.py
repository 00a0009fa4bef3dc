"""The CPU oracle against closed forms, invariants, brute force and the
paper's constants; plus planted mistakes that each pin must catch."""
import types

import numpy as np
import pytest

import oracle.core as oc
import synth
from tests import pins

PINS = [
    pins.check_filter_golden,
    pins.check_filter_diagonal,
    pins.check_filter_rotated,
    pins.check_filter_unit_at_mu1,
    pins.check_lanczos_bounds,
    pins.check_lanczos_full_spectrum,
    pins.check_dos_closed_form,
    pins.check_condest_golden,
    pins.check_condest_overflow,
    pins.check_degree_opt,
    pins.check_degree_order,
    pins.check_lock_order,
    pins.check_qr_selection,
    pins.check_shift_formula,
    pins.check_caqr_orthogonality,
    pins.check_caqr_fallback,
    pins.check_rr_invariant_subspace,
    pins.check_rr_interlacing,
    pins.check_residual_bruteforce,
    pins.check_eigval_grad,
]


@pytest.mark.parametrize("check", PINS, ids=lambda f: f.__name__)
def test_pin(check):
    check(oc)


# ---------------------------------------------------------------- generators

@pytest.mark.parametrize("basis", ["gaussian", "fourier"])
def test_generator_spectrum(basis):
    lam = synth.dft_like_spectrum(300)
    A = synth.hermitian_from_spectrum(lam, basis=basis, seed=3)
    assert np.array_equal(A, A.conj().T)
    ev = np.linalg.eigvalsh(A)
    assert np.max(np.abs(ev - lam)) <= 1e-13 * np.max(np.abs(lam))


def test_dft_like_spectrum_shape():
    lam = synth.dft_like_spectrum(20000)
    assert lam.shape == (20000,)
    assert np.all(np.diff(lam) > 0)
    low = lam[:1000]
    assert low.min() > -1.0 and low.max() < -0.8
    assert lam[1000] > -0.8 and lam[-1] == 10.0


def test_fourier_rotation_matches_dense_unitary():
    """The FFT construction equals F diag(phi) F diag(lam) (F diag(phi) F)^H."""
    N = 64
    lam = np.linspace(-1, 2, N)
    rng = np.random.default_rng(synth.problems.SEED_Q)
    phi = np.exp(2j * np.pi * rng.random(N))
    F = np.fft.fft(np.eye(N), axis=0, norm="ortho")
    Q = F @ np.diag(phi) @ F
    ref = (Q * lam) @ Q.conj().T
    got = synth.hermitian_from_spectrum(lam, "fourier")
    assert np.max(np.abs(got - 0.5 * (ref + ref.conj().T))) <= 1e-13


def test_symmetric_generators_spectrum():
    """Both real symmetric constructions: exactly symmetric, the prescribed
    spectrum, and the device one's rotation is orthogonal (checked on CPU)."""
    import torch
    lam = synth.dft_like_spectrum(200)
    A = synth.symmetric_from_spectrum(lam, seed=5)
    assert A.dtype == np.float64 and np.array_equal(A, A.T)
    assert np.max(np.abs(np.linalg.eigvalsh(A) - lam)) <= 1e-13 * np.max(np.abs(lam))
    T = synth.problems.symmetric_from_spectrum_torch(lam, seed=5, device="cpu").numpy()
    assert np.array_equal(T, T.T)
    assert np.max(np.abs(np.linalg.eigvalsh(T) - lam)) <= 1e-12 * np.max(np.abs(lam))
    assert np.max(np.abs(T - np.diag(np.diag(T)))) > 1e-3        # dense, not diagonal


def test_real_problem_inputs():
    p = synth.make_problem(50, 4, 2, spectrum="dft", seed=3, real=True)
    assert p.A.dtype == p.V0.dtype == p.starts.dtype == np.float64
    assert p.V0.shape == (50, 6) and p.starts.shape == (50, 4)


# ---------------------------------------------------------------- whole solve

def test_solve_bruteforce_small():
    pins.check_solve_bruteforce(oc, N=120, nev=10, nex=6, seed=12)


def test_solve_bruteforce_dft_like():
    pins.check_solve_bruteforce(oc, N=200, nev=8, nex=4, seed=14,
                                spectrum=synth.dft_like_spectrum(200))


def test_parity_problem_known_spectrum(parity_problem, parity_oracle):
    p, r = parity_problem, parity_oracle
    assert r.converged
    normA = p.norm2
    assert np.max(np.abs(r.evals - p.lam[: p.nev])) <= 1e-10 * normA
    X = r.evecs
    resid = np.linalg.norm(p.A @ X - X * r.evals, axis=0)
    assert np.max(resid) <= 1e-10 * normA
    assert np.linalg.norm(X.conj().T @ X - np.eye(p.nev), 2) <= 1e-12
    # reported residuals are the true ones
    assert np.max(np.abs(resid - r.resid)) <= 1e-12


@pytest.mark.parametrize("opt", [1, 0])
def test_condest_bounds_computed_condition(parity_problem, opt):
    """From the second iteration on, the estimate of Alg. 5 bounds kappa_2 of
    the filtered columns from above (Sec. 4.2 reports it for the filter's
    output at every iteration after the first, with and without degree
    optimisation).  With the filter normalised at mu_1 the locked columns keep
    norm 1 above the filtered ones, so kappa_2 of the whole block can exceed
    the estimate once pairs lock; it is bounded while none are locked."""
    p = parity_problem
    rec = []
    orig = oc.caqr

    def spy(X, cond, force=None):
        rec.append((cond, X.copy()))
        return orig(X, cond, force)

    try:
        oc.caqr = spy
        r = oc.chase(p.A, oc.Params(nev=p.nev, nex=p.nex, opt=opt), V0=p.V0, starts=p.starts)
    finally:
        oc.caqr = orig
    assert len(rec) >= 2 and len(rec) == len(r.history)

    def kappa(X):
        sv = np.linalg.svd(X, compute_uv=False)
        return sv[0] / sv[-1]

    for h, (est, X) in list(zip(r.history, rec))[1:]:
        lk = h["locked_before"]
        assert est >= kappa(X[:, lk:]), (h["iteration"], est)
        if lk == 0:
            assert est >= kappa(X), (h["iteration"], est)


def test_warm_start_from_exact_eigenvectors(parity_problem):
    """Approximate eigenvectors may be passed in (Sec. 1, Alg. 1's initial
    block): started from the exact lowest n_e eigenvectors, the filter and
    the QR keep their span, Rayleigh-Ritz returns the exact pairs and every
    wanted pair locks in the first iteration."""
    p = parity_problem
    w, Q = np.linalg.eigh(p.A)
    r = oc.chase(p.A, oc.Params(nev=p.nev, nex=p.nex), V0=Q[:, : p.ne], starts=p.starts)
    assert r.converged and r.iterations == 1
    assert np.max(np.abs(r.evals - w[: p.nev])) <= 1e-13


def test_householder_same_matvecs(parity_problem, parity_oracle):
    """CholeskyQR and Householder QR give the same MatVecs and iteration
    counts (Sec. 4.3, Table 2 discussion)."""
    p = parity_problem
    hh = oc.chase(p.A, oc.Params(nev=p.nev, nex=p.nex, force_qr=oc.QR_HOUSEHOLDER),
                  V0=p.V0, starts=p.starts)
    assert hh.iterations == parity_oracle.iterations
    assert hh.filter_matvecs == parity_oracle.filter_matvecs
    assert np.max(np.abs(hh.evals - parity_oracle.evals)) <= 1e-12


def test_not_converged_status(parity_problem):
    p = parity_problem
    r = oc.chase(p.A, oc.Params(nev=p.nev, nex=p.nex, max_iter=1), V0=p.V0, starts=p.starts)
    assert not r.converged and r.iterations == 1
    assert r.evals.shape == (p.nev,) and np.all(np.diff(r.evals) >= 0)


def test_invalid_arguments():
    A = np.eye(10, dtype=np.complex128)
    with pytest.raises(ValueError):
        oc.chase(A, oc.Params(nev=8, nex=2))
    with pytest.raises(ValueError):
        oc.chase(A, oc.Params(nev=2, nex=2, deg=3))


def test_degree_opt_properties():
    resd = np.array([1e-2, 1e-6, 1e-11, np.inf, 1e-3])
    Lam = np.array([-1.0, -0.9, -0.95, -0.5, 0.5])
    d = oc.degree_opt(resd, Lam, c=0.5, e=0.9, tol_abs=1e-10, max_deg=36, deg_extra=2)
    assert np.all(d % 2 == 0) and np.all(d >= 2) and np.all(d <= 36)
    assert d[0] > d[1]            # larger residual, same region -> more steps
    assert d[2] == 2              # already converged
    assert d[3] == 36             # non-finite residual -> cap
    assert d[4] == 36             # inside the damped interval -> cap


def test_lock_order():
    order, n = oc.lock_order(np.array([1.0, 1e-12, 1e-11, 1e-12, 1e-13]), 3, 1e-10)
    assert n == 2 and list(order) == [1, 2, 0, 3, 4]


# ---------------------------------------------------------------- planted mistakes

def _mutant(**overrides):
    m = types.ModuleType("oracle_mutant")
    m.__dict__.update({k: v for k, v in oc.__dict__.items() if not k.startswith("__")})
    m.__dict__.update(overrides)
    # functions look globals up in their own module: rebind them to the mutant
    for name, fn in list(m.__dict__.items()):
        if isinstance(fn, types.FunctionType) and name not in overrides:
            m.__dict__[name] = types.FunctionType(fn.__code__, m.__dict__, fn.__name__,
                                                  fn.__defaults__, fn.__closure__)
    return m


def _coeffs_wrong_beta_sign(c, e, mu1, m):
    return [(a, g, -b) for a, g, b in oc.filter_coefficients(c, e, mu1, m)]


def _coeffs_no_shift(c, e, mu1, m):
    return [(a, 0.0, b) for a, g, b in oc.filter_coefficients(c, e, mu1, m)]


def _coeffs_unscaled_first(c, e, mu1, m):
    out = oc.filter_coefficients(c, e, mu1, m)
    out[0] = (2.0 * out[0][0], out[0][1], out[0][2])
    return out


def _filter_transposed(A, V, degs, c, e, mu1):
    return oc.chebyshev_filter(A.T, V, degs, c, e, mu1)


def _rr_no_conj(A, Q):
    B = A @ Q
    G = Q.T @ B
    G = 0.5 * (G + G.conj().T)
    theta, W = np.linalg.eigh(G)
    return theta, Q @ W


def _resid_dropped_theta(A, X, theta):
    return np.linalg.norm(A @ X, axis=0)


def _cond_swapped(Lam, c, e, degs, locked):
    t_first = (Lam[0] - c) / e
    t_active = (Lam[locked] - c) / e
    d = int(degs[locked])
    d_max = int(np.max(degs[locked:]))
    return oc.rho(t_first) ** d * oc.rho(t_active) ** (d_max - d)


def _shift_ten(m, n, fro2):
    return 10.0 * (m * n + n * (n + 1)) * oc.U_ROUNDOFF * fro2


def _select_swapped(cond):
    if cond > oc.COND_SHIFTED:
        return oc.QR_SHIFTED
    if cond <= oc.COND_CHOLQR1:
        return oc.QR_CHOLQR1
    return oc.QR_CHOLQR2


def _rsolve_wrong(X, R):
    return X @ np.linalg.inv(R).T


def _bsup_no_beta(A, starts, ne, k=25):
    b, m1, mne, nrm = oc.lanczos_bounds(A, starts, ne, k)
    top = max(oc.tridiagonal_eig(*oc.lanczos_run(A, starts[:, r], min(k, A.shape[0])))[0][-1]
              for r in range(starts.shape[1]))
    return top, m1, min(mne, top), nrm


def _lanczos_missing_term(A, start, k):
    v = start / np.linalg.norm(start)
    alphas, betas = [], []
    for _ in range(k):
        w = A @ v
        alpha = float(np.real(np.vdot(v, w)))
        w = w - alpha * v
        beta = float(np.linalg.norm(w))
        alphas.append(alpha)
        betas.append(beta)
        v = w / beta
    return np.array(alphas), np.array(betas)


def _degree_floor(resd, Lam, c, e, tol_abs, max_deg, deg_extra):
    out = []
    for j in range(resd.shape[0]):
        r = oc.rho((Lam[j] - c) / e)
        if r <= 1.0 + 1e-12 or not np.isfinite(resd[j]):
            d = max_deg
        elif resd[j] <= tol_abs:
            d = deg_extra
        else:
            d = int(np.floor(np.log(resd[j] / tol_abs) / np.log(r))) + deg_extra
        d = min(max(d, 2), max_deg)
        out.append(d + d % 2)
    return np.array(out)


def _degree_no_margin(resd, Lam, c, e, tol_abs, max_deg, deg_extra):
    return oc.degree_opt(resd, Lam, c, e, tol_abs, max_deg, 0)


def _degree_order_descending(degs):
    return np.argsort(-np.asarray(degs), kind="stable")


def _degree_order_ties_reversed(degs):
    degs = np.asarray(degs)
    return np.lexsort((-np.arange(degs.shape[0]), degs))


def _degree_order_none(degs):
    return np.arange(np.asarray(degs).shape[0])


def _lock_past_nev(resd_active, n_lockable, tol_abs):
    return oc.lock_order(resd_active, resd_active.shape[0], tol_abs)


def _dos_next_count(A, starts, ne, k=25):
    return oc.lanczos_bounds(A, starts, ne + 1, k)


def _dos_last_component(A, starts, ne, k=25):
    N = A.shape[0]
    k = min(k, N)
    R = starts.shape[1]
    b_sup, mu_1, theta_max = -np.inf, np.inf, -np.inf
    nodes, weights = [], []
    for r in range(R):
        alpha, beta = oc.lanczos_run(A, starts[:, r], k)
        theta, Z = oc.tridiagonal_eig(alpha, beta)
        b_sup = max(b_sup, theta[-1] + beta[-1])
        mu_1 = min(mu_1, theta[0])
        theta_max = max(theta_max, theta[-1])
        nodes.append(theta)
        weights.append(np.abs(Z[-1, :]) ** 2)
    nodes, weights = np.concatenate(nodes), np.concatenate(weights)
    order = np.argsort(nodes, kind="stable")
    count = N * np.cumsum(weights[order]) / R
    idx = min(int(np.searchsorted(count, ne, side="left")), nodes.shape[0] - 1)
    mu_ne = min(max(float(nodes[order][idx]), mu_1), np.nextafter(b_sup, -np.inf))
    return float(b_sup), float(mu_1), mu_ne, float(max(abs(mu_1), abs(theta_max)))


def _grad_transposed(X, g):
    return (X.conj() * g[None, :]) @ X.T


MUTANTS = [
    ("beta sign", dict(filter_coefficients=_coeffs_wrong_beta_sign),
     [pins.check_filter_golden, pins.check_filter_diagonal]),
    ("no shift", dict(filter_coefficients=_coeffs_no_shift),
     [pins.check_filter_diagonal, pins.check_filter_rotated]),
    ("first step", dict(filter_coefficients=_coeffs_unscaled_first),
     [pins.check_filter_golden, pins.check_filter_unit_at_mu1]),
    ("transposed A", dict(chebyshev_filter=_filter_transposed), [pins.check_filter_rotated]),
    ("RR without conj", dict(rayleigh_ritz=_rr_no_conj),
     [pins.check_rr_invariant_subspace, pins.check_rr_interlacing]),
    ("residual theta dropped", dict(residual_norms=_resid_dropped_theta),
     [pins.check_residual_bruteforce, pins.check_rr_invariant_subspace]),
    ("condest exponents swapped", dict(cond_est=_cond_swapped), [pins.check_condest_golden]),
    ("shift factor", dict(shifted_shift=_shift_ten), [pins.check_shift_formula]),
    ("threshold inclusive", dict(select_qr=_select_swapped), [pins.check_qr_selection]),
    ("TRSM transposed", dict(_right_solve_upper=_rsolve_wrong), [pins.check_caqr_orthogonality]),
    ("b_sup too low", dict(lanczos_bounds=_bsup_no_beta), [pins.check_lanczos_bounds]),
    ("Lanczos three-term dropped", dict(lanczos_run=_lanczos_missing_term),
     [pins.check_lanczos_full_spectrum]),
    ("gradient transposed", dict(eigval_grad=_grad_transposed), [pins.check_eigval_grad]),
    ("degree rounded down", dict(degree_opt=_degree_floor), [pins.check_degree_opt]),
    ("degree without margin", dict(degree_opt=_degree_no_margin), [pins.check_degree_opt]),
    ("locking past nev", dict(lock_order=_lock_past_nev), [pins.check_lock_order]),
    ("degree sort descending", dict(degree_order=_degree_order_descending), [pins.check_degree_order]),
    ("degree sort with ties reversed", dict(degree_order=_degree_order_ties_reversed),
     [pins.check_degree_order]),
    ("no degree sort", dict(degree_order=_degree_order_none), [pins.check_degree_order]),
    ("DoS count off by one", dict(lanczos_bounds=_dos_next_count), [pins.check_dos_closed_form]),
    ("DoS weights from the last component", dict(lanczos_bounds=_dos_last_component),
     [pins.check_dos_closed_form]),
]


@pytest.mark.parametrize("name,overrides,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, overrides, checks):
    mutant = _mutant(**overrides)
    for check in checks:
        with pytest.raises(AssertionError):
            check(mutant)
