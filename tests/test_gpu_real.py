"""GPU parity of the real symmetric variant (FP64) through the C ABI.

The oracle solves a real symmetric problem as the Hermitian one it is (its
complex arithmetic on zero imaginary parts is the real arithmetic), so the
filter is compared element by element with the oracle's recurrence and whole
solves with the prescribed spectrum and the oracle's eigenvalues.
Tolerances as for the complex path: the real filter sums the same length-N
inner products (normwise 1e-11 over d <= 36 steps), eigenvalues within the
paper's 1e-10 ||A||.
"""
import numpy as np
import pytest

import oracle.core as oc
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_15595_amd import _lib
    _lib.load()
    return _lib


def cm(x):
    from paper_2309_15595_amd.api import colmajor
    return colmajor(np.asarray(x, dtype=np.float64))


def un(t):
    from paper_2309_15595_amd.api import from_colmajor
    return from_colmajor(t)


def sp():
    from paper_2309_15595_amd import _lib
    return _lib.stream_ptr()


# ---------------------------------------------------------------- filter

@pytest.mark.parametrize("N,degs", [
    (518, [2, 2, 4, 6, 6, 10, 20, 20, 36] + [20] * 60 + [36] * 7),   # 76 columns, ragged tiles
    (800, [20] * 80),
    (130, [2, 4]),
    (1024, [36] * 300),                                             # several column tiles
])
def test_real_filter_matches_oracle(L, N, degs):
    rng = np.random.default_rng(N)
    lam = np.sort(rng.uniform(-1.0, 2.0, N))
    A = synth.symmetric_from_spectrum(lam, seed=N)
    degs = np.sort(np.array(degs))
    n = degs.size
    V = rng.standard_normal((N, n))
    c, e, mu1 = 1.1, 0.9, lam[0] + 1e-3
    ref, mv_ref = oc.chebyshev_filter(A, V, degs, c, e, mu1)
    assert np.all(ref.imag == 0)
    ref = ref.real
    Ad, Vd = cm(A), cm(V)
    Wd = torch.zeros_like(Vd)
    mv = L.chase_filter_real(L.dptr(Ad), N, L.dptr(Vd), N, L.dptr(Wd), N, N, n, degs, c, e, mu1, sp())
    got = un(Vd)
    assert mv == mv_ref
    err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= 1e-11, err.max()


def test_real_filter_leading_dimension(L):
    """Even lda, ldv > N: the padding rows are neither read into nor written."""
    N, n, pad = 200, 9, 14
    rng = np.random.default_rng(3)
    A = synth.symmetric_from_spectrum(rng.uniform(-1, 1, N), seed=3)
    V = rng.standard_normal((N, n))
    Abig = np.full((N + pad, N), np.nan)
    Abig[:N] = A
    Vbig = np.full((N + pad, n), 7.0)
    Vbig[:N] = V
    Ad, Vd = cm(Abig), cm(Vbig)
    Wd = torch.zeros_like(Vd)
    degs = [4] * n
    L.chase_filter_real(L.dptr(Ad), N + pad, L.dptr(Vd), N + pad, L.dptr(Wd), N + pad, N, n, degs,
                        0.5, 0.6, -1.0, sp())
    got = un(Vd)
    ref, _ = oc.chebyshev_filter(A, V, np.array(degs), 0.5, 0.6, -1.0)
    assert np.all(got[N:] == 7.0)
    assert np.max(np.abs(got[:N] - ref.real)) <= 1e-11 * np.max(np.abs(ref))


def test_real_filter_rejects_odd_layout(L):
    d = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):   # odd N
        L.chase_filter_real(L.dptr(d), 8, L.dptr(d), 8, L.dptr(d), 8, 7, 1, [2], 0.0, 1.0, -1.5, sp())
    with pytest.raises(ValueError):   # odd ldv
        L.chase_filter_real(L.dptr(d), 8, L.dptr(d), 7, L.dptr(d), 8, 6, 1, [2], 0.0, 1.0, -1.5, sp())


# ---------------------------------------------------------------- whole solve

def solve_real(p, **kw):
    from paper_2309_15595_amd.api import Solver
    with Solver(p.N, p.nev, p.nex, dtype=torch.float64, **kw) as s:
        Vd = cm(p.V0)
        ritz, resid, info = s.solve_colmajor(cm(p.A), Vd, True, cm(p.starts))
        X = un(Vd)[:, : p.nev]
    return ritz, resid, X, info


def check_real_solution(p, ritz, resid, X, tol=1e-10):
    normA = p.norm2
    assert X.dtype == np.float64
    assert np.all(np.diff(ritz) >= 0)
    assert np.max(np.abs(ritz - p.lam[: p.nev])) <= tol * normA
    r_true = np.linalg.norm(p.A @ X - X * ritz, axis=0)
    assert np.max(r_true) <= tol * normA * (1 + 1e-6)
    assert np.max(np.abs(r_true - resid)) <= 1e-12 * normA
    assert np.linalg.norm(X.T @ X - np.eye(p.nev), 2) <= 1e-12


@pytest.mark.parametrize("N,nev,nex,spectrum", [(800, 60, 20, "uniform"), (333, 13, 7, "dft"),
                                                (1000, 90, 26, "uniform"), (201, 8, 4, "dft")])
def test_real_solve_matches_oracle(L, N, nev, nex, spectrum):
    """Even orders read H in place; odd ones (333, 201) go through the padded
    copy with its zero row."""
    p = synth.make_problem(N, nev, nex, spectrum=spectrum, seed=N, real=True)
    ritz, resid, X, info = solve_real(p)
    assert info.converged, info.stats
    check_real_solution(p, ritz, resid, X)
    r = oc.chase(p.A, oc.Params(nev=nev, nex=nex), V0=p.V0, starts=p.starts)
    assert np.max(np.abs(ritz - r.evals)) <= 1e-10 * p.norm2
    st = info.stats
    print(f"\nN={N}: GPU iters {st['iterations']} matvecs {st['filter_matvecs']}; "
          f"oracle iters {r.iterations} matvecs {r.filter_matvecs}")
    assert abs(st["iterations"] - r.iterations) <= 1
    assert abs(st["filter_matvecs"] - r.filter_matvecs) <= 0.05 * r.filter_matvecs
    assert st["filter_flops"] == pytest.approx(2.0 * N * N * st["filter_matvecs"])


@pytest.mark.parametrize("force", [0, 1, 2, 3])
def test_real_solve_forced_qr_variants(L, force):
    p = synth.make_problem(400, 20, 10, spectrum="uniform", seed=11, real=True)
    ritz, resid, X, info = solve_real(p, force_qr=force)
    assert info.converged
    check_real_solution(p, ritz, resid, X)
    assert info.stats["qr_count"][force] == info.stats["iterations"]


def test_real_solve_random_start_and_trace(L):
    """Library-drawn start block and Lanczos starts (odd order: the padding
    row must stay zero), and the trace's singular values of the real block."""
    from paper_2309_15595_amd.api import Solver
    p = synth.make_problem(301, 12, 6, spectrum="uniform", seed=9, real=True)
    with Solver(p.N, p.nev, p.nex, dtype=torch.float64) as s:
        s.set_trace(2)
        Vd = torch.empty((p.ne, p.N), dtype=torch.float64, device="cuda")
        ritz, resid, info = s.solve_colmajor(cm(p.A), Vd, False, None)
        tr = s.trace()
    X = un(Vd)[:, : p.nev]
    assert info.converged
    check_real_solution(p, ritz, resid, X)
    assert len(tr) == info.stats["iterations"]
    for t in tr[1:]:
        assert t["kappa_est"] >= t["kappa_com_active"] * (1 - 1e-8), t
    assert all(t["kappa_com"] >= 1.0 for t in tr)


def test_real_handle_guards(L):
    from paper_2309_15595_amd.api import Solver
    p = synth.make_problem(64, 4, 4, seed=1, real=True)
    with Solver(p.N, p.nev, p.nex, dtype=torch.float64) as s:
        with pytest.raises(TypeError):   # complex data for a real handle
            s.solve_colmajor(torch.zeros((64, 64), dtype=torch.complex128, device="cuda"),
                             torch.zeros((8, 64), dtype=torch.complex128, device="cuda"))
        rz = L.f64_array(4)
        assert L.load().chase_solve(s.h, L.dptr(cm(p.A)), 64, L.dptr(cm(p.V0)), 64, 1, None, 0, 0,
                                    rz, rz, None, None) == -1
    with pytest.raises(ValueError):      # mixed precision is FP64-only on the real path
        Solver(p.N, p.nev, p.nex, dtype=torch.float64, precision=L.CHASE_FP32_MIXED)


def test_eigsh_real(L):
    from paper_2309_15595_amd.api import eigsh
    p = synth.make_problem(256, 10, 6, spectrum="dft", seed=4, real=True)
    A = torch.from_numpy(p.A).cuda()
    evals, evecs, info = eigsh(A, p.nev, p.nex, V0=torch.from_numpy(p.V0).cuda(),
                               starts=torch.from_numpy(p.starts).cuda())
    assert evecs.dtype == torch.float64 and info.converged
    X = evecs.cpu().numpy()
    lam = evals.cpu().numpy()
    assert np.max(np.abs(lam - p.lam[: p.nev])) <= 1e-10 * p.norm2
    assert np.max(np.linalg.norm(p.A @ X - X * lam, axis=0)) <= 1e-10 * p.norm2 * (1 + 1e-6)


def test_real_solve_odd_leading_dimension(L):
    """Even order with an odd leading dimension (the padded copy of H) and a
    block with its own padding rows, through the C ABI: the same pairs as the
    in-place layout."""
    p = synth.make_problem(300, 12, 6, spectrum="dft", seed=31, real=True)
    ld = p.N + 3
    Abig = np.full((ld, p.N), np.nan)
    Abig[: p.N] = p.A
    Vbig = np.full((ld, p.ne), 5.0)
    Vbig[: p.N] = p.V0
    prm = L.default_params(nev=p.nev, nex=p.nex)
    h = L.chase_create_real(p.N, prm)
    try:
        Ad, Vd, Sd = cm(Abig), cm(Vbig), cm(p.starts)
        ritz, resid, st = L.chase_solve_real(h, L.dptr(Ad), ld, L.dptr(Vd), ld, 1, L.dptr(Sd), p.N, 4, p.nev,
                                             sp())
    finally:
        L.chase_destroy(h)
    assert st.status == 0
    got = un(Vd)
    assert np.all(got[p.N:] == 5.0)                      # padding rows untouched
    ref_ritz, ref_resid, X, info = solve_real(p)
    assert np.max(np.abs(np.array(ritz) - ref_ritz)) <= 1e-12 * p.norm2
    check_real_solution(p, np.array(ritz), np.array(resid), got[: p.N, : p.nev])


@pytest.mark.parametrize("N,nev,nex", [(2, 1, 0), (3, 1, 1), (5, 1, 1), (16, 2, 2), (17, 3, 1), (64, 1, 0),
                                       (33, 20, 12), (64, 40, 23)])   # n_e = N - 1
def test_real_tiny_orders(L, N, nev, nex):
    """Degenerate sizes: one-tile problems, odd orders (one padding row), a
    single wanted pair, a block of N - 1 columns, and nex = 0, where the damped interval starts at the
    wanted eigenvalue itself and the method (oracle alike) does not reach
    tol within MaxIter: the outcome must be the oracle's."""
    p = synth.make_problem(N, nev, nex, spectrum="uniform", seed=100 + N, real=True)
    ritz, resid, X, info = solve_real(p)
    r = oc.chase(p.A, oc.Params(nev=nev, nex=nex), V0=p.V0, starts=p.starts)
    assert info.converged == r.converged, (info.stats, r.converged)
    if r.converged:
        check_real_solution(p, ritz, resid, X)
        assert np.max(np.abs(ritz - r.evals)) <= 1e-10 * p.norm2
    else:
        assert info.status == 1 and info.stats["iterations"] == r.iterations
        assert np.max(np.abs(ritz - r.evals)) <= 1e-8 * p.norm2
        assert np.max(resid) <= 10 * np.max(r.resid)
