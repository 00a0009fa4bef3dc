"""GPU checks of the complex64 variant through the C ABI.

The solve works on H rounded to complex64 (the caller's data); its filter and
H Q products are FP32, so residuals bottom out near sqrt(N) u_32 ||H|| and the
tests use tol = 1e-5.  Checks: the reported residuals are the true ones of the
returned vectors against the complex64 matrix (up to the FP32 products),
eigenvalues within 1e-6 ||H|| of the prescribed spectrum and of the FP64
oracle, orthonormal vectors to complex64 accuracy.
"""
import numpy as np
import pytest

import oracle.core as oc
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_15595_amd import _lib
    _lib.load()
    return _lib


def cm64(x):
    from paper_2309_15595_amd.api import colmajor
    return colmajor(np.asarray(x, dtype=np.complex64))


def solve_c64(p, **kw):
    from paper_2309_15595_amd.api import Solver, from_colmajor
    kw.setdefault("tol", TOL)
    with Solver(p.N, p.nev, p.nex, dtype=torch.complex64, **kw) as s:
        Vd = cm64(p.V0)
        ritz, resid, info = s.solve_colmajor(cm64(p.A), Vd, True, cm64(p.starts))
        X = from_colmajor(Vd)[:, : p.nev]
    return ritz, resid, X, info


@pytest.mark.parametrize("N,nev,nex,spectrum", [(800, 60, 20, "uniform"), (333, 13, 7, "dft"),
                                                (1000, 90, 26, "uniform")])
def test_c64_solve(L, N, nev, nex, spectrum):
    """N = 333: odd order and leading dimension, so the FP32 steps take the
    staged kernel instead of the direct-to-LDS one."""
    p = synth.make_problem(N, nev, nex, spectrum=spectrum, seed=N)
    ritz, resid, X, info = solve_c64(p)
    assert info.converged, info.stats
    st = info.stats
    assert st["filter_matvecs_fp32"] == st["filter_matvecs"] > 0
    assert X.dtype == np.complex64
    normA = p.norm2
    A32 = p.A.astype(np.complex64).astype(np.complex128)   # the matrix actually solved
    Xd = X.astype(np.complex128)
    assert np.all(np.diff(ritz) >= 0)
    assert np.max(np.abs(ritz - p.lam[: nev])) <= 1e-6 * normA
    r_true = np.linalg.norm(A32 @ Xd - Xd * ritz, axis=0)
    assert np.max(r_true) <= 2 * TOL * normA
    assert np.max(np.abs(r_true - resid)) <= 1e-6 * normA
    assert np.linalg.norm(Xd.conj().T @ Xd - np.eye(nev), 2) <= 1e-5
    r = oc.chase(p.A, oc.Params(nev=nev, nex=nex, tol=TOL), V0=p.V0, starts=p.starts)
    assert np.max(np.abs(ritz - r.evals)) <= 1e-6 * normA
    print(f"\nN={N}: c64 iters {st['iterations']} matvecs {st['filter_matvecs']}; "
          f"oracle (FP64, same tol) iters {r.iterations} matvecs {r.filter_matvecs}")


def test_c64_lanczos_bounds_match_complex128(L):
    """The complex64 Lanczos (FP64 accumulation over complex64 H) gives the
    bounds of the complex128 one to FP32 accuracy."""
    from paper_2309_15595_amd.api import Solver
    p = synth.make_problem(400, 20, 10, spectrum="uniform", seed=11)
    with Solver(p.N, p.nev, p.nex, dtype=torch.complex64, tol=TOL, max_iter=1) as s:
        _, _, i32 = s.solve_colmajor(cm64(p.A), cm64(p.V0), True, cm64(p.starts))
    from paper_2309_15595_amd.api import colmajor
    with Solver(p.N, p.nev, p.nex, max_iter=1) as s:
        _, _, i64 = s.solve_colmajor(colmajor(p.A), colmajor(p.V0), True, colmajor(p.starts))
    b32, b64 = np.array(i32.stats["bounds"]), np.array(i64.stats["bounds"])
    assert np.max(np.abs(b32 - b64)) <= 1e-5 * p.norm2, (b32, b64)


def test_c64_guards(L):
    from paper_2309_15595_amd.api import Solver
    p = synth.make_problem(64, 4, 4, seed=1)
    with pytest.raises(ValueError):      # BF16x3 is not offered on complex64 data
        Solver(p.N, p.nev, p.nex, dtype=torch.complex64, precision=L.CHASE_BF16X3_MIXED)
    with Solver(p.N, p.nev, p.nex, dtype=torch.complex64) as s:
        with pytest.raises(TypeError):   # complex128 data for a complex64 handle
            s.solve_colmajor(torch.zeros((64, 64), dtype=torch.complex128, device="cuda"),
                             torch.zeros((8, 64), dtype=torch.complex128, device="cuda"))
        rz = L.f64_array(4)
        assert L.load().chase_solve(s.h, L.dptr(cm64(p.A)), 64, L.dptr(cm64(p.V0)), 64, 1, None, 0, 0,
                                    rz, rz, None, None) == -1


def test_c64_leading_dimension(L):
    """lda, ldv > N and odd: the FP32 steps take the staged kernel; padding
    rows of the block are untouched; the same pairs as the packed layout."""
    from paper_2309_15595_amd.api import from_colmajor
    p = synth.make_problem(256, 10, 6, spectrum="uniform", seed=5)
    ld = p.N + 5
    Abig = np.zeros((ld, p.N), dtype=np.complex64)
    Abig[: p.N] = p.A
    Vbig = np.full((ld, p.ne), 3.0 + 3.0j, dtype=np.complex64)
    Vbig[: p.N] = p.V0
    prm = L.default_params(nev=p.nev, nex=p.nex, tol=TOL)
    h = L.chase_create_c64(p.N, prm)
    try:
        Ad, Vd, Sd = cm64(Abig), cm64(Vbig), cm64(p.starts)
        ritz, resid, st = L.chase_solve_c64(h, L.dptr(Ad), ld, L.dptr(Vd), ld, 1, L.dptr(Sd), p.N, 4, p.nev,
                                            L.stream_ptr())
    finally:
        L.chase_destroy(h)
    assert st.status == 0
    got = from_colmajor(Vd)
    assert np.all(got[p.N:] == np.complex64(3.0 + 3.0j))
    ref_ritz, _, _, _ = solve_c64(p)
    assert np.max(np.abs(np.array(ritz) - ref_ritz)) <= 1e-6 * p.norm2
    assert np.max(np.abs(np.array(ritz) - p.lam[: p.nev])) <= 1e-6 * p.norm2


@pytest.mark.parametrize("N,nev,nex", [(2, 1, 0), (3, 1, 1), (8, 1, 1), (9, 2, 2), (64, 1, 1), (64, 40, 23)])
def test_c64_tiny_orders(L, N, nev, nex):
    p = synth.make_problem(N, nev, nex, spectrum="uniform", seed=200 + N)
    ritz, resid, X, info = solve_c64(p)
    assert info.converged, info.stats
    assert np.max(np.abs(ritz - p.lam[: nev])) <= 1e-6 * p.norm2


def test_c64_eigsh_torch_layout(L):
    """eigsh on a row-major complex64 torch tensor: A's (not conj(A)'s)
    vectors, eigenvalues within 1e-6 ||H|| of the prescribed spectrum, and
    the same eigenvalues as the column-major Solver call on the same data."""
    from paper_2309_15595_amd.api import eigsh
    p = synth.make_problem(256, 10, 6, spectrum="uniform", seed=44)
    A32 = p.A.astype(np.complex64)
    A = torch.from_numpy(A32).cuda()
    evals, evecs, info = eigsh(A, p.nev, p.nex, tol=TOL, V0=torch.from_numpy(p.V0.astype(np.complex64)).cuda(),
                               starts=torch.from_numpy(p.starts.astype(np.complex64)).cuda())
    assert info.converged, info.stats
    assert evecs.dtype == torch.complex64
    X = evecs.cpu().numpy().astype(np.complex128)
    ev = evals.cpu().numpy()
    A64 = A32.astype(np.complex128)
    assert np.max(np.abs(ev - p.lam[: p.nev])) <= 1e-6 * p.norm2
    assert np.max(np.linalg.norm(A64 @ X - X * ev, axis=0)) <= 4 * TOL * p.norm2
    assert np.linalg.norm(X.conj().T @ X - np.eye(p.nev), 2) <= 1e-5
    with pytest.raises(ValueError):
        eigsh(A, p.nev, p.nex, precision="bf16x3")
