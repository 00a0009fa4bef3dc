"""GPU parity of the small eigensolve of Rayleigh-Ritz (Alg. 2; the dense
solver step of Sec. 3.1), chase_heev, against numpy.linalg.eigh (LAPACK's
divide and conquer) on the host, through the C ABI.

Eigenvalues are unique: compared directly, within 1e-13 ||G||_2 (a backward
stable solver perturbs them by O(n u ||G||); the block-Jacobi sweeps stay
within a few hundred ulps of ||G|| up to n = 2400).  Eigenvectors are unique
only up to a phase, or a unitary mixing inside a cluster: they are checked by
residual max_j ||G x_j - theta_j x_j|| <= 1e-13 ||G||_2 and orthogonality
||X^H X - I||_2 <= 1e-13, and, for eigenvalues separated from their
neighbours by more than 1e-6 ||G||, by |x_j^H y_j| = 1 against LAPACK's
vector y_j (to 1e-13 / gap).
"""
import numpy as np
import pytest

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
    return colmajor(np.asarray(x, dtype=np.complex128))


def un(t):
    from paper_2309_15595_amd.api import from_colmajor
    return from_colmajor(t)


def gaussian_hermitian(n, seed):
    rng = np.random.default_rng(seed)
    X = synth.complex_gaussian(rng, (n, n))
    return (X + X.conj().T) / 2


def near_diagonal(n, seed, eps):
    """A late-iteration Rayleigh quotient: the DFT-like spectrum (clusters of
    five 1e-4 wide in [-1, -0.8], the rest spread to 10) in a basis eps away
    from the identity, diagonal in no particular order."""
    rng = np.random.default_rng(seed)
    lam = synth.dft_like_spectrum(max(n, 40))[:n]
    rng.shuffle(lam)
    Q, _ = np.linalg.qr(np.eye(n) + eps * synth.complex_gaussian(rng, (n, n)))
    G = (Q * lam) @ Q.conj().T
    return (G + G.conj().T) / 2


def run(L, G, ldg=None):
    n = G.shape[0]
    ldg = ldg or n
    Gbig = np.full((ldg, n), np.nan + 1j * np.nan)
    Gbig[:n] = np.tril(G)                       # only the lower triangle is read
    Gbig[:n][np.triu_indices(n, 1)] = np.nan + 1j * np.nan
    Gd = cm(Gbig)
    theta, sweeps = L.chase_heev(L.dptr(Gd), ldg, n, L.stream_ptr())
    out = un(Gd)
    return theta, out[:n], out[n:], sweeps


def check(G, theta, X, tag):
    n = G.shape[0]
    lam, Y = np.linalg.eigh(G)
    nrm = max(np.max(np.abs(lam)), 1e-300)
    eig = np.max(np.abs(theta - lam)) / nrm
    res = np.max(np.linalg.norm(G @ X - X * theta, axis=0)) / nrm
    orth = np.linalg.norm(X.conj().T @ X - np.eye(n), 2)
    gap = np.full(n, np.inf)
    if n > 1:
        d = np.diff(lam)
        gap[:-1] = d
        gap[1:] = np.minimum(gap[1:], d)
    sep = gap > 1e-6 * nrm
    ang = np.abs(np.abs(np.sum(X.conj() * Y, axis=0)) - 1.0)
    ang_ok = np.all(ang[sep] <= 1e-13 * nrm / gap[sep] + 1e-13)
    print(f"\n{tag}: n={n} eig {eig:.1e} resid {res:.1e} orth {orth:.1e}", flush=True)
    assert eig <= 1e-13
    assert res <= 1e-13
    assert orth <= 1e-13
    assert ang_ok, float(np.max(ang[sep]))


@pytest.mark.parametrize("n", [1, 2, 17, 33, 80, 300, 1300, 2400])
def test_heev_dense_matches_eigh(L, n):
    print(f"dense n={n}", flush=True)
    G = gaussian_hermitian(n, 7000 + n)
    theta, X, _, sweeps = run(L, G)
    check(G, theta, X, f"dense, {sweeps} sweeps")


@pytest.mark.parametrize("n,eps", [(80, 1e-3), (1300, 1e-6), (1300, 1e-2), (2400, 1e-4)])
def test_heev_near_diagonal_matches_eigh(L, n, eps):
    """The quotients of the later iterations: a few sweeps suffice once the
    basis is within 1e-4 of the eigenvectors (quadratic convergence from the
    first sweep on)."""
    G = near_diagonal(n, 7100 + n, eps)
    theta, X, _, sweeps = run(L, G)
    check(G, theta, X, f"near-diagonal eps={eps:g}, {sweeps} sweeps")
    if eps <= 1e-4:
        assert sweeps <= 4


def test_heev_degenerate_and_real(L):
    """Exactly repeated eigenvalues (multiplicity 10 and 4), real symmetric
    input (the real variant's quotient): real eigenvectors, imaginary parts
    exactly zero."""
    n = 150
    rng = np.random.default_rng(71)
    lam = np.r_[np.full(10, -1.0), np.full(4, 0.5), np.linspace(1.0, 3.0, n - 14)]
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    G = (Q * lam) @ Q.T
    G = (G + G.T) / 2
    theta, X, _, sweeps = run(L, G.astype(np.complex128))
    assert np.all(X.imag == 0.0)
    check(G.astype(np.complex128), theta, X, "degenerate real")


def test_heev_diagonal_and_zero(L):
    """A diagonal G needs no rotation: one sweep, eigenvalues its sorted
    diagonal exactly, eigenvectors the matching unit vectors; the zero matrix
    gives zeros and the identity."""
    d = np.array([3.0, -1.0, 2.0, -1.0, 0.0, 7.5, -4.25])
    theta, X, _, sweeps = run(L, np.diag(d).astype(np.complex128))
    assert sweeps == 1
    order = np.argsort(d, kind="stable")
    assert np.array_equal(theta, d[order])
    assert np.array_equal(X, np.eye(d.size)[:, order])
    theta, X, _, _ = run(L, np.zeros((40, 40), dtype=np.complex128))
    assert np.array_equal(theta, np.zeros(40)) and np.array_equal(X, np.eye(40))


def test_heev_leading_dimension_and_errors(L):
    n, ldg = 45, 61
    G = gaussian_hermitian(n, 9)
    theta, X, pad, _ = run(L, G, ldg=ldg)
    check(G, theta, X, "ldg > n")
    assert np.all(np.isnan(pad.real)) and np.all(np.isnan(pad.imag))   # rows n..ldg-1 untouched
    Gd = cm(np.eye(4))
    with pytest.raises(ValueError):
        L.chase_heev(L.dptr(Gd), 3, 4, L.stream_ptr())
    bad = np.eye(8, dtype=np.complex128)
    bad[5, 2] = np.nan
    Gd = cm(bad)
    with pytest.raises(L.ChaseError):
        L.chase_heev(L.dptr(Gd), 8, 8, L.stream_ptr())
