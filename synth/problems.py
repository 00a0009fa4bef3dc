"""Seeded Hermitian eigenproblems with a prescribed spectrum.

The paper benchmarks on artificial matrices built from a diagonal matrix of
prescribed eigenvalues rotated by the Q factor of the QR factorisation of a
random square matrix (Numerical Experiments, "Artificial Matrices"), with
eigenvalues spread uniformly over an interval.  In the complex Hermitian case
the rotation is A = Q diag(lam) Q^H.  Two rotations are provided:

* ``gaussian``: Q is the unitary factor of numpy's QR of a seeded complex
  Gaussian matrix, exactly the paper's recipe (cost O(N^3), used for N up to a
  few thousand).
* ``fourier``: Q = F diag(phi) F with F the unitary DFT and phi seeded random
  phases.  Q is dense and unitary, A is formed with two FFT sweeps in
  O(N^2 log N), which makes N = 20000 .. 50000 matrices cheap to build on the
  device.  Subspace iteration started from Gaussian blocks behaves the same in
  distribution for every unitary Q (a Gaussian block rotated by Q^H is again
  Gaussian), so the rotation only changes rounding, not convergence.

Random numbers the eigensolver itself draws (its initial block and the
Lanczos start vectors) are drawn here too and handed to both the oracle and
the GPU library as inputs.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

SEED_Q = 2309        # rotation / spectrum
SEED_V0 = 2310       # initial block
SEED_LANCZOS = 2311  # Lanczos start vectors
SEED_W = 2312        # loss weights of the eigenvalue-gradient workload


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """(x + i y)/sqrt(2) with x, y standard normal: unit variance per entry."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def uniform_spectrum(N: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Eigenvalues equispaced over [lo, hi] (the paper's "Uniform" matrices)."""
    return np.linspace(lo, hi, N)


def dft_like_spectrum(N: int) -> np.ndarray:
    """Spectrum shaped like a DFT Hamiltonian: a clustered low end, a wide tail.

    The lowest 5 % of the N eigenvalues fall in [-1, -0.8], grouped into
    min(n_low, 200) clusters whose centres are 0.2/n_cl apart (1e-3 when there
    are 200 clusters); the members of one cluster are spread evenly over a
    width of 1e-4 around its centre.  The remaining eigenvalues are equispaced
    in (-0.8, 10].  All values are distinct and returned ascending.
    """
    n_low = int(round(0.05 * N))
    parts = []
    if n_low > 0:
        n_cl = min(n_low, 200)
        sizes = np.full(n_cl, n_low // n_cl)
        sizes[: n_low % n_cl] += 1
        for k in range(n_cl):
            centre = -1.0 + (k + 0.5) * 0.2 / n_cl
            m = int(sizes[k])
            if m == 1:
                parts.append(np.array([centre]))
            else:
                parts.append(centre + np.linspace(-0.5e-4, 0.5e-4, m))
    n_high = N - n_low
    # equispaced in (-0.8, 10]: drop the left end point
    parts.append(np.linspace(-0.8, 10.0, n_high + 1)[1:])
    lam = np.concatenate(parts)
    return np.sort(lam)


def gaussian_unitary(N: int, rng: np.random.Generator) -> np.ndarray:
    """Unitary Q factor of numpy's QR of an N x N complex Gaussian matrix."""
    G = complex_gaussian(rng, (N, N))
    Q, _ = np.linalg.qr(G)
    return Q


def _hermitise_np(A: np.ndarray) -> np.ndarray:
    return 0.5 * (A + A.conj().T)


def hermitian_from_spectrum(lam: np.ndarray, basis: str = "gaussian",
                            seed: int = SEED_Q) -> np.ndarray:
    """Dense Hermitian A with eigenvalues ``lam`` (numpy, complex128, C order)."""
    lam = np.asarray(lam, dtype=np.float64)
    N = lam.shape[0]
    rng = np.random.default_rng(seed)
    if basis == "gaussian":
        Q = gaussian_unitary(N, rng)
        A = (Q * lam[None, :]) @ Q.conj().T
    elif basis == "fourier":
        phi = np.exp(2j * np.pi * rng.random(N))
        A = _fourier_rotate_np(lam, phi)
    else:
        raise ValueError(f"unknown basis {basis!r}")
    return _hermitise_np(A)


def real_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """Standard normal float64 entries."""
    return rng.standard_normal(shape)


def symmetric_from_spectrum(lam: np.ndarray, seed: int = SEED_Q) -> np.ndarray:
    """Dense real symmetric A = Q diag(lam) Q^T, Q the orthogonal factor of
    numpy's QR of a seeded real Gaussian matrix (float64, C order)."""
    lam = np.asarray(lam, dtype=np.float64)
    N = lam.shape[0]
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((N, N)))
    A = (Q * lam[None, :]) @ Q.T
    return 0.5 * (A + A.T)


def symmetric_from_spectrum_torch(lam: np.ndarray, seed: int = SEED_Q, device="cuda"):
    """Dense real symmetric matrix with eigenvalues ``lam`` built on a torch
    device: Q = C^T diag(s) C with C the orthonormal DCT-II matrix and s
    seeded random signs (dense and orthogonal; three N^3 products).  Returns
    a (N, N) float64 tensor, symmetric, so row- and column-major agree."""
    import torch

    lam = np.asarray(lam, dtype=np.float64)
    N = lam.shape[0]
    s = torch.from_numpy(np.where(np.random.default_rng(seed).random(N) < 0.5, -1.0, 1.0)).to(device)
    k = torch.arange(N, dtype=torch.float64, device=device)
    C = torch.cos(torch.pi * (2.0 * k[None, :] + 1.0) * k[:, None] / (2.0 * N)) * (2.0 / N) ** 0.5
    C[0] *= 0.5 ** 0.5
    B = (C.T * torch.from_numpy(lam).to(device)[None, :]) @ C      # C^T diag(lam) C
    B *= s[:, None] * s[None, :]                                   # S (.) S
    A = C.T @ (B @ C)                                              # C^T (.) C
    del B, C
    A += A.T.clone()
    A *= 0.5
    return A


def _circulant_first_column(lam: np.ndarray) -> np.ndarray:
    # With the unitary DFT F (F_jk = exp(-2 pi i j k / N) / sqrt(N)),
    # F diag(lam) F^H is circulant: entry (j, k) is fft(lam)[(j - k) mod N] / N.
    return np.fft.fft(lam) / lam.shape[0]


def _fourier_rotate_np(lam: np.ndarray, phi: np.ndarray) -> np.ndarray:
    N = lam.shape[0]
    c = _circulant_first_column(lam)
    j = np.arange(N)
    M = c[(j[:, None] - j[None, :]) % N]          # F diag(lam) F^H
    M = phi[:, None] * M * phi.conj()[None, :]     # diag(phi) (.) diag(phi)^H
    M = np.fft.fft(M, axis=0, norm="ortho")        # F (.)
    M = np.fft.ifft(M, axis=1, norm="ortho")       # (.) F^H
    return M


def hermitian_from_spectrum_torch(lam: np.ndarray, seed: int = SEED_Q,
                                  device="cuda", chunk: int = 1024):
    """Fourier-rotated Hermitian matrix built on a torch device.

    Returns a (N, N) complex128 torch tensor T with T[i, j] = A[i, j] in
    row-major order.  Peak memory is about two N x N complex128 buffers.
    """
    import torch

    lam = np.asarray(lam, dtype=np.float64)
    N = lam.shape[0]
    rng = np.random.default_rng(seed)
    phi_np = np.exp(2j * np.pi * rng.random(N))
    c = torch.from_numpy(_circulant_first_column(lam)).to(device)
    phi = torch.from_numpy(phi_np).to(device)
    rows = torch.arange(N, device=device)
    if N <= 16384:
        # the same steps on whole matrices, the two unitary DFTs as products
        # with the explicit DFT matrix (a transform length per problem would
        # each cost the FFT library a kernel build); a few N^2 buffers
        jk = torch.remainder(rows[:, None] * rows[None, :], N).to(torch.float64)
        F = torch.polar(torch.full_like(jk, 1.0 / np.sqrt(N)), jk * (-2.0 * np.pi / N))
        del jk
        M = c[torch.remainder(rows[:, None] - rows[None, :], N)] * phi[:, None] * phi.conj()[None, :]
        M = (F @ M) @ F.conj()
        del F
        return M.add_(M.conj().T.contiguous()).mul_(0.5)
    out = torch.empty((N, N), dtype=torch.complex128, device=device)
    # column blocks: M[:, blk] -> F M[:, blk] (FFT along rows index)
    for k0 in range(0, N, chunk):
        k1 = min(N, k0 + chunk)
        cols = torch.arange(k0, k1, device=device)
        idx = torch.remainder(rows[:, None] - cols[None, :], N)
        blk = c[idx] * phi[:, None] * phi[k0:k1].conj()[None, :]
        out[:, k0:k1] = torch.fft.fft(blk, dim=0, norm="ortho")
        del idx, blk
    # row blocks: X[blk, :] -> X[blk, :] F^H
    for r0 in range(0, N, chunk):
        r1 = min(N, r0 + chunk)
        out[r0:r1, :] = torch.fft.ifft(out[r0:r1, :], dim=1, norm="ortho")
    # Hermitise in place, tile pairs (i, j) and (j, i) together
    for r0 in range(0, N, chunk):
        r1 = min(N, r0 + chunk)
        for k0 in range(r0, N, chunk):
            k1 = min(N, k0 + chunk)
            a = out[r0:r1, k0:k1]
            b = out[k0:k1, r0:r1]
            h = 0.5 * (a + b.conj().T)
            out[r0:r1, k0:k1] = h
            out[k0:k1, r0:r1] = h.conj().T
    return out


@dataclasses.dataclass
class Problem:
    """One seeded eigenproblem: matrix, prescribed spectrum, solver inputs."""
    name: str
    N: int
    nev: int
    nex: int
    lam: np.ndarray                  # prescribed eigenvalues, ascending
    A: Optional[np.ndarray]          # host matrix (None when built on device)
    V0: np.ndarray                   # N x (nev+nex) complex Gaussian block
    starts: np.ndarray               # N x 4 complex Gaussian Lanczos starts
    deg: int = 20
    tol: float = 1e-10

    @property
    def ne(self) -> int:
        return self.nev + self.nex

    @property
    def norm2(self) -> float:
        return float(np.max(np.abs(self.lam)))


def make_problem(N: int, nev: int, nex: int, spectrum: str = "uniform",
                 basis: str = "gaussian", seed: int = SEED_Q,
                 seed_v0: int = SEED_V0, seed_lanczos: int = SEED_LANCZOS,
                 n_starts: int = 4, build_matrix: bool = True,
                 name: Optional[str] = None, deg: int = 20,
                 tol: float = 1e-10, real: bool = False) -> Problem:
    """real=True: a real symmetric matrix (Gaussian orthogonal rotation) with
    real Gaussian initial block and Lanczos starts."""
    if real:
        if spectrum not in ("uniform", "dft"):
            raise ValueError(f"unknown spectrum {spectrum!r}")
        lam = uniform_spectrum(N) if spectrum == "uniform" else dft_like_spectrum(N)
        A = symmetric_from_spectrum(lam, seed=seed) if build_matrix else None
        V0 = real_gaussian(np.random.default_rng(seed_v0), (N, nev + nex))
        starts = real_gaussian(np.random.default_rng(seed_lanczos), (N, n_starts))
        return Problem(name=name or f"{spectrum}-real-N{N}", N=N, nev=nev, nex=nex,
                       lam=lam, A=A, V0=V0, starts=starts, deg=deg, tol=tol)
    if spectrum == "uniform":
        lam = uniform_spectrum(N)
    elif spectrum == "dft":
        lam = dft_like_spectrum(N)
    else:
        raise ValueError(f"unknown spectrum {spectrum!r}")
    A = hermitian_from_spectrum(lam, basis=basis, seed=seed) if build_matrix else None
    V0 = complex_gaussian(np.random.default_rng(seed_v0), (N, nev + nex))
    starts = complex_gaussian(np.random.default_rng(seed_lanczos), (N, n_starts))
    return Problem(name=name or f"{spectrum}-{basis}-N{N}", N=N, nev=nev, nex=nex,
                   lam=lam, A=A, V0=V0, starts=starts, deg=deg, tol=tol)


# The small workload the oracle solves in seconds: N = 800 complex Hermitian,
# eigenvalues equispaced in [-1, 1], Gaussian-QR rotation, nev 60, nex 20,
# degree 20, tolerance 1e-10, random initial block.
CFG_PARITY = dict(N=800, nev=60, nex=20, spectrum="uniform", basis="gaussian",
                  deg=20, tol=1e-10)


def loss_weights(nev: int, seed: int = SEED_W) -> np.ndarray:
    """w_i ~ U(0, 1), weights of the eigenvalue loss sum_i w_i lambda_i."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, nev)
