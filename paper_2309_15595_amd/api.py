"""Python surface of the ChASE library: eigsh, an autograd eigenvalue op and
column-major helpers.  PyTorch provides device memory and streams only;
every step of the solve runs in libchase_hip.so.

Layout.  The library is column-major.  A row-major torch tensor T viewed
column-major is T^T, which for a Hermitian matrix is conj(T).  ``eigsh``
therefore hands A's memory over untouched, solves conj(A) (same
eigenvalues) and conjugates the returned vectors; no N^2 transpose is made.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib

_PRECISIONS = {"fp64": _lib.CHASE_FP64, "fp32": _lib.CHASE_FP32_MIXED,
               "mixed": _lib.CHASE_FP32_MIXED, "bf16x3": _lib.CHASE_BF16X3_MIXED}


def colmajor(x, device="cuda") -> torch.Tensor:
    """(rows x cols) array -> device tensor of shape (cols, rows) whose memory
    is the column-major layout of x (leading dimension = rows)."""
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    return x.transpose(-2, -1).contiguous().to(device)


def from_colmajor(t: torch.Tensor) -> np.ndarray:
    """Inverse of colmajor: (cols, rows) device tensor -> numpy (rows x cols)."""
    return t.detach().cpu().numpy().T.copy()


@dataclasses.dataclass
class SolveInfo:
    converged: bool
    status: int
    stats: dict


_VARIANTS = {torch.complex128: 0, torch.float64: 1, torch.complex64: 2}


def workspace_bytes(N: int, nev: int, nex: int, *, dtype=torch.complex128, **params) -> int:
    """Device bytes a Solver of these arguments allocates (host-side count;
    H and the block are the caller's and not included)."""
    if dtype not in _VARIANTS:
        raise TypeError(f"unsupported dtype {dtype}")
    return _lib.chase_workspace_bytes(N, _lib.default_params(nev=nev, nex=nex, **params), _VARIANTS[dtype])


class Solver:
    """A chase_create/chase_destroy handle for problems of order N."""

    _KINDS = {torch.complex128: (_lib.chase_create, _lib.chase_solve),
              torch.float64: (_lib.chase_create_real, _lib.chase_solve_real),
              torch.complex64: (_lib.chase_create_c64, _lib.chase_solve_c64)}

    def __init__(self, N: int, nev: int, nex: int, *, dtype=torch.complex128, **params):
        """dtype: complex128 (Hermitian), float64 (real symmetric,
        chase_create_real) or complex64 (chase_create_c64)."""
        if dtype not in self._KINDS:
            raise TypeError(f"unsupported dtype {dtype}")
        self.N, self.nev, self.nex, self.dtype = N, nev, nex, dtype
        self.params = _lib.default_params(nev=nev, nex=nex, **params)
        create, self._solve = self._KINDS[dtype]
        self.h = create(N, self.params)

    def close(self):
        if self.h is not None:
            _lib.chase_destroy(self.h)
            self.h = None

    def set_trace(self, level: int):
        """Record a per-iteration trace of the following solves (level 1), with
        the exact condition number of each filtered block (level 2)."""
        _lib.check(_lib.load().chase_set_trace(self.h, int(level)), "chase_set_trace")

    def trace(self):
        """Per-iteration records of the last traced solve, as dicts."""
        import ctypes
        buf = (_lib.chase_trace_t * _lib.CHASE_TRACE_MAX)()
        n = ctypes.c_int32(0)
        _lib.check(_lib.load().chase_get_trace(self.h, buf, _lib.CHASE_TRACE_MAX, ctypes.byref(n)),
                   "chase_get_trace")
        return [buf[i].as_dict() for i in range(n.value)]

    def trace_columns(self, iteration: int):
        """The active columns of a traced iteration (1-based), in filter order:
        dicts of origin (ascending-Ritz-value rank in the previous iteration),
        rung (0 FP64, 1 FP32, 2 BF16x3), degree, ritz and resid."""
        import ctypes
        cap = self.nev + self.nex
        buf = (_lib.chase_trace_column_t * cap)()
        n = ctypes.c_int32(0)
        _lib.check(_lib.load().chase_get_trace_columns(self.h, int(iteration), buf, cap, ctypes.byref(n)),
                   "chase_get_trace_columns")
        return [buf[i].as_dict() for i in range(n.value)]

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_colmajor(self, A_cm: torch.Tensor, V_cm: torch.Tensor, use_v0: bool = True,
                       starts_cm: Optional[torch.Tensor] = None, stream=None):
        """A_cm: (N, N) tensor holding A column-major; V_cm: (n_e, N) tensor
        holding the N x n_e block column-major (in/out)."""
        N = self.N
        dt = self.dtype
        _check_dev(A_cm, (N, N), dt)
        _check_dev(V_cm, (self.nev + self.nex, N), dt)
        ns = 0 if starts_cm is None else starts_cm.shape[0]
        if starts_cm is not None:
            _check_dev(starts_cm, (ns, N), dt)
        ritz, resid, stats = self._solve(
            self.h, _lib.dptr(A_cm), N, _lib.dptr(V_cm), N, int(use_v0), _lib.dptr(starts_cm),
            N, ns, self.nev, _lib.stream_ptr(stream))
        return np.array(ritz), np.array(resid), SolveInfo(stats.status == 0, stats.status,
                                                          stats.as_dict())


def solve_batched(A_cms, V_cms, nevs, nexs, starts_cms=None, stream=None, **params):
    """Solve many Hermitian problems of uneven N together (grouped filter).

    A_cms[i]: (N_i, N_i) column-major H_i; V_cms[i]: (n_e_i, N_i) initial
    blocks (in/out); starts_cms[i]: optional (r_i, N_i).  Returns lists of
    (ritz values, residuals) and per-problem stats dicts, and the status.
    """
    n = len(A_cms)
    Ns = [int(a.shape[0]) for a in A_cms]
    for i in range(n):
        _check_dev(A_cms[i], (Ns[i], Ns[i]))
        _check_dev(V_cms[i], (nevs[i] + nexs[i], Ns[i]))
    starts_cms = starts_cms or [None] * n
    plist = [_lib.default_params(nev=nevs[i], nex=nexs[i], **params) for i in range(n)]
    ritz, resid, stats, st = _lib.chase_solve_batched(
        Ns, [_lib.dptr(a) for a in A_cms], Ns, [_lib.dptr(v) for v in V_cms], Ns, [1] * n,
        [_lib.dptr(s) for s in starts_cms], Ns,
        [0 if s is None else int(s.shape[0]) for s in starts_cms], plist, _lib.stream_ptr(stream))
    return ([np.array(r) for r in ritz], [np.array(r) for r in resid],
            [s.as_dict() for s in stats], st)


def _check_dev(t: torch.Tensor, shape, dtype=torch.complex128):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"expected a contiguous tensor of shape {shape}, got {tuple(t.shape)}")


def eigsh(A: torch.Tensor, nev: int, nex: int, *, deg: int = 20, tol: float = 1e-10,
          opt: bool = True, max_deg: int = 36, max_iter: int = 25, V0=None, starts=None,
          precision: str = "fp64", seed: int = 2309, return_raw: bool = False):
    """nev lowest eigenpairs of the Hermitian (N, N) complex128 CUDA tensor A,
    of the real symmetric float64 one (then the real path, real vectors), or
    of a complex64 one (H used in place: FP32 filter and H Q products, the
    rest in FP64; residuals bottom out near sqrt(N) 2^-24 ||H||, so pass a
    tol such as 1e-5).

    Returns (evals (nev,) float64 tensor, evecs (N, nev) tensor of A's dtype,
    SolveInfo).  V0 (N, nev+nex) optional initial block, starts (N, r)
    optional Lanczos start vectors, both of A's dtype.
    """
    N = A.shape[0]
    ne = nev + nex
    if A.dtype == torch.complex64:
        if precision != "fp64":
            raise ValueError("the complex64 path fixes its own precisions (FP32 products, FP64 elsewhere)")
        _check_dev(A, (N, N), torch.complex64)
        with Solver(N, nev, nex, dtype=torch.complex64, deg=deg, tol=tol, opt=int(opt), max_deg=max_deg,
                    max_iter=max_iter, seed=seed) as s:
            # as for complex128: A's memory read column-major is conj(A)
            if V0 is not None:
                Vt = V0.conj().transpose(0, 1).contiguous()
            else:
                Vt = torch.empty((ne, N), dtype=torch.complex64, device=A.device)
            st = None if starts is None else starts.conj().transpose(0, 1).contiguous()
            ritz, resid, info = s.solve_colmajor(A, Vt, use_v0=V0 is not None, starts_cm=st)
        info.stats["resid"] = resid
        evals = torch.from_numpy(ritz).to(A.device)
        evecs = Vt[:nev].transpose(0, 1).conj()
        if return_raw:
            return evals, evecs, info, Vt
        return evals, evecs, info
    if A.dtype == torch.float64:
        if precision != "fp64":
            raise ValueError("the real symmetric path is FP64 only")
        _check_dev(A, (N, N), torch.float64)
        with Solver(N, nev, nex, dtype=torch.float64, deg=deg, tol=tol, opt=int(opt), max_deg=max_deg,
                    max_iter=max_iter, seed=seed) as s:
            # symmetric: the row-major memory is the column-major matrix
            if V0 is not None:
                Vt = V0.transpose(0, 1).contiguous()
            else:
                Vt = torch.empty((ne, N), dtype=torch.float64, device=A.device)
            st = None if starts is None else starts.transpose(0, 1).contiguous()
            ritz, resid, info = s.solve_colmajor(A, Vt, use_v0=V0 is not None, starts_cm=st)
        info.stats["resid"] = resid
        evals = torch.from_numpy(ritz).to(A.device)
        evecs = Vt[:nev].transpose(0, 1)
        if return_raw:
            return evals, evecs, info, Vt
        return evals, evecs, info
    _check_dev(A, (N, N))
    with Solver(N, nev, nex, deg=deg, tol=tol, opt=int(opt), max_deg=max_deg,
                max_iter=max_iter, precision=_PRECISIONS[precision], seed=seed) as s:
        # A's memory read column-major is conj(A): start from conj(V0) to stay
        # on the same iterates, conjugate the eigenvectors back at the end.
        if V0 is not None:
            Vt = V0.conj().transpose(0, 1).contiguous()
        else:
            Vt = torch.empty((ne, N), dtype=torch.complex128, device=A.device)
        st = None if starts is None else starts.conj().transpose(0, 1).contiguous()
        ritz, resid, info = s.solve_colmajor(A, Vt, use_v0=V0 is not None, starts_cm=st)
    evals = torch.from_numpy(ritz).to(A.device)
    evecs = Vt[:nev].transpose(0, 1).conj()
    info.stats["resid"] = resid
    if return_raw:
        return evals, evecs, info, Vt
    return evals, evecs, info


class ChaseEigvals(torch.autograd.Function):
    """Lowest nev eigenvalues of Hermitian A with dL/dA = X diag(g) X^H
    (Hellmann-Feynman); the backward recomputes nothing from the filter."""

    @staticmethod
    def forward(ctx, A, nev, nex, kwargs):
        evals, _, info, Vt = eigsh(A, nev, nex, return_raw=True, **(kwargs or {}))
        if not info.converged:
            raise RuntimeError(f"ChASE did not converge (status {info.status})")
        ctx.save_for_backward(Vt)
        ctx.nev = nev
        ctx.N = A.shape[0]
        return evals

    @staticmethod
    def backward(ctx, g):
        (Vt,) = ctx.saved_tensors
        N, nev = ctx.N, ctx.nev
        g = g.to(torch.float64).contiguous()
        G = torch.empty((N, N), dtype=torch.complex128, device=Vt.device)
        # Vt holds conj(X) column-major; the column-major product
        # conj(X) diag(g) X^T read row-major is X diag(g) X^H.
        _lib.chase_eigval_grad(N, nev, _lib.dptr(Vt), N, _lib.dptr(g), _lib.dptr(G), N, 0,
                               _lib.stream_ptr())
        return G, None, None, None


def eigvalsh_lowest(A: torch.Tensor, nev: int, nex: int, **kwargs) -> torch.Tensor:
    """Differentiable lowest-nev eigenvalues (see ChaseEigvals)."""
    return ChaseEigvals.apply(A, nev, nex, kwargs)
