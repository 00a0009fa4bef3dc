"""ctypes binding of libchase_hip.so: the C ABI of include/chase_hip.h.

Argument marshalling only.  Loading fails loudly when the library has not
been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchase_hip.so")

CHASE_FP64 = 0
CHASE_FP32_MIXED = 1
CHASE_BF16X3_MIXED = 2
CHASE_QR_AUTO = -1
CHASE_QR_CHOLQR1 = 0
CHASE_QR_CHOLQR2 = 1
CHASE_QR_SHIFTED = 2
CHASE_QR_HOUSEHOLDER = 3


class chase_params_t(C.Structure):
    _fields_ = [
        ("nev", C.c_int32), ("nex", C.c_int32), ("deg", C.c_int32), ("max_deg", C.c_int32),
        ("deg_extra", C.c_int32), ("max_iter", C.c_int32), ("opt", C.c_int32),
        ("precision", C.c_int32), ("lanczos_steps", C.c_int32), ("force_qr", C.c_int32),
        ("bounds_given", C.c_int32), ("autotune", C.c_int32),
        ("tol", C.c_double), ("b_sup", C.c_double), ("mu_1", C.c_double), ("mu_ne", C.c_double),
        ("norm_est", C.c_double), ("mixed_switch", C.c_double), ("bf16_switch", C.c_double),
        ("seed", C.c_uint64),
    ]


class chase_stats_t(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("iterations", C.c_int32), ("locked", C.c_int32),
        ("qr_count", C.c_int32 * 4), ("eig_sweeps", C.c_int32),
        ("filter_matvecs", C.c_int64), ("filter_matvecs_fp32", C.c_int64),
        ("filter_matvecs_bf16", C.c_int64),
        ("total_matvecs", C.c_int64), ("filter_launches", C.c_int64),
        ("filter_flops", C.c_double), ("t_total", C.c_double), ("t_lanczos", C.c_double),
        ("t_filter", C.c_double), ("t_qr", C.c_double), ("t_rr", C.c_double),
        ("t_resid", C.c_double), ("bounds", C.c_double * 4),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}
        d["qr_count"] = list(self.qr_count)
        d["bounds"] = list(self.bounds)
        return d


class chase_trace_t(C.Structure):
    _fields_ = [
        ("iteration", C.c_int32), ("locked", C.c_int32), ("n_active", C.c_int32),
        ("qr_variant", C.c_int32), ("filter_matvecs", C.c_int64), ("kappa_est", C.c_double),
        ("kappa_com", C.c_double), ("kappa_com_active", C.c_double), ("kappa_com_equil", C.c_double),
        ("t_filter", C.c_double), ("t_qr", C.c_double), ("t_rr", C.c_double),
        ("eig_sweeps", C.c_int32), ("pad0", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}


class chase_trace_column_t(C.Structure):
    _fields_ = [
        ("origin", C.c_int32), ("rung", C.c_int32), ("degree", C.c_int32), ("pad0", C.c_int32),
        ("ritz", C.c_double), ("resid", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}


CHASE_TRACE_MAX = 256

_I64, _I32, _D, _P = C.c_int64, C.c_int32, C.c_double, C.c_void_p
_DP = C.POINTER(C.c_double)
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)

SIGNATURES = {
    "chase_default_params": (C.c_int, [C.POINTER(chase_params_t)]),
    "chase_create": (C.c_int, [_I64, C.POINTER(chase_params_t), C.POINTER(_P)]),
    "chase_workspace_bytes": (C.c_int, [_I64, C.POINTER(chase_params_t), _I32, C.POINTER(_I64)]),
    "chase_solve": (C.c_int, [_P, _P, _I64, _P, _I64, _I32, _P, _I64, _I32, _DP, _DP,
                              C.POINTER(chase_stats_t), _P]),
    "chase_destroy": (C.c_int, [_P]),
    "chase_solve_batched": (C.c_int, [_I32, _I64P, C.POINTER(_P), _I64P, C.POINTER(_P), _I64P,
                                      _I32P, C.POINTER(_P), _I64P, _I32P,
                                      C.POINTER(chase_params_t), C.POINTER(_DP), C.POINTER(_DP),
                                      C.POINTER(chase_stats_t), _P]),
    "chase_eigval_grad": (C.c_int, [_I64, _I32, _P, _I64, _P, _P, _I64, _I32, _P]),
    "chase_filter": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _I64, _I64, _I32P, _D, _D, _D,
                               _I64P, _P]),
    "chase_filter_noalloc": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _I64, _I64, _I32P, _D, _D, _D,
                                       _I64P, _P]),
    "chase_filter_noalloc_scratch_bytes": (_I64, []),
    "chase_caqr": (C.c_int, [_P, _I64, _I64, _I64, _D, _I32, _I32P, _P]),
    "chase_caqr_real": (C.c_int, [_P, _I64, _I64, _I64, _D, _I32, _I32P, _P]),
    "chase_filter_lowp": (C.c_int, [_P, _I64, _P, _I64, _I64, _I64, _I32P, _D, _D, _D, _I32,
                                    _I64P, _P]),
    "chase_rayleigh_ritz": (C.c_int, [_P, _I64, _P, _I64, _I64, _I64, _DP, _DP, _P]),
    "chase_heev": (C.c_int, [_P, _I64, _I64, _DP, _I32P, _P]),
    "chase_lanczos": (C.c_int, [_P, _I64, _I64, _P, _I64, _I32, _I32, _I32, _DP, _P]),
    "chase_cond_est": (C.c_double, [_DP, _D, _D, _I32P, _I32, _I32]),
    "chase_degree_opt": (C.c_int, [_DP, _DP, _I32, _D, _D, _D, _I32, _I32, _I32P]),
    "chase_create_real": (C.c_int, [_I64, C.POINTER(chase_params_t), C.POINTER(_P)]),
    "chase_solve_real": (C.c_int, [_P, _P, _I64, _P, _I64, _I32, _P, _I64, _I32, _DP, _DP,
                                   C.POINTER(chase_stats_t), _P]),
    "chase_filter_real": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _I64, _I64, _I32P, _D, _D, _D,
                                    _I64P, _P]),
    "chase_create_c64": (C.c_int, [_I64, C.POINTER(chase_params_t), C.POINTER(_P)]),
    "chase_solve_c64": (C.c_int, [_P, _P, _I64, _P, _I64, _I32, _P, _I64, _I32, _DP, _DP,
                                  C.POINTER(chase_stats_t), _P]),
    "chase_set_trace": (C.c_int, [_P, _I32]),
    "chase_get_trace": (C.c_int, [_P, C.POINTER(chase_trace_t), _I32, _I32P]),
    "chase_get_trace_columns": (C.c_int, [_P, _I32, C.POINTER(chase_trace_column_t), _I32, _I32P]),
    "chase_status_string": (C.c_char_p, [C.c_int]),
    "chase_last_error": (C.c_char_p, []),
}

_lib = None


class ChaseError(RuntimeError):
    pass


def load():
    """Load libchase_hip.so (built in-tree by paper_2309_15595_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2309_15595_amd.build` "
                          "(the GPU path has no fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str, allow_not_converged: bool = False) -> int:
    if status == 0 or (allow_not_converged and status == 1):
        return status
    lib = load()
    msg = lib.chase_status_string(status).decode()
    detail = lib.chase_last_error().decode()
    if status < 0:
        raise ValueError(f"{what}: argument {-status} invalid ({msg})")
    raise ChaseError(f"{what}: status {status} ({msg}) {detail}")


def default_params(**kw) -> chase_params_t:
    p = chase_params_t()
    load().chase_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def dptr(x) -> int:
    """Device pointer of a torch tensor (0 for None)."""
    return 0 if x is None else int(x.data_ptr())


def stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def f64_array(n: int):
    return (C.c_double * n)()


# ---- thin wrappers with the C names ----------------------------------------

def chase_create(N: int, params: chase_params_t):
    h = _P()
    check(load().chase_create(N, C.byref(params), C.byref(h)), "chase_create")
    return h


def chase_create_real(N: int, params: chase_params_t):
    h = _P()
    check(load().chase_create_real(N, C.byref(params), C.byref(h)), "chase_create_real")
    return h


def chase_solve_real(h, A_ptr, lda, V_ptr, ldv, use_v0, starts_ptr, ld_starts, nstarts, nev, stream):
    ritz = f64_array(nev)
    resid = f64_array(nev)
    stats = chase_stats_t()
    st = load().chase_solve_real(h, A_ptr, lda, V_ptr, ldv, use_v0, starts_ptr or None, ld_starts,
                                 nstarts, ritz, resid, C.byref(stats), stream)
    check(st, "chase_solve_real", allow_not_converged=True)
    return list(ritz), list(resid), stats


def chase_workspace_bytes(N: int, params: chase_params_t, variant: int = 0) -> int:
    """Device bytes a handle of this order and params allocates (host only)."""
    out = _I64(0)
    check(load().chase_workspace_bytes(N, C.byref(params), variant, C.byref(out)), "chase_workspace_bytes")
    return out.value


def chase_create_c64(N: int, params: chase_params_t):
    h = _P()
    check(load().chase_create_c64(N, C.byref(params), C.byref(h)), "chase_create_c64")
    return h


def chase_solve_c64(h, A_ptr, lda, V_ptr, ldv, use_v0, starts_ptr, ld_starts, nstarts, nev, stream):
    ritz = f64_array(nev)
    resid = f64_array(nev)
    stats = chase_stats_t()
    st = load().chase_solve_c64(h, A_ptr, lda, V_ptr, ldv, use_v0, starts_ptr or None, ld_starts,
                                nstarts, ritz, resid, C.byref(stats), stream)
    check(st, "chase_solve_c64", allow_not_converged=True)
    return list(ritz), list(resid), stats


def chase_filter_real(A_ptr, lda, V_ptr, ldv, W_ptr, ldw, N, n, degs, c, e, mu_1, stream) -> int:
    d = (C.c_int32 * n)(*[int(x) for x in degs])
    mv = C.c_int64(0)
    check(load().chase_filter_real(A_ptr, lda, V_ptr, ldv, W_ptr, ldw, N, n, d, c, e, mu_1,
                                   C.byref(mv), stream), "chase_filter_real")
    return mv.value


def chase_destroy(h) -> None:
    check(load().chase_destroy(h), "chase_destroy")


def chase_solve(h, A_ptr, lda, V_ptr, ldv, use_v0, starts_ptr, ld_starts, nstarts, nev, stream):
    ritz = f64_array(nev)
    resid = f64_array(nev)
    stats = chase_stats_t()
    st = load().chase_solve(h, A_ptr, lda, V_ptr, ldv, use_v0, starts_ptr or None, ld_starts,
                            nstarts, ritz, resid, C.byref(stats), stream)
    check(st, "chase_solve", allow_not_converged=True)
    return list(ritz), list(resid), stats


def chase_solve_batched(Ns, A_ptrs, ldas, V_ptrs, ldvs, use_v0, start_ptrs, ld_starts, nstarts,
                        params, stream):
    """Arrays over problems; returns (ritz lists, resid lists, stats list, status)."""
    cnt = len(Ns)
    arr = lambda T, xs: (T * cnt)(*xs)
    ritz = [f64_array(p.nev) for p in params]
    resid = [f64_array(p.nev) for p in params]
    stats = (chase_stats_t * cnt)()
    st = load().chase_solve_batched(
        cnt, arr(C.c_int64, Ns), arr(_P, A_ptrs), arr(C.c_int64, ldas), arr(_P, V_ptrs),
        arr(C.c_int64, ldvs), arr(C.c_int32, use_v0), arr(_P, [p or None for p in start_ptrs]),
        arr(C.c_int64, ld_starts), arr(C.c_int32, nstarts), arr(chase_params_t, params),
        arr(_DP, [C.cast(r, _DP) for r in ritz]), arr(_DP, [C.cast(r, _DP) for r in resid]),
        stats, stream)
    check(st, "chase_solve_batched", allow_not_converged=True)
    return [list(r) for r in ritz], [list(r) for r in resid], list(stats), st


def chase_eigval_grad(N, nev, X_ptr, ldx, g_ptr, G_ptr, ldg, fill, stream) -> None:
    check(load().chase_eigval_grad(N, nev, X_ptr, ldx, g_ptr, G_ptr, ldg, fill, stream),
          "chase_eigval_grad")


def chase_filter(A_ptr, lda, V_ptr, ldv, W_ptr, ldw, N, n, degs, c, e, mu_1, stream) -> int:
    d = (C.c_int32 * n)(*[int(x) for x in degs])
    mv = C.c_int64(0)
    check(load().chase_filter(A_ptr, lda, V_ptr, ldv, W_ptr, ldw, N, n, d, c, e, mu_1,
                              C.byref(mv), stream), "chase_filter")
    return mv.value


def chase_filter_noalloc(A_ptr, lda, V_ptr, ldv, W_ptr, ldw, N, n, degs, c, e, mu_1, stream) -> int:
    """chase_filter on the library's fixed device scratch: allocates nothing
    and returns once the work is enqueued on `stream`."""
    d = (C.c_int32 * max(1, n))(*[int(x) for x in degs])
    mv = C.c_int64(0)
    check(load().chase_filter_noalloc(A_ptr, lda, V_ptr, ldv, W_ptr, ldw, N, n, d, c, e, mu_1,
                                      C.byref(mv), stream), "chase_filter_noalloc")
    return mv.value


def chase_heev(G_ptr, ldg, n, stream):
    """Eigenvalues (ascending, numpy array) and the number of Jacobi sweeps;
    the eigenvectors are written over G."""
    import numpy as np
    theta = np.zeros(n, dtype=np.float64)
    sw = C.c_int32(0)
    check(load().chase_heev(G_ptr, ldg, n, theta.ctypes.data_as(_DP), C.byref(sw), stream), "chase_heev")
    return theta, sw.value


def chase_caqr(V_ptr, ldv, N, n, cond, force, stream) -> int:
    v = C.c_int32(-1)
    check(load().chase_caqr(V_ptr, ldv, N, n, cond, force, C.byref(v), stream), "chase_caqr")
    return v.value


def chase_caqr_real(V_ptr, ldv, N, n, cond, force, stream) -> int:
    v = C.c_int32(-1)
    check(load().chase_caqr_real(V_ptr, ldv, N, n, cond, force, C.byref(v), stream), "chase_caqr_real")
    return v.value


def chase_filter_lowp(A_ptr, lda, V_ptr, ldv, N, n, degs, c, e, mu_1, precision, stream) -> int:
    d = (C.c_int32 * n)(*[int(x) for x in degs])
    mv = C.c_int64(0)
    check(load().chase_filter_lowp(A_ptr, lda, V_ptr, ldv, N, n, d, c, e, mu_1, precision,
                                   C.byref(mv), stream), "chase_filter_lowp")
    return mv.value


def chase_rayleigh_ritz(A_ptr, lda, Q_ptr, ldq, N, n, stream):
    th = f64_array(n)
    rs = f64_array(n)
    check(load().chase_rayleigh_ritz(A_ptr, lda, Q_ptr, ldq, N, n, th, rs, stream),
          "chase_rayleigh_ritz")
    return list(th), list(rs)


def chase_lanczos(A_ptr, lda, N, starts_ptr, ld_starts, nstarts, ksteps, ne, stream):
    out = f64_array(4)
    check(load().chase_lanczos(A_ptr, lda, N, starts_ptr, ld_starts, nstarts, ksteps, ne, out,
                               stream), "chase_lanczos")
    return tuple(out)


def chase_degree_opt(resd, lam, c, e, tol_abs, max_deg, extra):
    n = len(resd)
    rs = (C.c_double * n)(*[float(x) for x in resd])
    la = (C.c_double * n)(*[float(x) for x in lam])
    out = (C.c_int32 * n)()
    check(load().chase_degree_opt(rs, la, n, c, e, tol_abs, max_deg, extra, out), "chase_degree_opt")
    return [int(x) for x in out]


def chase_cond_est(lam, c, e, degs, locked) -> float:
    n = len(lam)
    la = (C.c_double * n)(*lam)
    dg = (C.c_int32 * n)(*[int(x) for x in degs])
    return load().chase_cond_est(la, c, e, dg, n, locked)
