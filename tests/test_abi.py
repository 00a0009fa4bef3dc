"""CPU checks of the C ABI: the built library loads and exports every entry
point include/chase_hip.h declares; host-only helpers behave."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chase_hip.h")


def declared_functions():
    text = open(HEADER).read()
    return re.findall(r"^\s*(?:int|double|const char\s*\*)\s+(chase_\w+)\s*\(", text, re.M)


def _lib():
    from paper_2309_15595_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libchase_hip.so not built: run python -m paper_2309_15595_amd.build")
    return L


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("chase_default_params", "chase_create", "chase_solve", "chase_destroy",
                 "chase_eigval_grad", "chase_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps every one of them
    assert set(declared_functions()) <= set(L.SIGNATURES)


def test_struct_layouts_match_header():
    L = _lib()
    # chase_params_t: 12 int32 + 7 double + uint64
    assert ctypes.sizeof(L.chase_params_t) == 12 * 4 + 7 * 8 + 8
    # chase_stats_t: 8 int32 + 5 int64 + 7 double + 4 double
    assert ctypes.sizeof(L.chase_stats_t) == 8 * 4 + 5 * 8 + 7 * 8 + 4 * 8


def test_default_params_host_only():
    L = _lib()
    p = L.default_params(nev=60, nex=20)
    assert (p.deg, p.max_deg, p.tol, p.opt, p.max_iter) == (20, 36, 1e-10, 1, 25)


def test_status_strings():
    lib = _lib().load()
    assert lib.chase_status_string(0) == b"ok"
    assert lib.chase_status_string(1).startswith(b"not converged")
    assert lib.chase_status_string(-3) == b"invalid argument"


def test_cond_est_matches_oracle_golden():
    """The library's host CondEst (Alg. 5) on the hand-derived cases."""
    import json
    L = _lib()
    cases = json.load(open(os.path.join(ROOT, "tests", "golden", "condest_cases.json")))["cases"]
    for case in cases:
        ne, locked = 5, 2
        lam = [9.0] * ne
        lam[0] = case["lam_first"]
        lam[locked] = case["lam_active"]
        degs = [case["d"]] * ne
        degs[-1] = case["d_max"]
        got = L.chase_cond_est(lam, case["c"], case["e"], degs, locked)
        assert abs(got - case["expected"]) <= 1e-12 * case["expected"]
    # an estimate beyond the double range is +inf (the shifted branch)
    assert L.chase_cond_est([-1.0, 0.0, 0.5], 1.0, 1e-3, [200, 200, 200], 0) == np.inf


def test_cond_est_any_order_of_active_columns():
    """The mixed-precision solve sorts its active block by rung, then degree.
    Alg. 5 reads the block sorted by degree (ties in ascending Ritz value, the
    order Rayleigh-Ritz leaves): the library's estimate of a rung-sorted
    block equals the oracle's on the degree-sorted one."""
    import oracle.core as oc
    L = _lib()
    rng = np.random.default_rng(5)
    for trial in range(200):
        ne = int(rng.integers(2, 30))
        locked = int(rng.integers(0, ne))
        c, e = 2.0, float(rng.uniform(0.5, 3.0))
        lam = np.sort(rng.uniform(-2.0, 4.0, ne))     # Rayleigh-Ritz order
        degs = rng.choice(np.arange(2, 38, 2), ne)
        # the oracle's block: active columns stable-sorted by degree
        order = np.argsort(degs[locked:], kind="stable")
        lam_d, degs_d = lam.copy(), degs.copy()
        lam_d[locked:] = lam[locked:][order]
        degs_d[locked:] = degs[locked:][order]
        ref = oc.cond_est(lam_d, c, e, degs_d, locked)
        # a two-rung block: a random subset of the active columns first
        rung = rng.integers(0, 2, ne - locked)
        order2 = sorted(range(ne - locked), key=lambda j: (-rung[j], degs[locked + j], j))
        lam_r, degs_r = lam.copy(), degs.copy()
        lam_r[locked:] = lam[locked:][order2]
        degs_r[locked:] = degs[locked:][order2]
        got = L.chase_cond_est(lam_r.tolist(), c, e, degs_r.tolist(), locked)
        if np.isinf(ref):
            assert np.isinf(got)
        else:
            assert abs(got - ref) <= 1e-12 * ref, (trial, got, ref)


def test_workspace_bytes_memory_model():
    """Eq. (2) at p = q = 1 on the host, with no device call.  Eq. (2) counts
    N^2 + 4 N n_e + n_e^2 words; the caller holds H and V (N^2 + N n_e), the
    library C2 and B (2 N n_e), three n_e x n_e matrices plus the 16 split-K
    partials of the n_e x n_e products (19 n_e^2), the block-Jacobi
    eigensolver's working matrix and eigenvector accumulator (2 n_p^2, n_p =
    n_e rounded up to a multiple of 32), a fixed 256 MiB of filter split-K
    tail partials and O(N + n_e) vectors.  Each option adds exactly what it
    documents."""
    L = _lib()
    lib = L.load()
    z = 16
    tail = 256 << 20
    for N, nev, nex in [(20000, 1000, 300), (5000, 200, 60), (1201, 90, 30)]:
        ne = nev + nex
        npad = 32 * -(-ne // 32)
        fp64 = L.chase_workspace_bytes(N, L.default_params(nev=nev, nex=nex), 0)
        core = z * (2 * N * ne + 19 * ne * ne + 2 * npad * npad) + tail
        assert core <= fp64 <= core + z * (64 * N + 128 * ne) + (1 << 20)
        # one N x n_e block fewer than Eq. (2); 18 n_e^2 + 2 n_p^2 words and the tail more
        eq2 = z * (N * N + 4 * N * ne + ne * ne)
        assert z * (N * N + N * ne) + fp64 <= (eq2 - z * N * ne + z * (18 * ne * ne + 2 * npad * npad) + tail
                                               + z * (64 * N + 128 * ne) + (1 << 20))
        fp32 = L.chase_workspace_bytes(N, L.default_params(nev=nev, nex=nex, precision=L.CHASE_FP32_MIXED), 0)
        assert fp32 - fp64 == 8 * N * N + 2 * 8 * N * ne     # complex64 H and two complex64 blocks
        bf16 = L.chase_workspace_bytes(N, L.default_params(nev=nev, nex=nex, precision=L.CHASE_BF16X3_MIXED), 0)
        assert bf16 - fp32 >= 4 * 2 * N * N                  # four bfloat16 planes of H
        c64 = L.chase_workspace_bytes(N, L.default_params(nev=nev, nex=nex), 2)
        assert fp64 < c64 < fp32                             # FP32 blocks, no copy of H
    # real variant: an odd order adds the zero-padded (N+1)^2 copy of H and
    # otherwise sizes like the next even order (same row-pair workspace)
    prm = L.default_params(nev=40, nex=20)
    even = L.chase_workspace_bytes(1002, prm, 1)
    odd = L.chase_workspace_bytes(1001, prm, 1)
    assert odd - even == 8 * 1002 * 1002
    assert even < L.chase_workspace_bytes(1002, prm, 0)
    out = ctypes.c_int64(0)
    assert lib.chase_workspace_bytes(1, ctypes.byref(prm), 0, ctypes.byref(out)) == -1
    assert lib.chase_workspace_bytes(60, ctypes.byref(prm), 0, ctypes.byref(out)) == -2   # nev+nex >= N
    assert lib.chase_workspace_bytes(1000, ctypes.byref(prm), 3, ctypes.byref(out)) == -3
    assert lib.chase_workspace_bytes(1000, ctypes.byref(prm), 0, None) == -4
    import torch
    from paper_2309_15595_amd.api import workspace_bytes
    assert workspace_bytes(1001, 40, 20, dtype=torch.float64) == odd
    bf = L.default_params(nev=40, nex=20, precision=L.CHASE_BF16X3_MIXED)
    assert lib.chase_workspace_bytes(1000, ctypes.byref(bf), 1, ctypes.byref(out)) == -2
    assert lib.chase_workspace_bytes(1000, ctypes.byref(bf), 2, ctypes.byref(out)) == -2


def test_degree_opt_matches_oracle():
    """The library's degree optimisation (the solve's own host routine)
    against the oracle's, integer for integer, over random residuals and
    Ritz values inside and outside the damped interval, including converged,
    non-finite and capped cases."""
    import oracle.core as oc
    L = _lib()
    rng = np.random.default_rng(2309)
    for trial in range(200):
        n = int(rng.integers(1, 40))
        c, e = float(rng.normal()), float(rng.uniform(0.1, 3.0))
        lam = c + e * rng.uniform(-4.0, 1.2, n)
        resd = 10.0 ** rng.uniform(-13, 1, n)
        resd[rng.random(n) < 0.05] = np.inf
        tol = 10.0 ** float(rng.uniform(-12, -6))
        max_deg = int(rng.choice([20, 36, 64]))
        extra = int(rng.integers(0, 4))
        got = L.chase_degree_opt(resd, lam, c, e, tol, max_deg, extra)
        ref = oc.degree_opt(resd, lam, c, e, tol, max_deg, extra)
        assert got == [int(x) for x in ref], (trial, got, list(ref))
    lib = L.load()
    out = (ctypes.c_int32 * 1)()
    one = (ctypes.c_double * 1)(1.0)
    assert lib.chase_degree_opt(None, one, 1, 0.0, 1.0, 1e-10, 36, 2, out) == -1
    assert lib.chase_degree_opt(one, one, 1, 0.0, 0.0, 1e-10, 36, 2, out) == -5
    assert lib.chase_degree_opt(one, one, 1, 0.0, 1.0, 1e-10, 35, 2, out) == -7


def test_invalid_arguments_rejected_on_host():
    """Argument checks run before any device call."""
    L = _lib()
    lib = L.load()
    p = L.default_params(nev=10, nex=5)
    h = ctypes.c_void_p()
    assert lib.chase_create(1, ctypes.byref(p), ctypes.byref(h)) == -1
    assert lib.chase_create(15, ctypes.byref(p), ctypes.byref(h)) == -2   # nev+nex >= N
    bad = L.default_params(nev=10, nex=5, deg=3)
    assert lib.chase_create(100, ctypes.byref(bad), ctypes.byref(h)) == -2
    assert lib.chase_eigval_grad(10, 0, None, 10, None, None, 10, 0, None) == -2
    assert lib.chase_solve_real(None, None, 0, None, 0, 1, None, 0, 0, None, None, None, None) == -1
    assert lib.chase_filter_real(None, 2, None, 2, None, 2, 2, 1, None, 0.0, 1.0, -1.5, None, None) == -1
    assert lib.chase_create_real(1, None, None) == -1
    assert lib.chase_create_c64(1, None, None) == -1
    assert lib.chase_solve_c64(None, None, 0, None, 0, 1, None, 0, 0, None, None, None, None) == -1
    assert lib.chase_set_trace(None, 1) == -1
    assert lib.chase_get_trace(None, None, 0, None) == -1
    assert lib.chase_filter(None, 10, None, 10, None, 10, 10, 1, None, 0.0, 1.0, -1.0, None, None) == -1
    assert lib.chase_caqr_real(None, 10, 10, 2, 1.0, -1, None, None) == -1
    assert lib.chase_filter_lowp(None, 10, None, 10, 10, 1, None, 0.0, 1.0, -1.0, 1, None, None) == -1
    assert lib.chase_get_trace_columns(None, 1, None, 0, None) == -1
    assert np.isnan(L.chase_cond_est([1.0], 0.0, 0.0, [2], 0))


def test_struct_sizes_match_c_compiler(tmp_path):
    """sizeof of the C structs (compiled from the header with the host C
    compiler) equals the ctypes mirrors."""
    import shutil
    import subprocess
    L = _lib()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "chase_hip.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(chase_params_t), sizeof(chase_stats_t),'
                   ' sizeof(chase_trace_t), sizeof(chase_trace_column_t));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(L.chase_params_t)
    assert int(out[1]) == ctypes.sizeof(L.chase_stats_t)
    assert int(out[2]) == ctypes.sizeof(L.chase_trace_t)
    assert int(out[3]) == ctypes.sizeof(L.chase_trace_column_t)


def _build_c_example(out_path):
    """Compile and link tests/native/c_abi_solve.c (plain C99, no torch)
    against the in-tree library with the host C compiler."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if cc is None or not os.path.isdir(os.path.join(rocm, "include", "hip")):
        pytest.skip("no host C compiler or HIP headers")
    libdir = os.path.join(ROOT, "paper_2309_15595_amd")
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(rocm, "include"), "-D__HIP_PLATFORM_AMD__",
           os.path.join(ROOT, "tests", "native", "c_abi_solve.c"), "-L", libdir, "-lchase_hip",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm", f"-Wl,-rpath,{libdir}",
           f"-Wl,-rpath,{os.path.join(rocm, 'lib')}", "-o", str(out_path)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out_path


def test_c_example_builds_against_the_abi(tmp_path):
    """The header and the library serve a plain C caller: the example builds
    warning-free with -Wall -Wextra and links against libchase_hip.so."""
    _lib().load()
    exe = _build_c_example(tmp_path / "c_abi_solve")
    assert exe.exists()
