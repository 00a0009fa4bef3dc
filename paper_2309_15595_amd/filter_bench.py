"""Time one Chebyshev filter call (Eq. 1, every column to the same degree) on
the N = 20000 DFT-like workload, in FP64 (chase_filter), FP32 or BF16x3
(chase_filter_lowp), for kernel profiling:

    python -m paper_2309_15595_amd.filter_bench --precision bf16x3 --n 1300 --deg 4

Prints one line per call (wall time, MatVecs, algorithmic TFLOP/s).  The
low-precision calls include their per-call set-up (the planes or the
complex64 copy of H), so profile the kernel itself (bfilter_step,
cfilter_step_dma, zfilter_step) with rocprofv3.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3"], default="fp64")
    ap.add_argument("--N", type=int, default=20000)
    ap.add_argument("--n", type=int, default=1300, help="columns")
    ap.add_argument("--deg", type=int, default=4, help="even degree of every column")
    ap.add_argument("--calls", type=int, default=2)
    args = ap.parse_args()
    import numpy as np
    import torch

    import synth
    from synth import problems as sp
    from paper_2309_15595_amd import _lib as L

    L.load()
    N, n = args.N, args.n
    lam = synth.dft_like_spectrum(N)
    A = sp.hermitian_from_spectrum_torch(lam, seed=sp.SEED_Q, device="cuda")
    V0 = torch.from_numpy(np.ascontiguousarray(
        synth.complex_gaussian(np.random.default_rng(sp.SEED_V0), (N, n)).T)).cuda()
    W = torch.empty_like(V0)
    c, e, mu1 = 4.6, 5.4, float(lam[0])   # damped interval [-0.8, 10], normalised at lambda_1
    degs = [args.deg] * n
    for i in range(args.calls):
        V = V0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if args.precision == "fp64":
            mv = L.chase_filter(L.dptr(A), N, L.dptr(V), N, L.dptr(W), N, N, n, degs, c, e, mu1, L.stream_ptr())
        else:
            code = L.CHASE_FP32_MIXED if args.precision == "fp32" else L.CHASE_BF16X3_MIXED
            mv = L.chase_filter_lowp(L.dptr(A), N, L.dptr(V), N, N, n, degs, c, e, mu1, code, L.stream_ptr())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"{args.precision} N={N} n={n} deg={args.deg}: {dt * 1e3:.2f} ms, {mv} MatVecs, "
              f"{8.0 * N * N * mv / dt / 1e12:.1f} TFLOP/s algorithmic (call {i})", flush=True)


if __name__ == "__main__":
    main()
