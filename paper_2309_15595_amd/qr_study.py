"""One-GPU versions of the paper's two QR experiments (Sec. 4.2 and 4.3).

  * Condition numbers (the comparison of Fig. 1): every iteration's estimate
    from Alg. 5 beside exact condition numbers (singular values) of the block 1D-CAQR
    receives, of its filtered columns alone and of the block with unit
    columns, with and without degree optimisation.
  * QR variants (the comparison of Table 2): time to solution, QR time,
    iterations and MatVecs with the CondEst-driven choice of Alg. 4 and with
    each variant forced, the blocked Householder QR included.

The workload is the synthetic Hermitian problem of the filter benchmark
(complex128, a spectrum shaped like a DFT Hamiltonian's, Gaussian random
start); one JSON document goes to --out and a summary to stdout.

    python -m paper_2309_15595_amd.qr_study --N 20000 --nev 1000 --nex 300 --out qr.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

VARIANTS = {"auto": -1, "cholqr2": 1, "shifted_cholqr2": 2, "householder": 3}
QR_NAMES = {0: "CholQR1", 1: "CholQR2", 2: "sCholQR2", 3: "HHQR"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=20000)
    ap.add_argument("--nev", type=int, default=1000)
    ap.add_argument("--nex", type=int, default=300)
    ap.add_argument("--out", default=None)
    ap.add_argument("--skip-kappa", action="store_true", help="only the QR-variant comparison")
    ap.add_argument("--skip-variants", action="store_true", help="only the condition numbers")
    args = ap.parse_args(argv)

    import torch

    import synth
    from synth import problems as sp
    from paper_2309_15595_amd import _lib as L
    from paper_2309_15595_amd.api import Solver

    L.load()
    N, nev, nex = args.N, args.nev, args.nex
    ne = nev + nex
    dev = torch.device("cuda:0")
    lam = synth.dft_like_spectrum(N)
    A = sp.hermitian_from_spectrum_torch(lam, seed=sp.SEED_Q, device=dev)
    V0 = torch.from_numpy(np.ascontiguousarray(
        synth.complex_gaussian(np.random.default_rng(sp.SEED_V0), (N, ne)).T)).to(dev)
    S = torch.from_numpy(np.ascontiguousarray(
        synth.complex_gaussian(np.random.default_rng(sp.SEED_LANCZOS), (N, 4)).T)).to(dev)
    V = torch.empty_like(V0)
    normA = float(np.max(np.abs(lam)))
    torch.cuda.synchronize()
    out = {"workload": {"N": N, "nev": nev, "nex": nex, "spectrum": "dft-like", "deg": 20, "max_deg": 36,
                        "tol": 1e-10}}

    def run(solver, level):
        solver.set_trace(level)
        V.copy_(V0)
        ritz, resid, info = solver.solve_colmajor(A, V, True, S)
        return ritz, resid, info, solver.trace()

    if not args.skip_kappa:
        out["kappa"] = {}
        for opt in (0, 1):
            with Solver(N, nev, nex, deg=20, max_deg=36, opt=opt, tol=1e-10) as s:
                t0 = time.perf_counter()
                ritz, _, info, tr = run(s, 2)
                dt = time.perf_counter() - t0
            name = "opt" if opt else "no-opt"
            out["kappa"][name] = {"converged": bool(info.converged), "iterations": info.stats["iterations"],
                                  "trace": tr}
            print(f"condition numbers, {name} ({dt:.1f} s with the singular values):", flush=True)
            print("  it  locked   kappa_est   com:whole   com:active   com:equil  est/active  QR", flush=True)
            for t in tr:
                ratio = t["kappa_est"] / t["kappa_com_active"]
                print(f"  {t['iteration']:2d}  {t['locked']:5d}  {t['kappa_est']:10.3e}  {t['kappa_com']:10.3e}  "
                      f"{t['kappa_com_active']:10.3e}  {t['kappa_com_equil']:10.3e}  {ratio:9.3g}  "
                      f"{QR_NAMES.get(t['qr_variant'], '?')}", flush=True)

    if not args.skip_variants:
        out["variants"] = {}
        ref = None
        for name, force in VARIANTS.items():
            with Solver(N, nev, nex, deg=20, max_deg=36, opt=1, tol=1e-10, force_qr=force) as s:
                run(s, 1)  # warm-up (library set-up, plans)
                ritz, resid, info, tr = run(s, 1)
            st = info.stats
            if ref is None:
                ref = ritz
            rec = {"converged": bool(info.converged), "iterations": st["iterations"],
                   "filter_matvecs": st["filter_matvecs"], "t_total": st["t_total"], "t_qr": st["t_qr"],
                   "t_filter": st["t_filter"], "t_rr": st["t_rr"], "qr_count": st["qr_count"],
                   "qr_ms_per_call": [t["t_qr"] * 1e3 for t in tr],
                   "max_abs_eig_err_over_normA": float(np.max(np.abs(ritz - lam[:nev])) / normA),
                   "max_abs_diff_vs_auto_over_normA": float(np.max(np.abs(ritz - ref)) / normA)}
            out["variants"][name] = rec
            print(f"{name:16s} conv {rec['converged']}  iters {rec['iterations']:2d}  "
                  f"matvecs {rec['filter_matvecs']:8d}  total {rec['t_total']:7.3f} s  "
                  f"QR {rec['t_qr']:7.3f} s  err {rec['max_abs_eig_err_over_normA']:.2e}  "
                  f"qr_count {rec['qr_count']}", flush=True)

    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1, default=float)
    return 0


if __name__ == "__main__":
    sys.exit(main())
