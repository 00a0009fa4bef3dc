"""GPU: the batched solve (grouped filter launch replayed from a HIP graph)
and the mixed-precision solve, against single-problem solves and the oracle."""
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
    return colmajor(np.asarray(x, dtype=np.complex128))


def un(t):
    from paper_2309_15595_amd.api import from_colmajor
    return from_colmajor(t)


def batch_problems(Ns, seed0=2309000):
    probs = []
    for i, N in enumerate(Ns):
        nev, nex = max(2, N // 20), max(2, N // 80)
        probs.append(synth.make_problem(N, nev, nex, spectrum="dft", basis="gaussian",
                                        seed=seed0 + i, seed_v0=seed0 + 100 + i,
                                        seed_lanczos=seed0 + 200 + i))
    return probs


def single(p):
    from paper_2309_15595_amd.api import Solver
    with Solver(p.N, p.nev, p.nex) as s:
        Vd = cm(p.V0)
        ritz, resid, info = s.solve_colmajor(cm(p.A), Vd, True, cm(p.starts))
    return ritz, resid, un(Vd)[:, : p.nev], info


@pytest.mark.parametrize("Ns", [[300, 517, 800, 256, 640, 1000], [450]])
def test_batched_matches_single_and_oracle(L, Ns):
    from paper_2309_15595_amd.api import solve_batched
    probs = batch_problems(Ns)
    A_cms = [cm(p.A) for p in probs]
    V_cms = [cm(p.V0) for p in probs]
    S_cms = [cm(p.starts) for p in probs]
    ritz, resid, stats, st = solve_batched(A_cms, V_cms, [p.nev for p in probs],
                                           [p.nex for p in probs], S_cms)
    assert st == 0
    iters = []
    for i, p in enumerate(probs):
        r1, res1, X1, info1 = single(p)
        X = un(V_cms[i])[:, : p.nev]
        # same kernels, same data, same decisions: identical results
        assert np.max(np.abs(ritz[i] - r1)) <= 1e-13 * p.norm2
        assert stats[i]["iterations"] == info1.stats["iterations"]
        assert stats[i]["filter_matvecs"] == info1.stats["filter_matvecs"]
        assert np.max(np.abs(ritz[i] - p.lam[: p.nev])) <= 1e-10 * p.norm2
        r_true = np.linalg.norm(p.A @ X - X * ritz[i], axis=0)
        assert np.max(r_true) <= 1e-10 * p.norm2 * (1 + 1e-6)
        assert np.linalg.norm(X.conj().T @ X - np.eye(p.nev), 2) <= 1e-12
        iters.append(stats[i]["iterations"])
    if len(Ns) > 1:
        # the oracle on one member of the batch
        p = probs[0]
        ref = oc.chase(p.A, oc.Params(nev=p.nev, nex=p.nex), V0=p.V0, starts=p.starts)
        assert np.max(np.abs(ritz[0] - ref.evals)) <= 1e-10 * p.norm2
    print("iterations per problem:", iters)


def test_batched_rejects_mixed_precision(L):
    from paper_2309_15595_amd.api import solve_batched
    p = batch_problems([200])[0]
    with pytest.raises(ValueError):
        solve_batched([cm(p.A)], [cm(p.V0)], [p.nev], [p.nex], precision=L.CHASE_FP32_MIXED)


# ---------------------------------------------------------------- mixed precision

@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("N,nev,nex,spectrum", [(800, 60, 20, "uniform"), (1200, 60, 15, "dft"),
                                                (517, 40, 12, "uniform")])   # odd order: staged FP32 step
def test_mixed_precision_reaches_fp64_accuracy(L, N, nev, nex, spectrum, prec):
    from paper_2309_15595_amd.api import Solver
    p = synth.make_problem(N, nev, nex, spectrum=spectrum, basis="gaussian", seed=N + 7)
    code = L.CHASE_FP32_MIXED if prec == "fp32" else L.CHASE_BF16X3_MIXED
    with Solver(N, nev, nex, precision=code) as s:
        Vd = cm(p.V0)
        ritz, resid, info = s.solve_colmajor(cm(p.A), Vd, True, cm(p.starts))
    assert info.converged, info.stats
    X = un(Vd)[:, :nev]
    ref = oc.chase(p.A, oc.Params(nev=nev, nex=nex), V0=p.V0, starts=p.starts)
    err = np.abs(ritz - ref.evals) / p.norm2
    st = info.stats
    print(f"\nmixed {prec}: max per-eigenpair |d lambda|/||A|| vs FP64 oracle = {err.max():.2e}; "
          f"MatVec shares FP32 {st['filter_matvecs_fp32'] / st['filter_matvecs']:.2f}, "
          f"BF16x3 {st['filter_matvecs_bf16'] / st['filter_matvecs']:.2f}")
    assert err.max() <= 1e-10
    assert st["filter_matvecs_fp32"] > 0
    if prec == "bf16x3":
        assert st["filter_matvecs_bf16"] > 0
    r_true = np.linalg.norm(p.A @ X - X * ritz, axis=0)
    assert np.max(r_true) <= 1e-10 * p.norm2 * (1 + 1e-6)
    assert np.linalg.norm(X.conj().T @ X - np.eye(nev), 2) <= 1e-12


# ---------------------------------------------------------------- autotuner

def test_autotuned_single_solve_matches(L):
    """autotune = 1 times the tile-shape candidates per size class; the
    choice changes only the summation order, so eigenpairs stay within
    rounding of the default solve and of the oracle."""
    from paper_2309_15595_amd.api import Solver
    p = synth.make_problem(900, 40, 12, spectrum="dft", basis="gaussian", seed=77)
    out = []
    for tune in (0, 1, 1):       # second tuned solve reuses the tuned table
        with Solver(p.N, p.nev, p.nex, autotune=tune) as s:
            Vd = cm(p.V0)
            ritz, resid, info = s.solve_colmajor(cm(p.A), Vd, True, cm(p.starts))
        assert info.converged
        out.append(ritz)
    assert np.max(np.abs(out[1] - out[0])) <= 1e-12 * p.norm2
    assert np.max(np.abs(out[2] - out[1])) <= 1e-12 * p.norm2
    assert np.max(np.abs(out[1] - p.lam[: p.nev])) <= 1e-10 * p.norm2


def test_autotuned_batched_matches(L):
    from paper_2309_15595_amd.api import solve_batched
    probs = batch_problems([300, 700, 520])
    res = []
    for tune in (0, 1):
        V_cms = [cm(p.V0) for p in probs]
        ritz, resid, stats, st = solve_batched([cm(p.A) for p in probs], V_cms,
                                               [p.nev for p in probs], [p.nex for p in probs],
                                               [cm(p.starts) for p in probs], autotune=tune)
        assert st == 0
        res.append(ritz)
    for i, p in enumerate(probs):
        assert np.max(np.abs(res[1][i] - res[0][i])) <= 1e-12 * p.norm2
        assert np.max(np.abs(res[1][i] - p.lam[: p.nev])) <= 1e-10 * p.norm2
