"""MI355X (gfx950) ChASE hot path: Chebyshev-filtered subspace iteration for
the lowest eigenpairs of dense Hermitian matrices (arXiv 2309.15595).

The compute path is libchase_hip.so (hand-written HIP kernels behind the C
ABI of include/chase_hip.h); this package is its thin Python binding.
"""
from ._lib import load, LIB_PATH, ChaseError  # noqa: F401


def __getattr__(name):
    # torch-dependent surface, imported on first use
    if name in ("eigsh", "eigvalsh_lowest", "ChaseEigvals", "Solver", "colmajor",
                "from_colmajor", "solve_batched"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
