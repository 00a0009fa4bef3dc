"""FP64 CPU oracle of ChASE's hot path (arXiv 2309.15595, Alg. 1-5, Eq. 1).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package's smoke
check and by the benchmark's CPU-baseline leg, never by the GPU library.
It shares no code with the GPU path.
"""
from .core import *  # noqa: F401,F403
from .core import Params, Result, chase  # noqa: F401
