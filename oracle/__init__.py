"""FP64 CPU oracle of the hybrid LB + finite-difference timestep.

Test infrastructure only: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may use it; the HIP product path never does.
"""
from .oracle import OracleSim, Params, Drop, grad9, lap9, div9, STAGES, load, num_threads  # noqa: F401
