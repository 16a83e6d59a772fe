"""MI355X-native hybrid lattice-Boltzmann / finite-difference solver for
chemically driven self-propelled droplets (Fadda et al., arXiv:1711.10984).

The timestep runs in hand-written HIP kernels for gfx950 behind a C ABI
(``include/lbm.h``); :mod:`paper_1711_10984_amd.lbm` is the thin Python
binding.  :mod:`paper_1711_10984_amd.workloads` builds seeded initial states.
"""
__all__ = ["lbm", "workloads"]
