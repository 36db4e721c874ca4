"""MI355X-native soft-sphere DEM hot path (Lethe-DEM, arXiv 2106.09576).

The simulation runs in HIP kernels for gfx950 inside ``libdem.so`` (C ABI in
``include/dem.h``); ``paper_2106_09576_amd.dem`` is its ctypes binding.
"""
from .dem import Dem, DemError, load_library  # noqa: F401
