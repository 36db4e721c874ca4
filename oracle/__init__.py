"""Plain FP64 CPU oracle of the Lethe-DEM time step (arXiv 2106.09576, Secs. 2-3).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the GPU
library and its binding) never imports it, and it imports nothing from them.
"""
from .binding import (OracleSim, build_oracle, oracle_from_scene, oracle_lib_path,  # noqa: F401
                      triangle_closest)
