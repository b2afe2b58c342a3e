"""MI355X bundle adjustment: LM over SE(3) cameras and 3D points with an explicit
Schur complement and block-Jacobi PCG, in HIP kernels for gfx950 behind a C-ABI.

``paper_2510_15271_amd.ba`` is the ctypes binding of ``libba_mi355x.so``;
``paper_2510_15271_amd.build_lib`` builds it.
"""
from . import ba  # noqa: F401
