"""Plain FP64 CPU reference of the VMAT column-generation hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never calls it, shares no code with it, and must not fall back to it.

Everything is NumPy float64 (D's float32 values are promoted exactly).  The
functions follow the paper's model and algorithm in its own order and
notation: eq. 1 (voxel penalty), eq. 2 (dose-rate smoothing), eq. 3 (the
model and its dose constraint), Sec. 2.2 (column generation: KKT prices,
per-row left-to-right aperture search, one aperture per beam, gradient
projection master).  Readings of what the paper leaves open are listed in
the module docstrings of ``vmat_oracle``.
"""
from .vmat_oracle import *  # noqa: F401,F403
