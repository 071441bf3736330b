"""MI355X (gfx950) HIP implementation of the column-generation VMAT hot path.

``vmat`` is the Python binding of the C ABI (include/vmat.h); ``build`` compiles
libvmat.so in-tree.
"""
from . import vmat  # noqa: F401
from .vmat import Problem, VmatError, master_opts  # noqa: F401
from .autograd import aperture_cost, fluence_cost  # noqa: F401
