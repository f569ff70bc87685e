"""MI355X-native SU(2) pure-gauge heat bath (Cardoso & Bicudo, "Lattice SU(2)
on GPU's") and the SU(3) heat bath built on it through SU(2) subgroups.  The
compute path is libsu2.so (HIP kernels for gfx950 behind the C ABI of
include/su2.h and include/su3.h); this package is its Python binding."""
from .su2 import *  # noqa: F401,F403
from .su2 import NN, Batch, Lattice, Lattice64, SU2Error, lib, header_functions  # noqa: F401
from .su3 import Batch3, Lattice3, header_functions3, lib3  # noqa: F401
