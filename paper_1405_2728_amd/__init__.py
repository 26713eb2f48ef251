"""MI355X (gfx950) finite-difference micromagnetic energy minimiser.

Hot path of Abert et al., arXiv:1405.2728: midpoint projected-gradient
iteration with Barzilai-Borwein step sizes, whose cost is the effective field
(FFT demag convolution plus exchange, anisotropy and Zeeman terms).  All
arithmetic runs in the HIP library libmmbb.so (C ABI in include/mm.h); this
package only loads it and marshals arguments.
"""

from .api import Context, MMError, supported  # noqa: F401
