"""MI355X (gfx950) Toeplitz spatio-angular MMSE tomographic reconstructor.

The product is the HIP library libtt.so behind the C ABI of include/tt.h; this
package holds its sources (csrc/), the build script (build.py) and a thin
ctypes binding (tt.py).  See tt.Context for the Python entry points.
"""
from . import tt  # noqa: F401
from .tt import Context, Kernels, Learned, TTError, load, matvec_batch, solve_batch, system_from  # noqa: F401

__all__ = ["tt", "Context", "Kernels", "Learned", "TTError", "system_from", "load"]
