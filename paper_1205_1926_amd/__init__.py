"""MI355X (gfx950) TFETI semismooth-Newton solver for elastoplasticity.

The method (Cermak, Kozubek, Sysala, Valdman) runs in the HIP library
libtfeti.so behind the C ABI of include/tfeti.h; this package only marshals
arguments (ctypes) and uses torch for device memory and streams.
"""

from ._capi import TfetiError, load  # noqa: F401
from .solver import GpuSolver, model_host, return_map  # noqa: F401
