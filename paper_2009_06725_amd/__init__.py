"""MI355X (gfx950) spectral complex-valued Stokes solver: HIP library + ctypes binding."""
from . import scvs  # noqa: F401
