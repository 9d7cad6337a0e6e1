"""MI355X-native latent time step of Continuous Reduced-Order Modeling
(CROM): HIP kernels for gfx950 behind the C interface include/crom.h, and a
thin ctypes binding (``crom``)."""
from . import crom  # noqa: F401
from .crom import Decoder, GNOptions, Stepper  # noqa: F401
