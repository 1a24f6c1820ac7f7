"""MI355X-native Wilson-fermion HMC hot path: libhmc (HIP, gfx950) and its binding."""
from . import hmc  # noqa: F401
