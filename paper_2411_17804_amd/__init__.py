"""MI355X-native EPIC direct imager: gfx950 HIP kernels behind the C ABI of
include/epic.h, with a thin ctypes binding in ``epic``."""
from . import epic  # noqa: F401
