"""MI355X-native hot path of local-expansion-move stereo (Taniai et al.,
arXiv 1603.08328): a HIP library for gfx950 behind the C ABI in
include/lexp.h, with a ctypes binding in :mod:`paper_1603_08328_amd.lexp`."""
from . import lexp  # noqa: F401
