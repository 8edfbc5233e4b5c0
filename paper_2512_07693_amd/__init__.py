"""MI355X-native conservative adaptive-precision EAM/ACE energies and forces (HIP, gfx950).

The compute path is libap.so (C ABI in include/ap.h); `ap` is its thin ctypes binding.
"""
from . import ap  # noqa: F401
from .ap import Context, APError  # noqa: F401
