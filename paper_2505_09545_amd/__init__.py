"""MI355X-native hot path of the Green's Dyadic Method (arXiv:2505.09545).

The compute lives in libgdm.so (HIP kernels for gfx950 behind the C-ABI of
include/gdm.h); ``paper_2505_09545_amd.gdm`` is its thin ctypes binding."""
__all__ = ["gdm"]
