"""MI355X-native per-cell reaction-network burn (FP64 BDF in HIP for gfx950).

The HIP kernels and their C ABI live in libburn.so (include/burn.h); this
package holds the ctypes binding (``burn``), the build step (``build``) and
the seeded synthetic inputs (``synth``).
"""

__all__ = ["synth", "build"]
