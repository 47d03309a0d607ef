"""vsr: visual-sphere perspective-map rasterization on AMD Instinct MI355X.

The compute path is the HIP library ``libvsr.so`` (sources in ``csrc/``,
C ABI in ``include/vsr.h``); ``vsr`` is its ctypes binding and ``pipeline``
holds the device-buffer plumbing.  Submodules are imported on demand so
that importing the package never touches the GPU.
"""
__all__ = ["vsr", "pipeline", "build"]

from .build import build  # noqa: E402  (compiles libvsr.so; no GPU needed)
