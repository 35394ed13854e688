"""MI355X-native SBR trace-integrate path (arXiv 2604.09243).

The computation lives in ``libsbr.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/sbr.h``); ``sbr`` is its ctypes binding.
"""
from . import sbr  # noqa: F401
from .sbr import Context, BVH, SbrError, plan_angle, load_library  # noqa: F401
