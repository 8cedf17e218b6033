"""MI355X-native BDDC-preconditioned CG for divergence-free VEM Stokes.

The hot path lives in the HIP library ``libvembddc.so`` (sources in
``csrc/``, C-ABI in ``include/vembddc.h``); ``binding`` is its ctypes
binding.
"""
from . import binding  # noqa: F401
