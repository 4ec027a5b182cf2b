"""MI355X-native particle-by-particle VMC hot path (QMCPACK overview paper, arXiv:1802.06922).

The compute path is the HIP library ``_lib/libqmc.so`` (C ABI in ``include/qmc.h``);
``qmc`` is its ctypes binding.
"""
from .qmc import (Batch, QMCError, System, estimate_device_bytes, load_library, KERNEL_GATHER,  # noqa: F401
                  KERNEL_CHAIN, KERNEL_MEASURE, KERNEL_REBUILD)

__all__ = ["Batch", "QMCError", "System", "estimate_device_bytes", "load_library", "KERNEL_GATHER",
           "KERNEL_CHAIN", "KERNEL_MEASURE", "KERNEL_REBUILD"]
