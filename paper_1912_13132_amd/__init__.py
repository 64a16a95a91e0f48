"""MI355X-native parallel cross-validation for Gaussian-process models.

The compute path lives in the shared library built from ``csrc/`` and is
reached through ``paper_1912_13132_amd.pcv`` (ctypes binding, loaded on
first use).  ``workloads`` and ``partition`` are host-side input preparation.
"""
__all__ = ["pcv", "workloads", "partition"]
