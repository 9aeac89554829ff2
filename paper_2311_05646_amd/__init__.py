"""MI355X-native shape-parameter gradients (AutoDiffGeo hot path).

The compute path is the C-ABI library ``libshapegrad.so`` built from
``csrc/`` (HIP kernels for gfx950); ``api`` is a thin ctypes binding over it.
Importing this package does not load the library; ``api`` does, and raises
if it is missing.
"""
__all__ = ["workloads", "api"]
