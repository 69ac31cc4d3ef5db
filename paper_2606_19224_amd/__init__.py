"""MI355X-native CGD-EnKF analysis (HIP for gfx950 behind a C ABI).

The library `libcgd_enkf.so` (built by `paper_2606_19224_amd.build`) holds
every kernel; `paper_2606_19224_amd.binding` marshals torch tensors into its
C entry points.  There is no CPU fallback: without the built library on a
GPU machine the binding raises.
"""
__version__ = "0.1.0"
