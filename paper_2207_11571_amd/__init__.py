"""MI355X-native hot path of the corrected DGSEM method of arXiv 2207.11571.

The DG residual, Runge-Kutta stepping, forcing network (inference and
training), filter and the solve server all run in ``libdgnn.so``, hand-written
HIP for gfx950 (``csrc/``), behind the C ABI of ``include/dgnn.h``.
``binding`` is its ctypes binding; build the library with
``python -m paper_2207_11571_amd.build``.
"""
