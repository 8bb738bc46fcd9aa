"""sqc: cut-circuit reconstruction (ScaleQC, arXiv 2207.00933) on AMD Instinct
MI355X.  The compute runs in ``libsqc.so`` (hand-written HIP for gfx950,
C interface in ``include/sqc.h``); ``sqc`` is its ctypes binding and
``runner`` drives whole workloads through it."""
