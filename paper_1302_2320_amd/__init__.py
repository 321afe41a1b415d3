"""MI355X implementation of the micromagnetic-ensemble Wang-Landau method
(B. D. Stosic, arXiv:1302.2320): independent flat-histogram walks, one or more
per fixed-magnetisation line of an L x L periodic Ising lattice, run by HIP
kernels behind the C ABI of include/wl.h.

``wl`` is the ctypes binding of libwl.so; ``workloads`` builds the line sets of
the benchmark configurations.
"""
from . import wl  # noqa: F401
from .wl import Batch, LineParams, assemble, line_run, line_run_ex  # noqa: F401
