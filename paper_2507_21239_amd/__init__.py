"""MI355X (gfx950) implementation of the representative-particle collision step
of mcdust (arXiv 2507.21239): adaptive equal-count binning, per-cell rate
matrices, cumulative-rate event selection with Philox4x32-10, sticking /
erosion / fragmentation, and transport -- HIP kernels behind the C ABI in
include/mcd.h.

Submodules: ``api`` (torch front end, needs the built libmcd.so), ``_lib``
(ctypes declarations), ``workloads`` (seeded synthetic inputs), ``build``.
"""

__all__ = ["api", "workloads", "build"]
