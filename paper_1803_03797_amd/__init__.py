"""MI355X (gfx950) stencil conjugate-gradient library.

Solves A x = b for the unscaled 5-point Laplacian on an nx-by-ny grid with zero
Dirichlet boundary (arXiv 1803.03797, Section II) by classic CG (Algorithm 1)
or the pipelined CG (Algorithm 2), with hand-written HIP kernels behind the C
ABI of include/cg.h.  `cg` is the ctypes binding; `workloads` draws the
seeded synthetic inputs.
"""
from . import cg  # noqa: F401
from .cg import Context, load  # noqa: F401
