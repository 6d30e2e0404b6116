"""lesjet on MI355X: explicit LES residual and RK5 step of the filtered
compressible Navier-Stokes equations (arXiv 2301.00817) as hand-written HIP
kernels behind a C-ABI (include/lesjet.h).

The compiled library is required: importing `binding` or `solver` without
`_lib/liblesjet.so` raises; there is no CPU fallback.
"""
__all__ = ["binding", "solver"]
