"""MI355X-native solver for the nonlocal Davey-Stewartson potential.

Phi = F^-1[-kx^2/|k|^2 rho_hat] split as in Mauser, Stimming, Zhang (Sec. 2.1):
a zero-padded FFT for the high frequencies and a polar quadrature whose
grid-to-node and node-to-grid sums are a type-2 and a type-1 NUFFT.  The
computation lives in a C-ABI library of hand-written HIP kernels
(include/phi_solve.h, built into lib/libphisolve.so); this package is the thin
Python binding.
"""
from .solver import (  # noqa: F401
    Plan,
    BatchPlan,
    PhiSolve,
    phi_solve,
    describe,
    make_params,
    host_gauss_legendre,
    host_es_kernel,
    host_es_transform,
    host_polar_nodes,
)
from .stepper import DSStepper, DSEvolve, ds_evolve  # noqa: F401
from ._binding import PhiError, LIB_PATH  # noqa: F401
