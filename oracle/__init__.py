"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct NumPy implementation of what the potential
solver computes, written from the paper (Mauser, Stimming, Zhang; Sec. 2.1 and
Sec. 3.1).  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it.  It shares no code, tables or constants with the GPU library,
and the GPU library never calls it: the product path fails when its HIP
library is missing instead of falling back here.

Modules
  split_solver  the split quadrature by direct sums: I1 (padded DFT), polar rule,
                type-2 / type-1 direct sums, Phi, literal transpose
  closed_forms  exact potentials that pin the oracle (Examples 1 and 2,
                anisotropic Gaussians, the I2 of a point source, the 2-D
                Coulomb potential of Gaussians)
  ds_stepper    split-step (Strang) time integration of the DS system with
                Phi from split_solver, the L4 loss and its reverse-mode gradient
  periodic      the standard periodic FFT potential solver the paper compares
                against (Tables 1 and 4)

Every function is pinned by a test under tests/ against values printed in the
paper (Tables 1, 2, 4 and 5), closed forms, invariants, or brute force.
"""
from .split_solver import (  # noqa: F401
    SplitParams,
    split_constants,
    grid_points,
    highfreq_multiplier,
    i1_padded_fft,
    i1_padded_dft_matrix,
    polar_nodes_weights,
    polar_rule,
    type2_direct,
    type1_direct,
    i2_direct,
    phi,
    phi_parts,
    phi_transpose,
)
from . import closed_forms  # noqa: F401
from . import ds_stepper  # noqa: F401
from . import periodic  # noqa: F401
