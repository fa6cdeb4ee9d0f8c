"""Plain FP64 CPU oracle for the fast Poisson solve (test infrastructure only).

This package is the independent checker of the GPU solver.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product library never calls into it and shares no code with it.

What it computes follows the paper directly:

* ``transforms`` -- the real and complex discrete transforms written as dense
  n x n matrices (Table 1, Eqs. 5-6) and their pairing with boundary
  conditions and grids, including the backward normalisations (Table 2).
* ``eigen``      -- the per-axis eigenvalues of the pseudo-spectral (Table 3)
  and second-order finite-difference (Table 4) Laplacians, and the domain
  length implied by each grid (Section 2.1, grid definitions).
* ``solve``      -- the three-step algorithm of Section 2.1 (forward
  transforms, division by the summed eigenvalues of Section 2.3, backward
  transforms), applied axis by axis with dense matrix products.
* ``fd``         -- the finite-difference operator of Eq. (FD2) with the
  boundary closures, its dense assembly and a dense LU solve, used to pin
  Table 4 and as the refinement residual reference.
* ``projection`` -- the projection step of Section 5.1 (divergence of a
  staggered velocity, the Poisson solve, velocity and pressure correction).

Beyond the paper's tables: axes with a Dirichlet condition on one face and a
Neumann condition on the other, and a Helmholtz shift (L - sigma) phi = g.

Everything is float64/complex128 NumPy.  There are no FFT calls, no blocking
and no reordering beyond the per-axis matrix products.
"""

from .transforms import (transform_matrix, forward_backward, dft_matrix,
                         idft_matrix, KINDS)
from .eigen import domain_length, eigenvalues, grid_points
from .solve import solve, solve_spectrum_scale, zero_mode_is_singular, Axis, axes_from
from .fd import (apply_laplacian, assemble_1d, assemble, lu_solve, weights,
                 weighted_mean, residual_eta, is_singular)
from .projection import (divergence, gradient, projection_step, velocity_shapes,
                         face_count)

__all__ = [
    "transform_matrix", "forward_backward", "dft_matrix", "idft_matrix", "KINDS",
    "domain_length", "eigenvalues", "grid_points",
    "solve", "solve_spectrum_scale", "zero_mode_is_singular", "Axis", "axes_from",
    "apply_laplacian", "assemble_1d", "assemble", "lu_solve", "weights",
    "weighted_mean", "residual_eta", "is_singular",
    "divergence", "gradient", "projection_step", "velocity_shapes", "face_count",
]
