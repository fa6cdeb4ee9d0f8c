"""Discrete eigenfunctions of the one-dimensional second-order stencil
(Table 4 eigenvalues on the Section 2.1 grids), for tests whose expected
solutions are closed forms: a right-hand side that is a sum of such modes
has as its exact solution each mode divided by its eigenvalue."""

import numpy as np


def eigenpair(bc, grid, n, k, h):
    """Mode k of the 1D second-difference operator with the given closure:
    (vector over the n nodes, eigenvalue).  The vertex grid has nodes at
    j h, the staggered one at (j + 1/2) h (Section 2.1)."""
    j = np.arange(n, dtype=np.float64)
    if bc == "P":
        v, theta = np.cos(2 * np.pi * k * j / n), np.pi * k / n
    elif bc == "N" and grid == "v":
        v, theta = np.cos(np.pi * k * j / (n - 1)), np.pi * k / (2 * (n - 1))
    elif bc == "D" and grid == "v":
        v, theta = np.sin(np.pi * (k + 1) * (j + 1) / (n + 1)), np.pi * (k + 1) / (2 * (n + 1))
    elif bc == "N" and grid == "s":
        v, theta = np.cos(np.pi * k * (j + 0.5) / n), np.pi * k / (2 * n)
    elif bc == "D" and grid == "s":
        v, theta = np.sin(np.pi * (k + 1) * (j + 0.5) / n), np.pi * (k + 1) / (2 * n)
    else:
        raise ValueError(bc + grid)
    return v, -(2.0 * np.sin(theta) / h) ** 2
