"""Per-axis eigenvalues of the discrete Laplacians (test infrastructure only).

* ``grid_points``   -- node positions of Section 2.1: periodic x_j = jL/n,
  regular (vertex) Dirichlet x_j = (j+1)L/(n+1), regular Neumann
  x_j = jL/(n-1), staggered x_j = (j+1/2)L/n.
* ``domain_length`` -- L implied by a spacing h on each of those grids.
* ``eigenvalues``   -- Table 3 (pseudo-spectral) and Table 4 (second-order
  finite differences), index k running over the output index of the
  matching forward transform of Table 2.

Axes with a Dirichlet condition on one face and a Neumann condition on the
other ("DN" / "ND", beyond Tables 3 and 4) have the eigenfunctions
sin / cos((k+1/2) pi x/L): pseudo-spectral lambda_k = -((k+1/2) pi/L)^2 and
finite differences lambda_k = -(2 sin(pi (2k+1)/(4n))/dx)^2, with L = n h on
both grids (vertex: unknowns on the Neumann node and the interior nodes).

Reading of the printed periodic pseudo-spectral cutoff: the two branches of
Table 3 select the aliased wavenumber min(k, n-k), which is what makes the
operator real and symmetric under k <-> n-k; the Nyquist mode of an even n
takes (n/2)^2.
"""

import numpy as np


def domain_length(bc, grid, n, h):
    """L such that the grid of Section 2.1 with n unknowns has spacing h."""
    if bc == "P" or grid == "s" or bc in ("DN", "ND"):
        return n * h
    if bc == "D":
        return (n + 1) * h
    if bc == "N":
        return (n - 1) * h
    raise ValueError(bc)


def grid_points(bc, grid, n, h):
    """Node coordinates x_j, j = 0..n-1 (Section 2.1)."""
    L = domain_length(bc, grid, n, h)
    j = np.arange(n, dtype=np.float64)
    if bc == "P":
        return j * L / n
    if grid == "s":
        return (j + 0.5) * L / n
    if bc == "DN":
        return (j + 1.0) * L / n
    if bc == "ND":
        return j * L / n
    if bc == "D":
        return (j + 1.0) * L / (n + 1)
    return j * L / (n - 1)


def _sinpi(num, den):
    num = np.mod(np.asarray(num, dtype=np.int64), 2 * den)
    return np.sin(np.pi * num.astype(np.float64) / den)


def eigenvalues(bc, grid, n, h, approx):
    """lambda_k, k = 0..n-1, for one axis.  approx is 'ps' or 'fd'."""
    k = np.arange(n, dtype=np.int64)
    if approx == "ps":
        L = domain_length(bc, grid, n, h)
        if bc == "P":
            m = np.minimum(k, n - k).astype(np.float64)
            return -(2.0 * np.pi * m / L) ** 2
        if bc == "D":
            return -(np.pi * (k + 1).astype(np.float64) / L) ** 2
        if bc == "N":
            return -(np.pi * k.astype(np.float64) / L) ** 2
        if bc in ("DN", "ND"):
            return -(np.pi * (k.astype(np.float64) + 0.5) / L) ** 2
        raise ValueError(bc)
    if approx == "fd":
        if bc == "P":
            s = _sinpi(k, n)
        elif bc == "D" and grid == "v":
            s = _sinpi(k + 1, 2 * (n + 1))
        elif bc == "D" and grid == "s":
            s = _sinpi(k + 1, 2 * n)
        elif bc == "N" and grid == "v":
            s = _sinpi(k, 2 * (n - 1))
        elif bc == "N" and grid == "s":
            s = _sinpi(k, 2 * n)
        elif bc in ("DN", "ND"):
            s = _sinpi(2 * k + 1, 4 * n)
        else:
            raise ValueError((bc, grid))
        return -(2.0 * s / h) ** 2
    raise ValueError(approx)
