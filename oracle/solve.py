"""The three-step fast Poisson solve as dense linear algebra (test infrastructure only).

Section 2.1 states the algorithm: forward transforms of Table 2 along every
axis, division of every coefficient by its eigenvalue, backward transforms.
Section 2.3 makes the multi-dimensional transform the separable product of
the one-dimensional ones and the eigenvalue the sum of the per-axis ones.
Written as one formula:

    phi = (prod_d B_d) diag(S) (prod_d F_d) g,   S[k] = 1 / sum_d lambda_d[k_d]

where F_d, B_d are the dense matrices of ``transforms.forward_backward`` and
lambda_d comes from ``eigen.eigenvalues``.  When every axis is periodic or
Neumann, the mode with all k_d = 0 has eigenvalue zero; the paper does not
say what to do with it, and this oracle sets its coefficient to zero.  That
is the same as solving for g minus its weighted mean and fixing the weighted
mean of phi to zero (``fd.weights`` gives the weights).

A Helmholtz shift sigma >= 0 ((L - sigma) phi = g, the problem FISHPACK also
solves) divides by sum_d lambda_d - sigma instead; with sigma > 0 nothing is
singular.
"""

from dataclasses import dataclass

import numpy as np

from .transforms import forward_backward
from .eigen import eigenvalues


@dataclass(frozen=True)
class Axis:
    bc: str      # 'P', 'D' or 'N' (both faces), or 'DN' / 'ND' (low face, high face)
    grid: str    # 'v' (regular/vertex) or 's' (staggered); ignored when bc == 'P'
    n: int
    h: float


def _axis_bc(b):
    """'P'/'D'/'N', or a pair of face conditions ('D', 'N') -> 'DN'."""
    if isinstance(b, str):
        return b
    lo, hi = b
    return lo if lo == hi else lo + hi


def axes_from(shape, h, bc, grid):
    """Build the per-axis description from plain sequences (bc entries may be
    face pairs such as ('D', 'N'))."""
    return [Axis(_axis_bc(b), g if _axis_bc(b) != "P" else "v", int(n), float(s))
            for n, s, b, g in zip(shape, h, bc, grid)]


def zero_mode_is_singular(axes, shift=0.0):
    """True when the mode k = 0 has eigenvalue zero on every axis (periodic or
    Neumann on both faces) and there is no shift."""
    return shift == 0.0 and all(a.bc in ("P", "N") for a in axes)


def _apply(mat, x, d):
    """Multiply axis d of x by the matrix (contraction over the matrix columns)."""
    y = np.tensordot(mat, x, axes=([1], [d]))
    return np.moveaxis(y, 0, d)


def solve_spectrum_scale(axes, approx, shift=0.0):
    """diag(S) as an array of the grid's shape: 1 / (sum_d lambda_d - shift), zero mode -> 0."""
    lam = np.full([a.n for a in axes], -float(shift), dtype=np.float64)
    for d, a in enumerate(axes):
        shp = [1] * len(axes)
        shp[d] = a.n
        lam = lam + eigenvalues(a.bc, a.grid, a.n, a.h, approx).reshape(shp)
    s = np.zeros_like(lam)
    if zero_mode_is_singular(axes, shift):
        mask = np.ones(lam.shape, dtype=bool)
        mask[(0,) * len(axes)] = False
        s[mask] = 1.0 / lam[mask]
    else:
        s = 1.0 / lam
    return s


def solve(g, axes, approx, imag_tol=1e-12, shift=0.0):
    """phi for the right-hand side g (any float array of the grid's shape).

    approx is 'ps' (Table 3) or 'fd' (Table 4); shift is the Helmholtz sigma.
    Returns float64.
    """
    g = np.asarray(g, dtype=np.float64)
    if g.shape != tuple(a.n for a in axes):
        raise ValueError(f"rhs shape {g.shape} does not match the axes")
    periodic = any(a.bc == "P" for a in axes)
    x = g.astype(np.complex128) if periodic else g.copy()
    mats = [forward_backward(a.bc, a.grid, a.n) for a in axes]
    for d, (fwd, _) in enumerate(mats):
        x = _apply(fwd, x, d)
    x = x * solve_spectrum_scale(axes, approx, shift)
    for d, (_, bwd) in enumerate(mats):
        x = _apply(bwd, x, d)
    if periodic:
        scale = max(float(np.max(np.abs(x.real))), 1e-300)
        if float(np.max(np.abs(x.imag))) > imag_tol * scale:
            raise AssertionError("solution of a real problem has an imaginary part")
        x = x.real
    return np.ascontiguousarray(x)
