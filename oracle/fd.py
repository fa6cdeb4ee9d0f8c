"""Finite-difference Laplacian of Eq. (FD2) and a dense LU solve (test infrastructure only).

Section 2.2 discretises d2/dx2 by (phi_{j+1} - 2 phi_j + phi_{j-1}) / dx^2 and
calls L the matrix that results together with the boundary conditions, without
writing the boundary rows.  The closures used here are the ones whose
eigenvectors are the transforms of Table 2 with the eigenvalues of Table 4
(a fact the tests check against the table itself):

  periodic           phi_{-1} = phi_{n-1},  phi_n = phi_0
  Dirichlet regular  phi_{-1} = phi_n = 0        (boundary nodes are not unknowns)
  Dirichlet stagg.   phi_{-1} = -phi_0, phi_n = -phi_{n-1}   (zero on the face)
  Neumann regular    phi_{-1} = phi_1,  phi_n = phi_{n-2}    (mirror about the node)
  Neumann stagg.     phi_{-1} = phi_0,  phi_n = phi_{n-1}    (zero flux on the face)

An axis with different conditions on its faces ("DN": Dirichlet low,
Neumann high; "ND" the reverse) closes each end by that face's rule:
  regular grid  Dirichlet end: the boundary node is 0 and not an unknown;
                Neumann end: mirror about the end node (phi_{-1} = phi_1),
                where phi_1 is the Dirichlet node (0) when n = 1
  staggered     Dirichlet face: phi_ghost = -phi_end; Neumann: +phi_end

The multi-dimensional operator is the sum over axes (Section 2.3).  A
Helmholtz shift sigma >= 0 subtracts sigma phi: (L_h - sigma) phi = g.

For singular problems (every axis periodic or Neumann) the solution is fixed
by the gauge sum_j w_j phi_j = 0 with the weights of ``weights``: 1 per node,
except 1/2 on the two end nodes of a regular-grid Neumann axis.  These are
the weights of the left null vector of L, so g - (w.g / w.1) is the part of g
the operator can reach.
"""

import numpy as np


def _pad_axis(phi, d, bc, grid):
    """phi with one ghost layer on each side of axis d, filled by the closure."""
    phi = np.moveaxis(phi, d, 0)
    n = phi.shape[0]
    if bc == "P":
        lo, hi = phi[n - 1], phi[0]
    elif bc == "D" and grid == "v":
        lo, hi = np.zeros_like(phi[0]), np.zeros_like(phi[0])
    elif bc == "D" and grid == "s":
        lo, hi = -phi[0], -phi[n - 1]
    elif bc == "N" and grid == "v":
        if n < 2:
            raise ValueError("regular-grid Neumann axis needs n >= 2")
        lo, hi = phi[1], phi[n - 2]
    elif bc == "N" and grid == "s":
        lo, hi = phi[0], phi[n - 1]
    elif bc in ("DN", "ND") and grid == "v":
        zero = np.zeros_like(phi[0])
        if bc == "DN":   # Dirichlet node below index 0; index n-1 is the Neumann node
            lo, hi = zero, (phi[n - 2] if n >= 2 else zero)
        else:            # index 0 is the Neumann node; Dirichlet node above index n-1
            lo, hi = (phi[1] if n >= 2 else zero), zero
    elif bc in ("DN", "ND") and grid == "s":
        sl, sh = (-1.0, 1.0) if bc == "DN" else (1.0, -1.0)
        lo, hi = sl * phi[0], sh * phi[n - 1]
    else:
        raise ValueError((bc, grid))
    out = np.concatenate([lo[None], phi, hi[None]], axis=0)
    return np.moveaxis(out, 0, d)


def apply_laplacian(phi, axes, shift=0.0):
    """L_h phi - shift phi, L_h phi = sum_d (phi_{j+1} - 2 phi_j + phi_{j-1}) / h_d^2
    with the closures above."""
    phi = np.asarray(phi, dtype=np.float64)
    out = -float(shift) * phi
    for d, a in enumerate(axes):
        p = _pad_axis(phi, d, a.bc, a.grid)
        n = phi.shape[d]
        lo = np.take(p, np.arange(0, n), axis=d)
        mid = np.take(p, np.arange(1, n + 1), axis=d)
        hi = np.take(p, np.arange(2, n + 2), axis=d)
        out += (hi - 2.0 * mid + lo) / (a.h * a.h)
    return out


def assemble_1d(bc, grid, n, h):
    """Dense n x n matrix of the one-dimensional operator (columns = unit vectors)."""
    m = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        p = _pad_axis(e, 0, bc, grid)
        m[:, j] = (p[2:] - 2.0 * p[1:-1] + p[:-2]) / (h * h)
    return m


def assemble(axes):
    """Dense N x N matrix of the multi-dimensional operator (C order, last axis fastest)."""
    mats = [assemble_1d(a.bc, a.grid, a.n, a.h) for a in axes]
    sizes = [a.n for a in axes]
    total = int(np.prod(sizes))
    big = np.zeros((total, total))
    for d, m in enumerate(mats):
        term = np.ones((1, 1))
        for e in range(len(axes)):
            term = np.kron(term, m if e == d else np.eye(sizes[e]))
        big += term
    return big


def is_singular(axes, shift=0.0):
    """The operator has the constant null vector: no shift, every axis periodic
    or Neumann on both faces."""
    return shift == 0.0 and all(a.bc in ("P", "N") for a in axes)


def weights(axes):
    """Gauge / compatibility weights w (product of per-axis weights)."""
    w = np.ones([a.n for a in axes])
    for d, a in enumerate(axes):
        wd = np.ones(a.n)
        if a.bc == "N" and a.grid == "v":
            wd[0] = 0.5
            wd[-1] = 0.5
        shp = [1] * len(axes)
        shp[d] = a.n
        w = w * wd.reshape(shp)
    return w


def weighted_mean(x, axes):
    """sum w x / sum w."""
    w = weights(axes)
    return float(np.sum(w * x) / np.sum(w))


def lu_solve(g, axes, shift=0.0):
    """Dense LU solve of (L - shift) phi = g; bordered system [[L, 1], [w^T, 0]]
    when singular.

    Returns (phi, m_g): m_g is the multiplier of the bordered system, i.e. the
    weighted mean removed from g (0 for nonsingular problems).
    """
    g = np.asarray(g, dtype=np.float64)
    L = assemble(axes) - float(shift) * np.eye(g.size)
    rhs = g.reshape(-1)
    if is_singular(axes, shift):
        N = rhs.size
        w = weights(axes).reshape(-1)
        A = np.zeros((N + 1, N + 1))
        A[:N, :N] = L
        A[:N, N] = 1.0
        A[N, :N] = w
        sol = np.linalg.solve(A, np.concatenate([rhs, [0.0]]))
        return sol[:N].reshape(g.shape), float(sol[N])
    return np.linalg.solve(L, rhs).reshape(g.shape), 0.0


def residual_eta(g, phi, axes, shift=0.0):
    """Scaled residual ||g_c - (L - shift) phi|| / (||L - shift|| ||phi|| + ||g_c||),
    ||L - shift|| <= sum_d 4/h_d^2 + shift.

    g_c is g with its weighted mean removed when the problem is singular.
    """
    g = np.asarray(g, dtype=np.float64)
    if is_singular(axes, shift):
        g = g - weighted_mean(g, axes)
    r = g - apply_laplacian(phi, axes, shift)
    lnorm = sum(4.0 / (a.h * a.h) for a in axes) + float(shift)
    return float(np.linalg.norm(r) / (lnorm * np.linalg.norm(phi) + np.linalg.norm(g)))
