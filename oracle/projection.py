"""Projection step of an incompressible-flow solver (test infrastructure only).

Section 5.1 of the paper (the CLMM model) corrects a predicted velocity u* in
every Runge-Kutta stage k:

    Lap phi = div u* / (alpha_k dt),
    u^(k+1) = u* - alpha_k dt grad phi,
    p^(k+1) = p^(k) + phi,

with second-order central differences on a staggered (MAC) grid, the
pressure and phi at cell centres and velocity component d on the faces
normal to axis d.  The paper does not write the discrete operators out; this
module takes the usual MAC reading:

* cells 0..n-1 of width h along every axis; face f of axis d lies on the low
  side of cell f.  A periodic axis has n faces (face n is face 0); any other
  axis has n + 1, faces 0 and n on the boundary;
* div at cell c: sum_d (u_d[c + e_d] - u_d[c]) / h_d;
* grad_d at an interior face f: (phi[f] - phi[f - 1]) / h_d (periodic: every
  face is interior, cell -1 is cell n - 1).  At a boundary face the face's
  condition closes it as in the staggered Laplacian: Neumann (no flux) gives
  0, so the face velocity stays as it is; Dirichlet (phi = 0 on the face, the
  ghost value is -phi of the adjacent cell) gives 2 phi[0] / h at face 0 and
  -2 phi[n-1] / h at face n.

With these closures div(grad phi) is the FD operator of Eq. (FD2) on a
staggered grid, so the corrected velocity has zero divergence whenever the
Poisson problem is solvable (the tests check both facts).  Only staggered
(or periodic) axes and the FD approximation are meaningful here.

Plain NumPy in float64: slicing and the oracle's own dense solve.
"""

import numpy as np

from .solve import solve


def _check(axes):
    for a in axes:
        if a.bc != "P" and a.grid != "s":
            raise ValueError("the projection step needs staggered (or periodic) axes")


def _faces(bc):
    """Boundary condition of the low and the high face of an axis."""
    if bc == "P":
        return "P", "P"
    if len(bc) == 2:
        return bc[0], bc[1]
    return bc, bc


def face_count(a):
    """Number of velocity faces along axis a: n when periodic, else n + 1."""
    return a.n if a.bc == "P" else a.n + 1


def velocity_shapes(axes):
    """Array shape of each velocity component (component d has face_count
    entries along axis d and n along the others)."""
    shapes = []
    for d in range(len(axes)):
        shapes.append(tuple(face_count(a) if e == d else a.n for e, a in enumerate(axes)))
    return shapes


def divergence(vel, axes):
    """div u at the cell centres: sum over axes of (face above - face below) / h."""
    _check(axes)
    out = np.zeros([a.n for a in axes])
    for d, a in enumerate(axes):
        u = np.moveaxis(np.asarray(vel[d], dtype=np.float64), d, 0)
        if a.bc == "P":
            above = np.concatenate([u[1:], u[:1]], axis=0)   # face n is face 0
            below = u
        else:
            above = u[1:]
            below = u[:-1]
        out += np.moveaxis((above - below) / a.h, 0, d)
    return out


def gradient(phi, axes):
    """grad phi on the faces, one array per axis (velocity_shapes)."""
    _check(axes)
    phi = np.asarray(phi, dtype=np.float64)
    grads = []
    for d, a in enumerate(axes):
        q = np.moveaxis(phi, d, 0)
        n = a.n
        if a.bc == "P":
            below = np.concatenate([q[n - 1:], q[:n - 1]], axis=0)   # cell -1 is cell n-1
            g = (q - below) / a.h
        else:
            lo, hi = _faces(a.bc)
            g = np.zeros((n + 1,) + q.shape[1:])
            g[1:n] = (q[1:] - q[:-1]) / a.h
            if lo == "D":
                g[0] = 2.0 * q[0] / a.h
            if hi == "D":
                g[n] = -2.0 * q[n - 1] / a.h
        grads.append(np.moveaxis(g, 0, d))
    return grads


def projection_step(vel, p, axes, adt):
    """One projection: returns (corrected velocity list, new pressure, phi).

    phi solves Lap phi = div(u*) / adt by the oracle's FD solve (on a singular
    problem the part of the right-hand side the operator cannot reach is
    dropped and phi has zero mean)."""
    _check(axes)
    g = divergence(vel, axes) / float(adt)
    phi = solve(g, axes, "fd")
    grads = gradient(phi, axes)
    new_vel = [np.asarray(u, dtype=np.float64) - float(adt) * gd for u, gd in zip(vel, grads)]
    return new_vel, np.asarray(p, dtype=np.float64) + phi, phi
