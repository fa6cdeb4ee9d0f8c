"""Seeded synthetic right-hand sides and problem descriptions.

This module serves both the GPU solver's tests and benchmark and the CPU
oracle's checks.  It draws random numbers and lays out input fields; it holds
none of the solver's arithmetic (no transforms, eigenvalues or stencils of
the Poisson operator).  Every generator is deterministic for its seed.

Problem descriptions are plain dicts:

    {"shape": (n0, n1, n2), "h": (h0, h1, h2), "bc": ("P", "D", "N"),
     "grid": ("v", "s", "s"), "approx": "fd" | "ps"}

with bc 'P'/'D'/'N' (periodic / Dirichlet / Neumann, the same on both faces
of an axis), grid 'v' (vertex, the paper's regular grid) or 's' (staggered),
and arrays in C order with the last axis contiguous.

The workloads stand in for the paper's experiments, whose data (the CLMM city
case) is not available: uniform noise on a periodic box, a sum of discrete
eigenmodes on a mixed-boundary box, Gaussian blobs on an all-Neumann vertex
cube, a batch of random 2D problems, and a stream of divergences of random
staggered velocity fields in a channel.
"""

import numpy as np


def desc(shape, h, bc, grid, approx):
    return {"shape": tuple(int(n) for n in shape), "h": tuple(float(x) for x in h),
            "bc": tuple(bc), "grid": tuple(grid), "approx": approx}


def _is_singular(d):
    return all(b in ("P", "N") for b in d["bc"])


def remove_weighted_mean(g, d):
    """g minus its weighted mean, the mean that makes a right-hand side of a
    singular problem (every axis periodic or Neumann) compatible: node weights
    are the product over axes of 1/2 at both end nodes of a vertex-grid
    Neumann axis and 1 elsewhere (the trapezoid rule on those axes)."""
    w = np.ones((), dtype=np.float64)
    for n, b, gr in zip(d["shape"], d["bc"], d["grid"]):
        wd = np.ones(n)
        if b == "N" and gr == "v" and n >= 2:
            wd[0] = wd[-1] = 0.5
        w = np.multiply.outer(w, wd)
    return g - float((w * g).sum() / w.sum())


# --------------------------------------------------------------------------- periodic box
def periodic_noise(n=32, seed=1):
    """n^3 periodic box, FD, h = 1/n; g ~ U(-1, 1) with its mean subtracted."""
    d = desc((n, n, n), (1.0 / n,) * 3, ("P",) * 3, ("v",) * 3, "fd")
    rng = np.random.default_rng(seed)
    g = rng.uniform(-1.0, 1.0, size=d["shape"])
    g -= g.mean()
    return d, g


# --------------------------------------------------------------------------- mixed box
def mixed_modes(n=256, seed=2, approx="fd", n_modes=16, noise=1e-3):
    """n^3 staggered box: periodic x, Dirichlet y, Neumann z; h = 1/n.

    g = sum_m a_m v_m + noise * U(-1, 1), a_m ~ N(0, 1), where each v_m is a
    product of one periodic cosine or sine in x, one staggered-grid sine
    sin(pi (j+1/2)(ky+1)/n) in y and one staggered-grid cosine
    cos(pi (j+1/2) kz/n) in z.  Returns (desc, g, modes) with modes a list of
    (a, "cos"|"sin", kx, ky, kz) so a test can build the noise-free solution.
    """
    d = desc((n, n, n), (1.0 / n,) * 3, ("P", "D", "N"), ("v", "s", "s"), approx)
    rng = np.random.default_rng(seed)
    j = np.arange(n, dtype=np.float64)
    g = np.zeros(d["shape"])
    modes = []
    for _ in range(n_modes):
        a = float(rng.standard_normal())
        kx = int(rng.integers(0, n // 2 + 1))
        kind = "cos" if rng.integers(0, 2) == 0 else "sin"
        if kind == "sin" and (kx == 0 or 2 * kx == n):
            kind = "cos"
        ky = int(rng.integers(0, n))
        kz = int(rng.integers(0, n))
        ang_x = 2.0 * np.pi * np.mod(kx * np.arange(n), n) / n
        vx = np.cos(ang_x) if kind == "cos" else np.sin(ang_x)
        vy = np.sin(np.pi * (j + 0.5) * (ky + 1) / n)
        vz = np.cos(np.pi * (j + 0.5) * kz / n)
        g += a * vx[:, None, None] * vy[None, :, None] * vz[None, None, :]
        modes.append((a, kind, kx, ky, kz))
    g += noise * rng.uniform(-1.0, 1.0, size=d["shape"])
    return d, g, modes


# --------------------------------------------------------------------------- Neumann cube
def neumann_blobs(n=512, seed=3, n_blobs=64, sigma=0.02):
    """n^3 vertex-grid all-Neumann cube on [0,1]^3, FD, h = 1/(n-1).

    g = sum_c a_c exp(-|x - x_c|^2 / (2 sigma^2)), x_c ~ U[0,1]^3, a_c ~ N(0,1),
    evaluated separably at x_j = j/(n-1); the trapezoid-weighted mean (end
    nodes weighted 1/2 on every axis) is subtracted, so g is compatible.
    """
    h = 1.0 / (n - 1)
    d = desc((n, n, n), (h,) * 3, ("N",) * 3, ("v",) * 3, "fd")
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_blobs, 3))
    amps = rng.standard_normal(n_blobs)
    x = np.arange(n, dtype=np.float64) * h
    gx = np.exp(-(x[None, :] - centres[:, 0:1]) ** 2 / (2 * sigma * sigma))
    gy = np.exp(-(x[None, :] - centres[:, 1:2]) ** 2 / (2 * sigma * sigma))
    gz = np.exp(-(x[None, :] - centres[:, 2:3]) ** 2 / (2 * sigma * sigma))
    yz = (gy[:, :, None] * gz[:, None, :]).reshape(n_blobs, n * n)
    g = ((gx * amps[:, None]).T @ yz).reshape(n, n, n)
    return d, remove_weighted_mean(g, d)


# --------------------------------------------------------------------------- 2D batch
_BC = ("P", "D", "N")
_GRID = ("v", "s")


def batch_2d(count=2048, lo=64, hi=1024, seed=4):
    """`count` independent 2D problem descriptions, FD, h_d = 1/n_d.

    n0, n1 ~ U{lo..hi}; bc per axis ~ U{P, D, N}; grid per problem ~ U{v, s}.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(lo, hi + 1, size=(count, 2))
    bcs = rng.integers(0, 3, size=(count, 2))
    grids = rng.integers(0, 2, size=count)
    out = []
    for i in range(count):
        n0, n1 = int(ns[i, 0]), int(ns[i, 1])
        g = _GRID[int(grids[i])]
        out.append(desc((n0, n1), (1.0 / n0, 1.0 / n1),
                        (_BC[int(bcs[i, 0])], _BC[int(bcs[i, 1])]), (g, g), "fd"))
    return out


def batch_rhs(d, i, seed=4):
    """g_i ~ N(0, 1) for problem i of a batch; when the problem is singular its
    weighted mean (remove_weighted_mean) is removed, so g_i is compatible."""
    rng = np.random.default_rng([seed, i])
    g = rng.standard_normal(d["shape"])
    if _is_singular(d):
        g = remove_weighted_mean(g, d)
    return g


# --------------------------------------------------------------------------- channel stream
def channel_desc(n0=1024, n1=512, n2=256):
    """Channel of aspect 4:1:1: periodic x and z, staggered Neumann y, dx = 2 dy = dz."""
    dx = 4.0 / n0
    dy = 1.0 / n1
    dz = 1.0 / n2
    return desc((n0, n1, n2), (dx, dy, dz), ("P", "N", "P"), ("v", "s", "v"), "fd")


def channel_divergence(d, s, seed=5, device="cpu", noise=0.1):
    """Divergence of a random staggered (MAC) velocity field, as a float64 torch tensor.

    The velocity is the discrete curl of an edge-centred vector potential with
    N(0, 1) entries plus N(0, noise^2) face noise; the wall-normal component is
    zero on both y walls.  Face u_i sits left of cell i in x (periodic), v_j
    below cell j in y (n1 + 1 faces, the end ones on the walls), w_k behind
    cell k in z (periodic).  g = du/dx + dv/dy + dw/dz on cell centres, so the
    sum of g vanishes up to rounding.  Stream index s selects the field.
    """
    import torch
    n0, n1, n2 = d["shape"]
    dx, dy, dz = d["h"]
    gen = torch.Generator(device=device)
    gen.manual_seed(seed * 1_000_003 + s)
    f64 = torch.float64

    def randn(*shape, std=1.0):
        return std * torch.randn(*shape, generator=gen, device=device, dtype=f64)

    # vector potential on edges: Ax on x-edges, Ay on y-edges, Az on z-edges
    ax = randn(n0, n1 + 1, n2)
    ay = randn(n0, n1, n2)
    az = randn(n0, n1 + 1, n2)
    ax[:, 0, :] = 0.0
    ax[:, n1, :] = 0.0
    az[:, 0, :] = 0.0
    az[:, n1, :] = 0.0
    # curl on faces: u = dAz/dy - dAy/dz, v = dAx/dz - dAz/dx, w = dAy/dx - dAx/dy
    u = (az[:, 1:, :] - az[:, :-1, :]) / dy - (torch.roll(ay, -1, 2) - ay) / dz
    v = (torch.roll(ax, -1, 2) - ax) / dz - (torch.roll(az, -1, 0) - az) / dx
    w = (torch.roll(ay, -1, 0) - ay) / dx - (ax[:, 1:, :] - ax[:, :-1, :]) / dy
    u = u + randn(n0, n1, n2, std=noise)
    v = v + randn(n0, n1 + 1, n2, std=noise)
    w = w + randn(n0, n1, n2, std=noise)
    v[:, 0, :] = 0.0
    v[:, n1, :] = 0.0
    g = ((torch.roll(u, -1, 0) - u) / dx + (v[:, 1:, :] - v[:, :-1, :]) / dy
         + (torch.roll(w, -1, 2) - w) / dz)
    return g.contiguous()


# --------------------------------------------------------------------------- projection step
def mac_velocity(d, seed=6, std=1.0):
    """Predicted velocity of a projection step on the staggered (MAC) grid of
    problem d (every axis periodic or staggered), as float64 numpy arrays.

    Component k has n_k faces along axis k when that axis is periodic and
    n_k + 1 otherwise (face f on the low side of cell f), and n_j along the
    other axes.  Entries ~ N(0, std^2); on an axis with a Neumann face the
    velocity on that boundary face is 0 (no flow through a wall), so the
    Poisson problem of the projection is solvable.
    """
    rng = np.random.default_rng([seed, len(d["shape"])] + list(d["shape"]))
    vel = []
    for k, (n, b) in enumerate(zip(d["shape"], d["bc"])):
        faces = n if b == "P" else n + 1
        shape = tuple(faces if j == k else m for j, m in enumerate(d["shape"]))
        u = std * rng.standard_normal(shape)
        lo, hi = (b, b) if isinstance(b, str) else b
        um = np.moveaxis(u, k, 0)
        if b != "P" and lo == "N":
            um[0] = 0.0
        if b != "P" and hi == "N":
            um[n] = 0.0
        vel.append(u)
    return vel
