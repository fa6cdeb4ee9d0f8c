"""Pins of the projection-step oracle (paper Section 5.1) against facts that
do not come from the oracle itself: the discrete divergence of the discrete
gradient is the FD Laplacian with the staggered closures of Eq. (FD2); a
corrected velocity is divergence-free; fields whose answer is known by hand
(a discrete curl, a discrete gradient, one-dimensional flows)."""

import itertools

import numpy as np
import pytest

import oracle
import workloads
from oracle import projection as pj

AXIS_BCS = ["P", "N", "D", ("D", "N"), ("N", "D")]


def _axes(shape, h, bcs):
    return oracle.axes_from(shape, h, bcs, ("s",) * len(shape))


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_div_grad_is_the_fd_laplacian(ndim):
    """div(grad phi) equals the dense FD operator (Eq. FD2 with the staggered
    closures: ghost = +phi at a Neumann face, -phi at a Dirichlet face,
    wrap-around when periodic) for every combination of axis conditions."""
    rng = np.random.default_rng(ndim)
    shape = (5, 4, 6)[:ndim]
    h = (0.3, 0.7, 1.1)[:ndim]
    for bcs in itertools.product(AXIS_BCS, repeat=ndim):
        axes = _axes(shape, h, bcs)
        phi = rng.standard_normal(shape)
        dg = pj.divergence(pj.gradient(phi, axes), axes)
        dense = (oracle.assemble(axes) @ phi.reshape(-1)).reshape(shape)
        assert np.allclose(dg, dense, rtol=0, atol=1e-12 * np.abs(dense).max()), bcs


def test_divergence_and_gradient_by_hand():
    """A 1D staggered axis of three cells, h = 0.5, Dirichlet low face and
    Neumann high face: faces 0..3, div_c = (u_{c+1} - u_c)/h, grad at face 0 =
    2 phi_0 / h (phi = 0 on the face), at face 3 = 0 (no flux)."""
    axes = _axes((3,), (0.5,), [("D", "N")])
    u = np.array([1.0, 4.0, -2.0, 0.5])
    assert np.allclose(pj.divergence([u], axes), [6.0, -12.0, 5.0], rtol=0, atol=1e-15)
    phi = np.array([1.0, 3.0, 2.0])
    g = pj.gradient(phi, axes)[0]
    assert np.allclose(g, [4.0, 4.0, -2.0, 0.0], rtol=0, atol=1e-15)
    # periodic: three faces, face 0 between cell 2 and cell 0
    axp = _axes((3,), (2.0,), ["P"])
    assert np.allclose(pj.divergence([np.array([1.0, 2.0, 7.0])], axp), [0.5, 2.5, -3.0], atol=1e-15)
    assert np.allclose(pj.gradient(phi, axp)[0], [-0.5, 1.0, -0.5], atol=1e-15)


def test_one_dimensional_walls_give_zero_velocity():
    """Between two no-flux walls the only divergence-free 1D flow is 0, and phi
    is the cumulative sum of u*/adt with zero mean (worked out by hand for
    three cells: u* = (0, a, b, 0) on the faces, h = 1)."""
    a, b, adt = 0.7, -1.9, 0.25
    axes = _axes((3,), (1.0,), ["N"])
    vel, p, phi = pj.projection_step([np.array([0.0, a, b, 0.0])], np.zeros(3), axes, adt)
    assert np.allclose(vel[0], 0.0, atol=1e-13)
    want = np.array([-(2 * a + b), a - b, a + 2 * b]) / 3.0 / adt
    assert np.allclose(phi, want, rtol=0, atol=1e-13)
    assert np.allclose(p, phi, atol=0)


def test_one_dimensional_periodic_keeps_the_mean_flow():
    """On a periodic axis the divergence-free part of a 1D flow is its mean."""
    rng = np.random.default_rng(3)
    u = rng.standard_normal(8)
    axes = _axes((8,), (0.1,), ["P"])
    vel, _, _ = pj.projection_step([u], np.zeros(8), axes, 1.3)
    assert np.allclose(vel[0], u.mean(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("bcs", [("P", "P"), ("P", "N"), ("N", "D"), (("D", "N"), "P"), ("N", "N")])
def test_projected_velocity_is_divergence_free(bcs):
    shape, h = (9, 7), (0.2, 0.35)
    axes = _axes(shape, h, bcs)
    d = workloads.desc(shape, h, bcs, ("s", "s"), "fd")
    vel = workloads.mac_velocity(d, seed=11)
    p0 = np.random.default_rng(1).standard_normal(shape)
    new_vel, p1, phi = pj.projection_step(vel, p0, axes, 0.4)
    div0 = np.abs(pj.divergence(vel, axes)).max()
    assert np.abs(pj.divergence(new_vel, axes)).max() <= 1e-12 * div0
    assert np.allclose(p1 - p0, phi, rtol=0, atol=1e-15)
    # Neumann boundary faces are left alone
    for k, b in enumerate(bcs):
        lo, hi = (b, b) if isinstance(b, str) else b
        if b == "P":
            continue
        um, vm = np.moveaxis(vel[k], k, 0), np.moveaxis(new_vel[k], k, 0)
        if lo == "N":
            assert np.array_equal(um[0], vm[0])
        if hi == "N":
            assert np.array_equal(um[-1], vm[-1])


def test_discrete_curl_is_left_unchanged():
    """u = d psi/dy, v = -d psi/dx with psi on the cell corners of a doubly
    periodic grid is divergence-free by construction: phi = 0, velocity kept."""
    rng = np.random.default_rng(5)
    n0, n1, h0, h1 = 6, 8, 0.5, 0.25
    psi = rng.standard_normal((n0, n1))          # psi[i, j] at the corner below-left of cell (i, j)
    u = (np.roll(psi, -1, axis=1) - psi) / h1    # x-face (i, j): corners (i, j) and (i, j + 1)
    v = -(np.roll(psi, -1, axis=0) - psi) / h0   # y-face (i, j): corners (i, j) and (i + 1, j)
    axes = _axes((n0, n1), (h0, h1), ["P", "P"])
    assert np.abs(pj.divergence([u, v], axes)).max() < 1e-12
    vel, p, phi = pj.projection_step([u, v], np.zeros((n0, n1)), axes, 0.3)
    assert np.abs(phi).max() < 1e-12
    assert np.allclose(vel[0], u, atol=1e-12) and np.allclose(vel[1], v, atol=1e-12)


def test_gradient_field_is_removed():
    """u* = grad psi (a discrete gradient) projects to zero velocity with
    phi = (psi - mean psi) / adt on an all-Neumann box."""
    rng = np.random.default_rng(8)
    shape, h = (5, 6, 4), (0.3, 0.2, 0.5)
    axes = _axes(shape, h, ["N", "N", "N"])
    psi = rng.standard_normal(shape)
    adt = 0.6
    vel, _, phi = pj.projection_step(pj.gradient(psi, axes), np.zeros(shape), axes, adt)
    for u in vel:
        assert np.abs(u).max() < 1e-12
    assert np.allclose(phi, (psi - psi.mean()) / adt, rtol=0, atol=1e-12)


def test_vertex_axes_are_refused():
    axes = oracle.axes_from((4,), (1.0,), ["N"], ["v"])
    with pytest.raises(ValueError):
        pj.divergence([np.zeros(5)], axes)
