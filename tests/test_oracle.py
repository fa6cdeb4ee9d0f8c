"""Pins of the CPU oracle to facts other than itself (no GPU).

Each group names the passage it checks and what independent fact it is
compared with: a library routine (scipy.fft), a dense LU solve of the
assembled stencil, continuous closed forms, hand-derived fixtures, the
eigenvalues printed in Table 4, convergence orders and invariants.
"""

import itertools
import json
import os

import numpy as np
import pytest
import scipy.fft as sfft
import scipy.linalg as sla

import oracle
from oracle import transforms as T
from oracle.solve import Axis

HERE = os.path.dirname(os.path.abspath(__file__))
KINDS = [("P", "v"), ("D", "v"), ("D", "s"), ("N", "v"), ("N", "s")]
# different conditions on the two faces of an axis (Dirichlet low / Neumann high, and the reverse)
MIXED = [("DN", "v"), ("DN", "s"), ("ND", "v"), ("ND", "s")]
SIZES_P1 = list(range(1, 33)) + [48, 64, 100, 127, 511, 512, 1021]


def _valid(bc, grid, n):
    return not (bc == "N" and grid == "v" and n < 2)


# ---------------------------------------------------------------- Table 1 vs scipy.fft
@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 9, 16, 31, 64, 100])
def test_table1_matches_scipy(n):
    """Table 1 sums equal scipy's unnormalised DCT/DST types 1-3 (column by column), and
    the type-IV transforms of the mixed-face axes equal scipy's type 4."""
    eye = np.eye(n)
    pairs = [("DCT-II", lambda x: sfft.dct(x, type=2, axis=0)),
             ("DCT-III", lambda x: sfft.dct(x, type=3, axis=0)),
             ("DST-I", lambda x: sfft.dst(x, type=1, axis=0)),
             ("DST-II", lambda x: sfft.dst(x, type=2, axis=0)),
             ("DST-III", lambda x: sfft.dst(x, type=3, axis=0)),
             ("DCT-I", lambda x: sfft.dct(x, type=1, axis=0)),
             ("DST-IV", lambda x: sfft.dst(x, type=4, axis=0)),
             ("DCT-IV", lambda x: sfft.dct(x, type=4, axis=0))]
    for name, lib in pairs:
        mine = T.transform_matrix(name, n)
        ref = lib(eye)
        assert np.max(np.abs(mine - ref)) <= 1e-13 * n, name


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 33])
def test_dft_pair_matches_numpy(n):
    """Eqs. (5)-(6): forward = fft / n, inverse = n * ifft."""
    x = np.random.default_rng(n).standard_normal(n) + 1j * np.random.default_rng(n + 1).standard_normal(n)
    assert np.allclose(T.dft_matrix(n) @ x, np.fft.fft(x) / n, atol=1e-14, rtol=0)
    assert np.allclose(T.idft_matrix(n) @ x, np.fft.ifft(x) * n, atol=1e-13, rtol=0)


# ---------------------------------------------------------------- Table 2 normalisations
@pytest.mark.parametrize("bc,grid", KINDS + MIXED)
def test_table2_backward_inverts_forward(bc, grid):
    """Table 2: the scaled backward transform is the inverse of the forward one."""
    for n in SIZES_P1:
        if not _valid(bc, grid, n):
            continue
        F, B = T.forward_backward(bc, grid, n)
        err = np.max(np.abs(B @ F - np.eye(n)))
        assert err <= 2e-13 * max(1, np.log2(n)), (n, err)


# ---------------------------------------------------------------- Table 4 vs the stencil
@pytest.mark.parametrize("bc,grid", KINDS + MIXED)
def test_table4_eigenvalues_of_stencil_matrix(bc, grid):
    """The assembled Eq. (FD2) matrix has exactly the eigenvalues printed in Table 4."""
    for n in [1, 2, 3, 4, 5, 8, 13, 32]:
        if not _valid(bc, grid, n):
            continue
        h = 0.37
        L = oracle.assemble_1d(bc, grid, n, h)
        lam_table = np.sort(oracle.eigenvalues(bc, grid, n, h, "fd"))
        lam_mat = np.sort(np.linalg.eigvals(L).real)
        assert np.allclose(lam_mat, lam_table, atol=1e-11 / h ** 2, rtol=1e-12), (n,)


@pytest.mark.parametrize("bc,grid", KINDS + MIXED)
def test_backward_columns_are_stencil_eigenvectors(bc, grid):
    """Column k of the backward transform is an eigenvector of L with Table 4's lambda_k
    (pins the index pairing between Tables 2 and 4)."""
    for n in [1, 2, 3, 6, 11, 16]:
        if not _valid(bc, grid, n):
            continue
        h = 0.5
        L = oracle.assemble_1d(bc, grid, n, h)
        _, B = T.forward_backward(bc, grid, n)
        lam = oracle.eigenvalues(bc, grid, n, h, "fd")
        err = np.max(np.abs(L @ B - B * lam[None, :]))
        assert err <= 1e-12 * np.max(np.abs(lam) + 1.0), (n, err)


# ---------------------------------------------------------------- FD solve vs dense LU
def _all_axes_combos(ns):
    for kinds in itertools.product(KINDS + MIXED, repeat=len(ns)):
        yield [Axis(b, g, n, 1.0 / (n + 1.3 * i + 0.7)) for i, ((b, g), n) in enumerate(zip(kinds, ns))]


@pytest.mark.parametrize("ns", [(1,), (2,), (3,), (4,), (7,), (2, 3), (4, 4), (3, 5), (2, 3, 2), (4, 3, 2)])
def test_fd_solve_matches_dense_lu(ns):
    """Every combination of boundary kinds: the transform solve equals the LU solve of the
    assembled stencil (bordered by the gauge row when singular)."""
    rng = np.random.default_rng(sum(ns))
    for axes in _all_axes_combos(ns):
        if any(not _valid(a.bc, a.grid, a.n) for a in axes):
            continue
        g = rng.standard_normal(ns)
        phi = oracle.solve(g, axes, "fd")
        ref, _ = oracle.lu_solve(g, axes)
        scale = np.max(np.abs(ref)) + 1e-300
        assert np.max(np.abs(phi - ref)) <= 1e-11 * scale, [(a.bc, a.grid) for a in axes]


@pytest.mark.parametrize("ns", [(8, 8, 8), (8, 7, 6)])
def test_fd_solve_matches_dense_lu_8cubed(ns):
    """Dense LU on up to 8^3 unknowns with mixed boundary kinds."""
    rng = np.random.default_rng(7)
    combos = [[("P", "v"), ("D", "s"), ("N", "s")], [("N", "v")] * 3, [("D", "v"), ("P", "v"), ("N", "v")],
              [("P", "v")] * 3]
    for kinds in combos:
        axes = [Axis(b, g, n, 1.0 / n) for (b, g), n in zip(kinds, ns)]
        g = rng.standard_normal(ns)
        phi = oracle.solve(g, axes, "fd")
        ref, _ = oracle.lu_solve(g, axes)
        assert np.max(np.abs(phi - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("bc,grid", [("D", "v"), ("D", "s"), ("N", "s"), ("N", "v")])
def test_fd_1d_matches_banded_solver(bc, grid):
    """1D nonsingular cases against scipy's banded (Thomas-type) solver; singular
    Neumann against the bordered solve."""
    n = 300
    h = 1.0 / n
    axes = [Axis(bc, grid, n, h)]
    g = np.random.default_rng(3).standard_normal(n)
    phi = oracle.solve(g, axes, "fd")
    if bc == "D":
        L = oracle.assemble_1d(bc, grid, n, h)
        ab = np.zeros((3, n))
        ab[0, 1:] = np.diag(L, 1)
        ab[1] = np.diag(L)
        ab[2, :-1] = np.diag(L, -1)
        ref = sla.solve_banded((1, 1), ab, g)
    else:
        ref, _ = oracle.lu_solve(g, axes)
    assert np.max(np.abs(phi - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_fd_periodic_1d_reduced_banded():
    """Cyclic system: fixing phi_0 = 0 and dropping the (redundant, since sum g = 0) first
    equation leaves a tridiagonal system for a banded solver; the zero-mean gauge is
    restored afterwards."""
    n = 257
    h = 1.0 / n
    g = np.random.default_rng(11).standard_normal(n)
    g -= g.mean()
    phi = oracle.solve(g, [Axis("P", "v", n, h)], "fd")
    # pin phi_0 = 0 to make the cyclic system nonsingular, solve the rest, then shift
    L = oracle.assemble_1d("P", "v", n, h)
    A = L[1:, 1:]
    ab = np.zeros((3, n - 1))
    ab[0, 1:] = np.diag(A, 1)
    ab[1] = np.diag(A)
    ab[2, :-1] = np.diag(A, -1)
    # A is tridiagonal except for the wrap entries, which vanish once phi_0 = 0 is fixed
    assert np.count_nonzero(A - np.diag(np.diag(A)) - np.diag(np.diag(A, 1), 1) - np.diag(np.diag(A, -1), -1)) == 0
    rest = sla.solve_banded((1, 1), ab, g[1:])
    ref = np.concatenate([[0.0], rest])
    ref -= ref.mean()
    assert np.max(np.abs(phi - ref)) <= 1e-10 * np.max(np.abs(ref))


# ---------------------------------------------------------------- hand-derived fixtures
def test_golden_tiny_cases():
    """Hand-solved one-dimensional systems (tests/golden/tiny_1d.json)."""
    with open(os.path.join(HERE, "golden", "tiny_1d.json")) as f:
        cases = json.load(f)["cases"]
    assert len(cases) >= 8
    for c in cases:
        axes = [Axis(c["bc"], c["grid"], c["n"], c["h"])]
        phi = oracle.solve(np.array(c["g"]), axes, c["approx"])
        want = np.array(c["phi"]) if "phi" in c else np.array(c["phi_over_pi2"]) / np.pi ** 2
        assert np.allclose(phi, want, atol=1e-14, rtol=0), c["name"]


# ---------------------------------------------------------------- Table 3: continuous closed forms
def _eigfun(bc, grid, m, x, L):
    if bc == "P":
        return np.cos(2 * np.pi * m * x / L), -(2 * np.pi * m / L) ** 2
    if bc == "D":
        return np.sin(np.pi * m * x / L), -(np.pi * m / L) ** 2
    if bc == "DN":  # zero at x = 0, zero slope at x = L
        return np.sin((m + 0.5) * np.pi * x / L), -((m + 0.5) * np.pi / L) ** 2
    if bc == "ND":  # zero slope at x = 0, zero at x = L
        return np.cos((m + 0.5) * np.pi * x / L), -((m + 0.5) * np.pi / L) ** 2
    return np.cos(np.pi * m * x / L), -(np.pi * m / L) ** 2


@pytest.mark.parametrize("bc,grid", KINDS + MIXED)
def test_ps_exact_on_continuous_eigenfunctions(bc, grid):
    """Pseudo-spectral solve of a sampled continuous eigenfunction of d2/dx2 returns
    g / lambda_continuous: pins Table 3 together with the grid positions and L."""
    for n in [5, 8, 12]:
        h = 0.3
        L = oracle.domain_length(bc, grid, n, h)
        x = oracle.grid_points(bc, grid, n, h)
        # grid spacing must be h
        if n > 1:
            assert np.allclose(np.diff(x), h)
        modes = {"P": range(1, (n + 1) // 2), "D": range(1, n + 1), "N": range(1, n),
                 "DN": range(0, n), "ND": range(0, n)}[bc]
        for m in modes:
            g, lam = _eigfun(bc, grid, m, x, L)
            phi = oracle.solve(g, [Axis(bc, grid, n, h)], "ps")
            assert np.allclose(phi, g / lam, atol=1e-12 * np.max(np.abs(g / lam)), rtol=0), (n, m)


def test_ps_3d_product_of_eigenfunctions():
    """Section 2.3: a product of per-axis eigenfunctions has the summed eigenvalue."""
    kinds = [("P", "v"), ("D", "s"), ("N", "v")]
    ns = (8, 6, 7)
    hs = (0.25, 0.4, 0.3)
    axes = [Axis(b, g, n, h) for (b, g), n, h in zip(kinds, ns, hs)]
    ms = (3, 2, 4)
    fs, lams = [], []
    for (b, g), n, h, m in zip(kinds, ns, hs, ms):
        L = oracle.domain_length(b, g, n, h)
        f, lam = _eigfun(b, g, m, oracle.grid_points(b, g, n, h), L)
        fs.append(f)
        lams.append(lam)
    g3 = fs[0][:, None, None] * fs[1][None, :, None] * fs[2][None, None, :]
    phi = oracle.solve(g3, axes, "ps")
    assert np.allclose(phi, g3 / sum(lams), atol=1e-13 * np.max(np.abs(g3)), rtol=0)


def test_ps_periodic_aliased_sine_is_real_and_symmetric():
    """Reading of the garbled Table 3 periodic cutoff: sines and cosines of the same
    wavenumber m and n-m share one eigenvalue, and the solution stays real."""
    n = 8
    h = 1.0 / n
    x = oracle.grid_points("P", "v", n, h)
    for m in range(1, n):
        g = np.sin(2 * np.pi * m * x)
        mm = min(m, n - m)
        phi = oracle.solve(g, [Axis("P", "v", n, h)], "ps")
        assert np.allclose(phi, -g / (2 * np.pi * mm) ** 2, atol=1e-14)


# ---------------------------------------------------------------- convergence order (FD)
def _fd_error(kind, n):
    bc, grid = kind
    if bc == "P":
        h = 1.0 / n
        x = np.arange(n) * h
        phi = np.exp(np.sin(2 * np.pi * x))
        g = phi * (4 * np.pi ** 2 * np.cos(2 * np.pi * x) ** 2 - 4 * np.pi ** 2 * np.sin(2 * np.pi * x))
    elif bc == "D":
        h = 1.0 / (n + 1) if grid == "v" else 1.0 / n
        x = oracle.grid_points(bc, grid, n, h)
        phi = np.sin(np.pi * x) * np.exp(x)
        g = np.exp(x) * ((1 - np.pi ** 2) * np.sin(np.pi * x) + 2 * np.pi * np.cos(np.pi * x))
    else:
        # Neumann on both faces, or one Dirichlet face: x^2 (1-x)^2 has zero value
        # and zero slope at both ends of [0, 1]
        h = 1.0 / (n - 1) if (grid == "v" and bc == "N") else 1.0 / n
        x = oracle.grid_points(bc, grid, n, h)
        phi = x ** 2 * (1 - x) ** 2
        g = 2 - 12 * x + 12 * x ** 2
    axes = [Axis(bc, grid, n, h)]
    num = oracle.solve(g, axes, "fd")
    if bc in ("P", "N"):
        phi = phi - oracle.weighted_mean(phi, axes)
    return np.max(np.abs(num - phi))


@pytest.mark.parametrize("kind", KINDS + MIXED)
def test_fd_second_order_convergence(kind):
    """Eq. (FD2) is second order: halving h divides the error by about 4."""
    e1, e2 = _fd_error(kind, 64), _fd_error(kind, 128)
    ratio = e1 / e2
    assert 3.6 < ratio < 4.4, ratio


# ---------------------------------------------------------------- invariants
def test_invariants_gauge_realness_linearity_scaling_permutation():
    rng = np.random.default_rng(5)
    axes = [Axis("P", "v", 6, 0.2), Axis("N", "v", 5, 0.3), Axis("N", "s", 4, 0.25)]
    g = rng.standard_normal((6, 5, 4))
    g2 = rng.standard_normal((6, 5, 4))
    phi = oracle.solve(g, axes, "fd")
    w = oracle.weights(axes)
    # gauge: weighted mean of phi is zero
    assert abs(np.sum(w * phi)) <= 1e-13 * np.sum(w * np.abs(phi))
    # residual of the compatible part
    assert oracle.residual_eta(g, phi, axes) <= 1e-15 * 10
    # linearity
    a, b = 1.7, -0.3
    assert np.allclose(oracle.solve(a * g + b * g2, axes, "fd"),
                       a * phi + b * oracle.solve(g2, axes, "fd"), atol=1e-12)
    # h-scaling: phi(c h) = c^2 phi(h)
    c = 3.0
    axes_c = [Axis(x.bc, x.grid, x.n, c * x.h) for x in axes]
    assert np.allclose(oracle.solve(g, axes_c, "fd"), c * c * phi, atol=1e-12)
    # axis permutation
    perm = (2, 0, 1)
    axes_p = [axes[p] for p in perm]
    phi_p = oracle.solve(np.transpose(g, perm), axes_p, "fd")
    assert np.allclose(phi_p, np.transpose(phi, perm), atol=1e-12)


def test_zero_mode_projection_equals_weighted_mean_removal():
    """Setting the zero-mode coefficient to zero solves for g minus its weighted mean."""
    axes = [Axis("N", "v", 7, 0.1), Axis("P", "v", 6, 0.1)]
    g = np.random.default_rng(9).standard_normal((7, 6)) + 3.0
    m = oracle.weighted_mean(g, axes)
    assert np.allclose(oracle.solve(g, axes, "fd"), oracle.solve(g - m, axes, "fd"), atol=1e-13)
    _, mult = oracle.lu_solve(g, axes)
    assert abs(mult - m) <= 1e-12 * abs(m)


def test_nonsingular_mode_zero_is_kept():
    """Dirichlet on one axis makes the problem nonsingular: a constant g has a nonzero solution."""
    axes = [Axis("D", "s", 5, 0.2), Axis("P", "v", 4, 0.2)]
    g = np.ones((5, 4))
    phi = oracle.solve(g, axes, "fd")
    ref, _ = oracle.lu_solve(g, axes)
    assert np.allclose(phi, ref, atol=1e-13) and np.max(np.abs(phi)) > 0.01


# ---------------------------------------------------------------- planted-mistake check
def test_a_planted_index_shift_is_caught(monkeypatch):
    """Shifting the Dirichlet-staggered FD eigenvalue index by one breaks the LU pin."""
    import importlib
    eigen = importlib.import_module("oracle.eigen")
    solve_mod = importlib.import_module("oracle.solve")
    orig = eigen.eigenvalues

    def shifted(bc, grid, n, h, approx):
        lam = orig(bc, grid, n, h, approx)
        if bc == "D" and grid == "s":
            return np.roll(lam, 1)
        return lam

    monkeypatch.setattr(solve_mod, "eigenvalues", shifted)
    axes = [Axis("D", "s", 6, 0.2)]
    g = np.random.default_rng(1).standard_normal(6)
    ref, _ = oracle.lu_solve(g, axes)
    assert np.max(np.abs(oracle.solve(g, axes, "fd") - ref)) > 1e-3 * np.max(np.abs(ref))


def test_generated_singular_rhs_are_compatible():
    """The seeded inputs of singular problems have zero weighted mean, so the
    solve does not have to project them (Neumann cube, 2D batch entries)."""
    import workloads
    d, g = workloads.neumann_blobs(24, seed=3)
    axes = oracle.axes_from(d["shape"], d["h"], d["bc"], d["grid"])
    assert abs(oracle.weighted_mean(g, axes)) <= 1e-15 * np.abs(g).max()
    for i, dd in enumerate(workloads.batch_2d(count=40, lo=5, hi=30, seed=4)):
        gi = workloads.batch_rhs(dd, i)
        if all(b in ("P", "N") for b in dd["bc"]):
            ax = oracle.axes_from(dd["shape"], dd["h"], dd["bc"], dd["grid"])
            assert abs(oracle.weighted_mean(gi, ax)) <= 1e-14, (i, dd)


# ---------------------------------------------------------------- mixed faces and the Helmholtz shift
@pytest.mark.parametrize("ns", [(1,), (2,), (5,), (3, 4), (4, 3, 2)])
def test_helmholtz_shift_matches_dense_lu(ns):
    """(L - sigma) phi = g: the transform solve with the shifted divisor equals the
    dense LU solve of the shifted stencil, for every kind combination including
    mixed faces; with sigma > 0 nothing is singular (no gauge row)."""
    rng = np.random.default_rng(100 + sum(ns))
    for axes in _all_axes_combos(ns):
        if any(not _valid(a.bc, a.grid, a.n) for a in axes):
            continue
        sigma = 3.7
        g = rng.standard_normal(ns)
        phi = oracle.solve(g, axes, "fd", shift=sigma)
        ref, mg = oracle.lu_solve(g, axes, shift=sigma)
        assert mg == 0.0
        assert np.max(np.abs(phi - ref)) <= 1e-11 * np.max(np.abs(ref)), [(a.bc, a.grid) for a in axes]
        assert oracle.residual_eta(g, phi, axes, shift=sigma) <= 1e-14


@pytest.mark.parametrize("bc,grid", KINDS + MIXED)
def test_helmholtz_ps_continuous_eigenfunction(bc, grid):
    """Pseudo-spectral (d2/dx2 - sigma) phi = g on a sampled eigenfunction: phi = g / (lambda - sigma)."""
    n, h, sigma = 9, 0.2, 2.5
    L = oracle.domain_length(bc, grid, n, h)
    x = oracle.grid_points(bc, grid, n, h)
    m = 0 if bc in ("DN", "ND") else (1 if bc != "D" else 2)
    g, lam = _eigfun(bc, grid, m, x, L)
    phi = oracle.solve(g, [Axis(bc, grid, n, h)], "ps", shift=sigma)
    assert np.allclose(phi, g / (lam - sigma), atol=1e-13 * np.max(np.abs(g)), rtol=0)


def test_mixed_face_closures_by_hand():
    """Boundary rows of the mixed-face stencil written out (h = 1): vertex Dirichlet-low /
    Neumann-high has rows [-2, 1, 0], [1, -2, 1], [0, 2, -2]; staggered has [-3, 1, 0]
    (Dirichlet face) and [0, 1, -1] (Neumann face); the reverse orientations mirror them."""
    dn_v = oracle.assemble_1d("DN", "v", 3, 1.0)
    assert np.array_equal(dn_v, np.array([[-2, 1, 0], [1, -2, 1], [0, 2, -2]], dtype=float))
    nd_v = oracle.assemble_1d("ND", "v", 3, 1.0)
    assert np.array_equal(nd_v, np.array([[-2, 2, 0], [1, -2, 1], [0, 1, -2]], dtype=float))
    dn_s = oracle.assemble_1d("DN", "s", 3, 1.0)
    assert np.array_equal(dn_s, np.array([[-3, 1, 0], [1, -2, 1], [0, 1, -1]], dtype=float))
    nd_s = oracle.assemble_1d("ND", "s", 3, 1.0)
    assert np.array_equal(nd_s, np.array([[-1, 1, 0], [1, -2, 1], [0, 1, -3]], dtype=float))
    # one unknown: vertex D|N closes with the Dirichlet node (0) on both sides of the mirror
    assert np.array_equal(oracle.assemble_1d("DN", "v", 1, 1.0), np.array([[-2.0]]))


def test_eigenmode_helper_matches_assembled_stencil():
    """The closed-form eigenpairs the longest-line GPU tests use are exact
    eigenpairs of the oracle's assembled 1D stencil, for every kind."""
    from eigenmodes import eigenpair
    from oracle.fd import assemble_1d
    for bc, grid in [("P", "v"), ("N", "v"), ("D", "v"), ("N", "s"), ("D", "s")]:
        for n in (5, 8, 9, 16):
            h = 0.37
            L = assemble_1d(bc, grid, n, h)
            for k in range(n):
                v, lam = eigenpair(bc, grid, n, k, h)
                assert np.linalg.norm(L @ v - lam * v) <= 1e-12 * max(abs(lam), 1.0) * np.linalg.norm(v), \
                    (bc, grid, n, k)
