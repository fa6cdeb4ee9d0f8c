"""Dense matrices of the discrete transforms (test infrastructure only).

Each function returns the n x n matrix T with  fhat = T @ f  for the
transform named, written straight from its definition:

* DFT / IDFT        -- Eqs. (5)-(6) of Section 2.1: the forward transform
  carries the 1/n factor, the inverse is unscaled.
* DST-I/II/III, DCT-I/II/III -- Table 1 (unnormalised sums).
* DST-IV, DCT-IV -- not in Table 1; written in the same unnormalised form
  (2 sum_j f_j sin / cos(pi (j+1/2)(k+1/2)/n)).  They are the transforms of
  a staggered axis with a Dirichlet condition on one face and a Neumann
  condition on the other (a combination beyond the paper's Table 2).

``forward_backward`` pairs them with a boundary condition and grid as in
Table 2, including the scale factor in front of each backward transform;
an axis with different conditions on its two faces ("DN": Dirichlet at the
low end, Neumann at the high end, or "ND") gets the transform whose basis
vectors are the sampled eigenfunctions sin / cos((k+1/2) pi x/L) of that
axis, with the same backward factor convention.

Angles are formed from exact integer products reduced modulo their period
before the single multiplication by pi, so every entry is the correctly
rounded value of its definition to within one or two ulps.
"""

import numpy as np

# (bc, grid) pairs with a transform of their own; periodic axes ignore the grid.
# "DN" / "ND": different conditions on the low and high face of the axis.
KINDS = (("P", "v"), ("D", "v"), ("D", "s"), ("N", "v"), ("N", "s"),
         ("DN", "v"), ("DN", "s"), ("ND", "v"), ("ND", "s"))


def _sinpi(num, den):
    """sin(pi * num / den) for integer arrays num and a positive integer den."""
    num = np.mod(np.asarray(num, dtype=np.int64), 2 * den)
    return np.sin(np.pi * num.astype(np.float64) / den)


def _cospi(num, den):
    """cos(pi * num / den) for integer arrays num and a positive integer den."""
    num = np.mod(np.asarray(num, dtype=np.int64), 2 * den)
    return np.cos(np.pi * num.astype(np.float64) / den)


def _kj(n):
    k = np.arange(n, dtype=np.int64)[:, None]
    j = np.arange(n, dtype=np.int64)[None, :]
    return k, j


def dst1(n):
    """Table 1, DST-I: 2 sum_j f_j sin(pi (j+1)(k+1)/(n+1))."""
    k, j = _kj(n)
    return 2.0 * _sinpi((j + 1) * (k + 1), n + 1)


def dst2(n):
    """Table 1, DST-II: 2 sum_j f_j sin(pi (j+1/2)(k+1)/n)."""
    k, j = _kj(n)
    return 2.0 * _sinpi((2 * j + 1) * (k + 1), 2 * n)


def dst3(n):
    """Table 1, DST-III: (-1)^k f_{n-1} + 2 sum_{j<n-1} f_j sin(pi (j+1)(k+1/2)/n)."""
    k, j = _kj(n)
    t = 2.0 * _sinpi((j + 1) * (2 * k + 1), 2 * n)
    t[:, n - 1] = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return t


def dct1(n):
    """Table 1, DCT-I: f_0 + (-1)^k f_{n-1} + 2 sum_{0<j<n-1} f_j cos(pi j k/(n-1)).  n >= 2."""
    if n < 2:
        raise ValueError("DCT-I needs n >= 2")
    k, j = _kj(n)
    t = 2.0 * _cospi(j * k, n - 1)
    t[:, 0] = 1.0
    t[:, n - 1] = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return t


def dct2(n):
    """Table 1, DCT-II: 2 sum_j f_j cos(pi (j+1/2) k/n)."""
    k, j = _kj(n)
    return 2.0 * _cospi((2 * j + 1) * k, 2 * n)


def dct3(n):
    """Table 1, DCT-III: f_0 + 2 sum_{j>0} f_j cos(pi j (k+1/2)/n)."""
    k, j = _kj(n)
    t = 2.0 * _cospi(j * (2 * k + 1), 2 * n)
    t[:, 0] = 1.0
    return t


def dst4(n):
    """DST-IV, unnormalised like Table 1: 2 sum_j f_j sin(pi (j+1/2)(k+1/2)/n)."""
    k, j = _kj(n)
    return 2.0 * _sinpi((2 * j + 1) * (2 * k + 1), 4 * n)


def dct4(n):
    """DCT-IV, unnormalised like Table 1: 2 sum_j f_j cos(pi (j+1/2)(k+1/2)/n)."""
    k, j = _kj(n)
    return 2.0 * _cospi((2 * j + 1) * (2 * k + 1), 4 * n)


def dft_matrix(n):
    """Eq. (6): fhat_k = (1/n) sum_j f_j exp(-2 pi i k j/n)."""
    k, j = _kj(n)
    ang = np.mod(k * j, n).astype(np.float64) * (2.0 * np.pi / n)
    return (np.cos(ang) - 1j * np.sin(ang)) / n


def idft_matrix(n):
    """Eq. (5): f_j = sum_k fhat_k exp(+2 pi i k j/n); rows index j."""
    k, j = _kj(n)
    ang = np.mod(k * j, n).astype(np.float64) * (2.0 * np.pi / n)
    return np.cos(ang) + 1j * np.sin(ang)


_TABLE1 = {"DST-I": dst1, "DST-II": dst2, "DST-III": dst3, "DST-IV": dst4,
           "DCT-I": dct1, "DCT-II": dct2, "DCT-III": dct3, "DCT-IV": dct4,
           "DFT": dft_matrix, "IDFT": idft_matrix}


def transform_matrix(name, n):
    """The matrix of a named transform (Table 1 names, or DFT / IDFT)."""
    return _TABLE1[name](n)


def forward_backward(bc, grid, n):
    """Table 2: (forward matrix, backward matrix) for one axis.

    bc is 'P', 'D' or 'N'; grid is 'v' (the paper's regular grid) or 's'
    (staggered); the grid is irrelevant for periodic axes.  The backward
    matrix includes the factor printed in front of the backward transform,
    so that backward @ forward is the identity.
    """
    if bc == "P":
        return dft_matrix(n), idft_matrix(n)
    if bc == "D" and grid == "v":
        return dst1(n), dst1(n) / (2.0 * (n + 1))
    if bc == "D" and grid == "s":
        return dst2(n), dst3(n) / (2.0 * n)
    if bc == "N" and grid == "v":
        return dct1(n), dct1(n) / (2.0 * (n - 1))
    if bc == "N" and grid == "s":
        return dct2(n), dct3(n) / (2.0 * n)
    # Different conditions on the two faces.  Vertex grid, Dirichlet low /
    # Neumann high: unknowns at x = (j+1) h, j < n (the Neumann node x = L = n h
    # included); the eigenvectors sin((k+1/2) pi (j+1)/n) are orthogonal with
    # weight 1/2 on that end node, which makes the forward transform the
    # DST-III of Table 1 and its inverse the DST-II.  Neumann low / Dirichlet
    # high: unknowns at x = j h, cos((k+1/2) pi j/n), weight 1/2 at x = 0:
    # DCT-III forward, DCT-II backward.  Staggered: DST-IV / DCT-IV, each its
    # own inverse up to 1/(2n).
    if bc == "DN" and grid == "v":
        return dst3(n), dst2(n) / (2.0 * n)
    if bc == "ND" and grid == "v":
        return dct3(n), dct2(n) / (2.0 * n)
    if bc == "DN" and grid == "s":
        return dst4(n), dst4(n) / (2.0 * n)
    if bc == "ND" and grid == "s":
        return dct4(n), dct4(n) / (2.0 * n)
    raise ValueError(f"unknown boundary condition / grid {bc!r}/{grid!r}")
