"""Pins of the oracle's interstitial output density (oracle/basis.c) against
facts other than itself: the closed-form norm of a Slater-type function
(int phi^2 = (2n)!/(2 zeta)^(2n+1)) by grid quadrature, an independent
evaluation of the orbitals with scipy's harmonics, invariance of the density
under an orthogonal mix of equally occupied states, and the nodes the
spheres take away."""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle as O

SHELLS = [(5, 0, 1.0), (6, 0, 2.0), (5, 1, 1.0), (6, 1, 2.0), (4, 2, 2.2), (5, 2, 2.6), (4, 3, 1.6)]   # Table 1


def _real_sph(L, M, d):
    th = np.arccos(np.clip(d[:, 2], -1, 1))
    ph = np.arctan2(d[:, 1], d[:, 0])
    Y = sp.sph_harm_y(L, abs(M), th, ph) * (-1) ** abs(M)
    if M == 0:
        return Y.real
    return math.sqrt(2) * (Y.real if M > 0 else Y.imag)


def _scipy_basis(pts, centers, shells):
    cols = []
    for c in centers:
        r_vec = pts - c
        r = np.linalg.norm(r_vec, axis=1)
        d = r_vec / r[:, None]
        for n, l, z in shells:
            for m in range(-l, l + 1):
                cols.append(r ** (n - 1) * np.exp(-z * r) * _real_sph(l, m, d))
    return np.array(cols).T    # [npts][n_basis]


@pytest.mark.parametrize("shell", [(5, 0, 1.0), (5, 1, 1.0), (4, 2, 2.2), (4, 3, 1.6), (6, 1, 2.0)])
def test_slater_norm_by_grid_quadrature(shell):
    """one state, one basis function: int rho = int phi^2 = (2n)!/(2 zeta)^(2n+1)
    (radial Gamma integral; the angular factor is 1 for orthonormal y_lm), by
    the grid rule sum vol_n rho_n on a uniform box large enough for the tail"""
    n, l, z = shell
    half = 30.0 / z + 4
    h = 0.3 / max(z, 1.0) * 1.5
    m = int(2 * half / h) | 1
    x = np.linspace(-half, half, m)
    nb = 2 * l + 1
    errs = []
    for mm in (0, nb - 1):
        coef = np.zeros((nb, 1))
        coef[mm, 0] = 1.0
        rho = O.interstitial_density([x, x, x], np.zeros((1, 3)), [0.0], [shell], coef, [1.0])
        w = np.full(m, x[1] - x[0])
        w[0] = w[-1] = 0.5 * (x[1] - x[0])
        total = np.einsum("k,j,i,kji->", w, w, w, rho)
        want = math.factorial(2 * n) / (2 * z) ** (2 * n + 1)
        errs.append(abs(total - want) / want)
    assert max(errs) < 1e-6, errs


def test_orbitals_match_scipy_harmonics():
    rng = np.random.default_rng(41)
    centers = np.array([[0.3, -0.2, 0.1], [3.9, 1.1, -2.0]])
    nb = 2 * sum(2 * l + 1 for _, l, _ in SHELLS)
    n_occ = 5
    coef = rng.normal(size=(nb, n_occ))
    occ = rng.uniform(0.5, 2.0, n_occ)
    pts = rng.uniform(-5, 7, size=(40, 3))
    got = O.density_points(centers, SHELLS, coef, occ, pts)
    Phi = _scipy_basis(pts, centers, SHELLS)
    psi = Phi @ coef
    want = (psi * psi) @ occ
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_density_invariant_under_state_rotation():
    """equal occupations: C -> C Q (Q orthogonal) leaves sum_k psi_k^2 unchanged"""
    rng = np.random.default_rng(42)
    centers = np.array([[0.0, 0.0, 0.0], [2.5, -1.0, 1.5], [-2.0, 2.0, 0.5]])
    nb = 3 * sum(2 * l + 1 for _, l, _ in SHELLS)
    coef = rng.normal(size=(nb, 6))
    Q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
    pts = rng.uniform(-4, 4, size=(30, 3))
    a = O.density_points(centers, SHELLS, coef, np.full(6, 2.0), pts)
    b = O.density_points(centers, SHELLS, coef @ Q, np.full(6, 2.0), pts)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    # unequal occupations break it
    occ = np.array([2.0, 2.0, 1.0, 0.5, 2.0, 0.0])
    c = O.density_points(centers, SHELLS, coef, occ, pts)
    d = O.density_points(centers, SHELLS, coef @ Q, occ, pts)
    assert np.abs(c - d).max() > 1e-3 * np.abs(c).max()


def test_interstitial_density_zero_inside_spheres():
    """uniform h = 0.5: a sphere of radius 2h about a node zeroes exactly the
    27 nodes with |x - C|^2 < 4 h^2; elsewhere the grid values are the
    point values"""
    h = 0.5
    x = np.arange(-4, 5) * h
    rng = np.random.default_rng(43)
    shells = [(5, 0, 1.0), (4, 2, 2.2)]
    coef = rng.normal(size=(6, 2))
    occ = [2.0, 1.0]
    c = np.array([[0.0, 0.0, 0.0]])
    rho = O.interstitial_density([x, x, x], c, [2 * h], shells, coef, occ)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    inside = X * X + Y * Y + Z * Z < 4 * h * h
    assert inside.sum() == 27
    assert np.all(rho[inside] == 0.0)
    pts = np.stack([X[~inside], Y[~inside], Z[~inside]], axis=1)
    assert np.array_equal(rho[~inside], O.density_points(c, shells, coef, occ, pts))
    assert np.all(rho[~inside] > 0)
