"""Pins of the oracle's interstitial matrix elements (oracle/basis.c,
eq. (3.11)-(3.14)) against facts other than itself: the closed-form kinetic
term (3.14) against a finite-difference Laplacian of an independent
evaluation of the basis with scipy's harmonics, the same-atom overlap and
kinetic integrals (Gamma functions) by grid quadrature, linearity in the
potential, symmetry, and the nodes the spheres take away."""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle as O


def _real_sph(L, M, d):
    th = np.arccos(np.clip(d[:, 2], -1, 1))
    ph = np.arctan2(d[:, 1], d[:, 0])
    Y = sp.sph_harm_y(L, abs(M), th, ph) * (-1) ** abs(M)
    if M == 0:
        return Y.real
    return math.sqrt(2) * (Y.real if M > 0 else Y.imag)


def _phi_scipy(pts, c, shells):
    rv = pts - c
    r = np.linalg.norm(rv, axis=1)
    d = rv / r[:, None]
    cols = []
    for n, l, z in shells:
        for m in range(-l, l + 1):
            cols.append(r ** (n - 1) * np.exp(-z * r) * _real_sph(l, m, d))
    return np.array(cols).T


SHELLS = [(5, 0, 1.0), (6, 1, 2.0), (4, 2, 2.2), (5, 2, 2.6), (4, 3, 1.6), (2, 1, 0.8), (3, 0, 1.5)]


def test_kinetic_closed_form_matches_finite_differences():
    """(-1/2 Laplacian) phi from eq. (3.14) against central second differences
    (step 1e-3) of phi evaluated through scipy's harmonics"""
    rng = np.random.default_rng(61)
    c = np.array([0.2, -0.1, 0.3])
    pts = c + rng.normal(size=(25, 3)) * 1.5
    phi, tphi = O.basis_points(c[None], SHELLS, pts)
    h = 1e-3
    lap = -6.0 * _phi_scipy(pts, c, SHELLS)
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        lap += _phi_scipy(pts + e, c, SHELLS) + _phi_scipy(pts - e, c, SHELLS)
    lap /= h * h
    want = -0.5 * lap
    assert np.abs(phi - _phi_scipy(pts, c, SHELLS)).max() <= 1e-12 * np.abs(phi).max()
    err = np.abs(tphi - want)
    assert (err <= 1e-5 * np.abs(want) + 1e-6 * np.abs(want).max(axis=0)).all()


def _uniform(half, h):
    m = int(round(2 * half / h)) + 1
    return np.linspace(-half, half, m)


@pytest.mark.parametrize("shells", [[(4, 2, 2.2), (5, 2, 2.6)], [(6, 1, 2.0), (5, 1, 2.4)], [(4, 3, 1.6), (6, 0, 2.0)]])
def test_same_atom_overlap_and_kinetic_integrals(shells):
    """one atom, V = 0, no sphere: S and H tend to the same-atom integrals
    S = (n+n')!/a^(n+n'+1), T = 1/2 [(l(l+1) - n'(n'-1)) (n+n'-2)!/a^(n+n'-1)
    + 2 zeta' n' (n+n'-1)!/a^(n+n') - zeta'^2 (n+n')!/a^(n+n'+1)], a = zeta + zeta',
    for equal (l, m), and 0 between different (l, m)"""
    x = _uniform(13.0, 0.25)
    c = np.array([[0.125, 0.125, 0.125]])   # no node at the centre
    S, H = O.matrix_elements([x, x, x], np.zeros((len(x),) * 3), c, [0.0], shells)
    idx = [(n, l, z, m) for n, l, z in shells for m in range(-l, l + 1)]
    Sw = np.zeros_like(S)
    Tw = np.zeros_like(S)
    for a, (n, l, z, m) in enumerate(idx):
        for b, (n2, l2, z2, m2) in enumerate(idx):
            if (l, m) != (l2, m2):
                continue
            al = z + z2
            Sw[a, b] = math.factorial(n + n2) / al ** (n + n2 + 1)
            Tw[a, b] = 0.5 * ((l * (l + 1) - n2 * (n2 - 1)) * math.factorial(n + n2 - 2) / al ** (n + n2 - 1)
                              + 2 * z2 * n2 * math.factorial(n + n2 - 1) / al ** (n + n2)
                              - z2 * z2 * math.factorial(n + n2) / al ** (n + n2 + 1))
    Tw = 0.5 * (Tw + Tw.T)
    scale = np.sqrt(np.outer(np.diag(Sw), np.diag(Sw)))
    assert np.abs(S - Sw).max() / scale.max() < 1e-5
    assert (np.abs(S - Sw) / scale).max() < 1e-4
    assert (np.abs(H - Tw) / scale).max() < 1e-3
    assert np.array_equal(S, S.T) and np.array_equal(H, H.T)


def test_potential_enters_linearly_and_spheres_remove_nodes():
    """H(V = c) - H(V = 0) = c S; a sphere of radius 2h about a node removes
    the 27 nodes with |x - C|^2 < 4 h^2 from both sums"""
    h = 0.5
    x = np.arange(-8, 9) * h
    shells = [(4, 2, 2.2), (6, 1, 2.0)]
    c = np.array([[0.0, 0.0, 0.0], [1.5, -1.0, 0.5]])
    r = np.array([2 * h, 0.6])
    zero = np.zeros((17, 17, 17))
    S0, H0 = O.matrix_elements([x, x, x], zero, c, r, shells)
    S1, H1 = O.matrix_elements([x, x, x], zero + 0.7, c, r, shells)
    assert np.array_equal(S0, S1)
    assert np.abs((H1 - H0) - 0.7 * S0).max() <= 1e-12 * np.abs(S0).max()
    # the 27 nodes of the first sphere (and the second's), one by one
    Sf, Hf = O.matrix_elements([x, x, x], zero, c, np.zeros(2), shells)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    d0 = X ** 2 + Y ** 2 + Z ** 2 < 4 * h * h
    d1 = (X - 1.5) ** 2 + (Y + 1.0) ** 2 + (Z - 0.5) ** 2 < 0.36
    assert d0.sum() == 27
    gone = d0 | d1
    pts = np.stack([X[gone], Y[gone], Z[gone]], axis=1)
    phi, _ = O.basis_points(c, shells, pts)
    w = np.full(len(pts), h ** 3)
    assert np.abs((Sf - S0) - (phi * w[:, None]).T @ phi).max() <= 1e-12 * np.abs(Sf).max()
