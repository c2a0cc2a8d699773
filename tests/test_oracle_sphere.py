"""Pins of the oracle's sphere part (oracle/sphere.c) against facts other than
itself: numpy's Gauss-Legendre rule, quadrature exactness for harmonics,
tricubic exactness on cubic fields, closed-form potentials of Gaussian,
hydrogen-like and polynomial densities inside a sphere (eq. (3.4) under the
literal sign of (3.2)), the fourth-order convergence of the radial rule, the
Coulomb self-energy of a Gaussian, and lattice-point counts for the nodes
the grid part of the energy leaves to the spheres."""
import math

import numpy as np
import pytest
import scipy.special as sp

SQ4PI = math.sqrt(4.0 * math.pi)
R_MIN = 1e-5


def lm_of(L, M):
    return L * L + L + M


def test_rule_is_gauss_legendre_times_uniform_azimuths(oracle_mod):
    for nt, nph in ((8, 9), (5, 9), (3, 4)):
        d, w = oracle_mod.sphere_rule(nt, nph)
        t, wt = np.polynomial.legendre.leggauss(nt)
        dd = d.reshape(nt, nph, 3)
        assert np.abs(dd[:, :, 2] - t[:, None]).max() < 1e-14
        ph = 2 * np.pi * (np.arange(nph) + 0.5) / nph
        st = np.sqrt(1 - t * t)
        assert np.abs(dd[:, :, 0] - st[:, None] * np.cos(ph)[None]).max() < 1e-14
        assert np.abs(dd[:, :, 1] - st[:, None] * np.sin(ph)[None]).max() < 1e-14
        assert np.abs(w.reshape(nt, nph) - wt[:, None] * 2 * np.pi / nph).max() < 1e-14


def _real_sph(L, M, d):
    """real orthonormal harmonic from scipy's complex one, no Condon-Shortley phase"""
    th = np.arccos(np.clip(d[:, 2], -1, 1))
    ph = np.arctan2(d[:, 1], d[:, 0])
    Y = sp.sph_harm_y(L, abs(M), th, ph) * (-1) ** abs(M)
    if M == 0:
        return Y.real
    return math.sqrt(2) * (Y.real if M > 0 else Y.imag)


@pytest.mark.parametrize("nt,nph,exact", [(8, 9, True), (5, 9, True), (8, 8, False), (4, 9, False)])
def test_projection_recovers_harmonics(oracle_mod, nt, nph, exact):
    """eq. (3.6) on sampled sums of scipy harmonics: exact for L <= 4 with
    n_theta >= 5 and n_phi >= 9; eight azimuths alias M = +-4 into each other,
    four Legendre nodes cannot integrate degree-8 products."""
    d, _ = oracle_mod.sphere_rule(nt, nph)
    rng = np.random.default_rng(3)
    a = rng.normal(size=(2, 25))
    vals = np.zeros((2, len(d)))
    for L in range(5):
        for M in range(-L, L + 1):
            vals += a[:, lm_of(L, M), None] * _real_sph(L, M, d)[None]
    got = oracle_mod.sphere_project(vals, nt, nph)
    err = np.abs(got - a).max()
    if exact:
        assert err < 1e-13
    else:
        assert err > 1e-3
    if exact:
        # degree 5 with |M| <= 4 is orthogonal to every L <= 4 harmonic under the rule
        v5 = sum(_real_sph(5, M, d) for M in range(-4, 5))[None]
        assert np.abs(oracle_mod.sphere_project(v5, nt, nph)).max() < 1e-13


def test_projection_of_interpolated_cubic_fields(oracle_mod):
    """Solid harmonics of degree <= 3 about each centre are cubic in every
    coordinate, so tricubic interpolation reproduces them; the projection of
    r^l y_lm(x - C_a) on the sphere of atom a is then R_a^l (and 0 elsewhere)."""
    rng = np.random.default_rng(5)
    xs = []
    for n in (23, 19, 21):
        h = rng.uniform(0.5, 1.5, n - 1)
        xs.append(-6 + 12 * np.concatenate([[0], np.cumsum(h)]) / h.sum())
    centers = np.array([[0.3, -0.4, 0.5], [-1.1, 1.2, -0.7]])
    radii = np.array([2.3, 1.7])
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    d, _ = oracle_mod.sphere_rule(8, 9)
    for (L, M) in ((0, 0), (1, -1), (2, 1), (3, -2), (3, 3)):
        lm = lm_of(L, M)
        vals = []
        for a in range(2):
            f = np.zeros(X.shape)
            for idx in np.ndindex(X.shape):
                f[idx] = oracle_mod.solid_harmonics(X[idx] - centers[a, 0], Y[idx] - centers[a, 1],
                                                    Z[idx] - centers[a, 2])[lm]
            v = np.ascontiguousarray(f.transpose(2, 1, 0))   # [z][y][x]
            pts = oracle_mod.sphere_points(centers[a:a + 1], radii[a:a + 1], d)
            vals.append(oracle_mod.interp(xs, v, pts))
        got = oracle_mod.sphere_project(np.array(vals), 8, 9)
        want = np.zeros((2, 25))
        want[:, lm] = radii ** L
        assert np.abs(got - want).max() < 1e-11 * max(1, radii.max() ** L), (L, M)


# ------------------------------------------------------------ radial solve
import oracle as O   # noqa: E402


def _core_gauss(n, Z=46.0, zeta=46.0, q=10.0, w=0.5, R=2.5):
    """hydrogen-like core of Z electrons (zeta^3/pi) exp(-2 zeta r), a
    Gaussian of q electrons, a nucleus of charge Z; exact potential under
    Laplacian(V) = 4 pi (rho - Z delta)"""
    r = O.radial_mesh(R, R_MIN, n)
    rho = np.zeros((1, 25, n))
    rho[0, 0] = SQ4PI * (Z * zeta ** 3 / math.pi * np.exp(-2 * zeta * r) + q * (math.pi * w * w) ** -1.5 * np.exp(-(r / w) ** 2))

    def V(r):
        return -q * sp.erf(r / w) / r + Z * (1 / r + zeta) * np.exp(-2 * zeta * r)

    vR = np.zeros((1, 25))
    vR[0, 0] = SQ4PI * V(R)
    got = O.sphere_radial([R], [Z], R_MIN, vR, rho)[0, 0]
    want = SQ4PI * V(r)
    return np.abs(got - want).max() / np.abs(want).max()


def test_radial_core_and_gaussian_closed_form():
    """With a nucleus: the delta_L0 Z (1/r - 1/R) term, the P and Q integrals
    and the boundary term together reproduce -q erf(r/w)/r + Z (1/r + zeta)
    exp(-2 zeta r); the error falls by ~16 per halving of the log step."""
    e1, e2 = _core_gauss(215), _core_gauss(429)
    assert e2 < 1e-10
    assert e1 / e2 > 12


def _lterm(n, L, M, c=0.7, R=2.5):
    r = O.radial_mesh(R, R_MIN, n)
    lm = lm_of(L, M)
    rho = np.zeros((1, 25, n))
    rho[0, lm] = c * r ** L * np.exp(-r * r)
    x = r * r
    g = sp.gammainc(L + 1.5, x) * sp.gamma(L + 1.5)
    want = -(4 * math.pi * c / (2 * L + 1)) * (r ** -(L + 1) * 0.5 * g + r ** L * 0.5 * np.exp(-x))
    vR = np.zeros((1, 25))
    vR[0, lm] = want[-1]
    out = O.sphere_radial([R], [0.0], R_MIN, vR, rho)[0]
    others = np.delete(out, lm, axis=0)
    assert np.abs(others).max() == 0.0
    return np.abs(out[lm] - want).max() / np.abs(want).max()


@pytest.mark.parametrize("L,M", [(1, -1), (2, 2), (3, 0), (4, -3)])
def test_radial_gaussian_multipole_closed_form(L, M):
    """rho_LM = c r^L exp(-r^2): V_LM = -(4 pi c/(2L+1)) [r^-(L+1) gamma(L+3/2, r^2)/2
    + r^L exp(-r^2)/2] (the free-space potential; its value at R is the
    Dirichlet datum). Fourth order in the log step."""
    e1, e2 = _lterm(215, L, M), _lterm(429, L, M)
    assert e2 < 2e-5
    assert e1 / e2 > 10


def test_radial_every_lm_takes_its_degree():
    """each of the 25 entries solves with its own L (index L*L + L + M)"""
    for L in range(5):
        for M in range(-L, L + 1):
            assert _lterm(429, L, M) < 2e-5, (L, M)


@pytest.mark.parametrize("r_min,tol", [(R_MIN, 2e-4), (0.3, 1e-7)])
@pytest.mark.parametrize("L", [0, 1, 2, 4])
def test_radial_polynomial_density_zero_boundary(L, r_min, tol):
    """rho_LM = r^L with V(R) = 0: V = 4 pi (r^(L+2) - R^2 r^L)/(4L + 6),
    since Laplacian(r^(L+2) y) = (4L+6) r^L y. The integrand grows like
    exp((2L+3) t) on the log mesh, so the rule's constant grows with L. With
    r_min = 0.3 the step is small and the piece [0, r_0] (exact here, rho ~ r^L)
    and the first interval weigh in."""
    R = 2.5

    def err(n):
        r = O.radial_mesh(R, r_min, n)
        rho = np.zeros((1, 25, n))
        rho[0, lm_of(L, 0)] = r ** L
        got = O.sphere_radial([R], [0.0], r_min, np.zeros((1, 25)), rho)[0, lm_of(L, 0)]
        want = 4 * math.pi * (r ** (L + 2) - R * R * r ** L) / (4 * L + 6)
        return np.abs(got - want).max() / np.abs(want).max()

    e1, e2 = err(215), err(429)
    assert e2 < tol
    assert e1 / e2 > 10


def test_radial_boundary_value_and_mesh():
    """r_0 = r_min, r_(n-1) = R, uniform in ln r; V_LM(R) is the Dirichlet datum."""
    R, n = 2.3, 429
    r = O.radial_mesh(R, R_MIN, n)
    assert abs(r[0] - R_MIN) < 1e-18 and abs(r[-1] - R) < 1e-15
    assert np.abs(np.diff(np.log(r)) - math.log(R / R_MIN) / (n - 1)).max() < 1e-12
    rng = np.random.default_rng(8)
    rho = rng.normal(size=(2, 25, n)) * np.exp(-r)[None, None]
    vR = rng.normal(size=(2, 25))
    out = O.sphere_radial([R, R], [3.0, 0.0], R_MIN, vR, rho)
    assert np.abs(out[:, :, -1] - vR).max() < 1e-12 * np.abs(vR).max() + 1e-12
    # linear in (V(R), rho, Z)
    out2 = O.sphere_radial([R, R], [6.0, 0.0], R_MIN, 2 * vR, 2 * rho)
    assert np.abs(out2 - 2 * out).max() < 1e-12 * np.abs(out).max()


# ----------------------------------------------------------------- energy
def test_sphere_energy_gaussian_self_energy():
    """int V rho dV for a Gaussian charge and its own potential is twice the
    Coulomb self-energy, -2 q^2 / (sqrt(2 pi) w) under eq. (3.2)'s sign (the
    tail beyond R = 5w is below 1e-10 of it)."""
    q, w, R = 10.0, 0.5, 2.5
    for n, tol in ((215, 1e-8), (429, 1e-10)):
        r = O.radial_mesh(R, R_MIN, n)
        rho = np.zeros((1, 25, n))
        v = np.zeros((1, 25, n))
        rho[0, 0] = SQ4PI * q * (math.pi * w * w) ** -1.5 * np.exp(-(r / w) ** 2)
        v[0, 0] = SQ4PI * (-q * sp.erf(r / w) / r)
        e = O.sphere_energy([R], R_MIN, v, rho)[0]
        assert abs(e + 2 * q * q / (math.sqrt(2 * math.pi) * w)) < tol * 2 * q * q / w


def test_sphere_energy_sums_lm_products():
    """orthonormal y_LM: the angular integral of V rho is sum_LM V_LM rho_LM;
    with V_LM = rho_LM = r on one LM: int_0^R r^4 dr = R^5/5 (to the rule's
    fourth-order error in the log step)."""
    R = 2.0

    def err(n, lm):
        r = O.radial_mesh(R, R_MIN, n)
        f = np.zeros((1, 25, n))
        f[0, lm] = r
        return abs(O.sphere_energy([R], R_MIN, f, f)[0] - R ** 5 / 5) / (R ** 5 / 5)

    for lm in (0, 7, 24):
        e1, e2 = err(215, lm), err(429, lm)
        assert e2 < 1e-5 and e1 / e2 > 8
    # constant V_00 rho_00 = 1 from r_min = 0.3: int_0^R r^2 dr = R^3/3, the
    # piece [0, r_0] (r_0^3/3) exact
    n, r_min = 429, 0.3
    f = np.zeros((1, 25, n))
    f[0, 0] = 1.0
    assert abs(O.sphere_energy([R], r_min, f, f)[0] - R ** 3 / 3) < 1e-8 * R ** 3 / 3


def test_grid_energy_without_spheres_is_box_volume():
    """dual widths telescope: sum of vol_n over all nodes = box volume"""
    rng = np.random.default_rng(9)
    xs = [np.sort(rng.uniform(-3, 4, n)) for n in (9, 7, 8)]
    shape = (8, 7, 9)
    one = np.ones(shape)
    e = O.energy_grid(xs, one, one, np.zeros((0, 3)), np.zeros(0))
    vol = np.prod([x[-1] - x[0] for x in xs])
    assert abs(e - vol) < 1e-12 * vol
    # and it is bilinear in (v, rho)
    v = rng.normal(size=shape)
    rho = rng.normal(size=shape)
    e1 = O.energy_grid(xs, v, rho, np.zeros((0, 3)), np.zeros(0))
    e2 = O.energy_grid(xs, 2 * v + 1, rho, np.zeros((0, 3)), np.zeros(0))
    e3 = O.energy_grid(xs, one, rho, np.zeros((0, 3)), np.zeros(0))
    assert abs(e2 - (2 * e1 + e3)) < 1e-12 * (abs(e1) + abs(e3)) * 4


def test_grid_energy_leaves_lattice_ball_to_sphere():
    """uniform h = 0.5 (exact binary squares): a sphere of radius 2h about a
    node takes the 27 nodes with |x - C|^2 < 4 h^2 (1 + 6 + 12 + 8; the 6 at
    distance exactly 2h stay outside); a sphere of radius 1.5 h about a cell
    centre takes the 8 corners of that cell (|d|^2 = 3/4 h^2; the next nodes
    lie at 11/4 h^2)."""
    h = 0.5
    x = np.arange(-8, 9) * h
    xs = [x, x, x]
    one = np.ones((17, 17, 17))
    full = O.energy_grid(xs, one, one, np.zeros((0, 3)), np.zeros(0))
    e = O.energy_grid(xs, one, one, np.array([[0.0, 0.0, 0.0]]), np.array([2 * h]))
    assert abs((full - e) / h ** 3 - 27) < 1e-12
    c2 = np.array([[1.25, 1.25, 1.25]])
    e2 = O.energy_grid(xs, one, one, c2, np.array([1.5 * h]))
    assert abs((full - e2) / h ** 3 - 8) < 1e-12


# ------------------------------------------------- tabulated density terms
def _real_sph(L, M, d):
    th = np.arccos(np.clip(d[:, 2], -1, 1))
    ph = np.arctan2(d[:, 1], d[:, 0])
    Y = sp.sph_harm_y(L, abs(M), th, ph) * (-1) ** abs(M)
    if M == 0:
        return Y.real
    return math.sqrt(2) * (Y.real if M > 0 else Y.imag)


def test_density_terms_exact_for_cubics_in_log_r():
    """rho_LM(r) = p_LM(ln r), p cubic: the four-point Lagrange interpolant in
    ln r reproduces it, so the grid term is sum_LM p_LM(ln r) y_LM (scipy's
    harmonics) at every node inside the sphere with r >= r_0; below r_0 it is
    rho_LM(r_0) (r/r_0)^L y_LM; nodes outside are untouched; lmin drops L < lmin"""
    rng = np.random.default_rng(91)
    x = np.linspace(-3, 3, 25) + 0.013
    xs = [x, x + 0.007, x - 0.011]
    c = np.array([[0.0, 0.0, 0.0]])
    R, r_min, n = 2.2, 0.3, 40
    coef = rng.normal(size=(25, 4))
    r = O.radial_mesh(R, r_min, n)
    t = np.log(r)
    tab = np.zeros((1, 25, n))
    for lm in range(25):
        tab[0, lm] = coef[lm, 0] + coef[lm, 1] * t + coef[lm, 2] * t * t + coef[lm, 3] * t ** 3
    base = rng.normal(size=(25, 25, 25))
    for lmin in (0, 1, 2):
        rho = base.copy()
        O.sphere_density_terms(xs, c, [R], r_min, tab, lmin, rho)
        Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
        d2 = X * X + Y * Y + Z * Z
        inside = d2 < R * R
        assert np.array_equal(rho[~inside], base[~inside])
        pts = np.stack([X[inside], Y[inside], Z[inside]], axis=1)
        rr = np.sqrt((pts ** 2).sum(1))
        dirs = pts / rr[:, None]
        want = np.zeros(len(pts))
        for L in range(lmin, 5):
            for M in range(-L, L + 1):
                lm = L * L + L + M
                p = coef[lm, 0] + coef[lm, 1] * np.log(rr) + coef[lm, 2] * np.log(rr) ** 2 + coef[lm, 3] * np.log(rr) ** 3
                below = rr < r[0]
                p[below] = tab[0, lm, 0] * (rr[below] / r[0]) ** L
                want += p * _real_sph(L, M, dirs)
        got = rho[inside] - base[inside]
        assert (rr < r[0]).any() and (rr >= r[0]).any()
        assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def test_density_terms_match_gaussian_multipoles():
    """the synthetic sphere densities' l-terms c r^l exp(-r^2), tabulated on
    429 points and put back on the grid, agree with the analytic
    c S_lm exp(-r^2) to the interpolation error (for r^4 the samples grow
    like exp(4 t): (4 D)^4 / 24 with D = 0.029, about 2e-5)"""
    rng = np.random.default_rng(92)
    x = np.linspace(-3, 3, 31)
    c = np.array([[0.05, -0.02, 0.03]])
    R, r_min, n = 2.5, 1e-5, 429
    r = O.radial_mesh(R, r_min, n)
    cl = rng.normal(size=24) * 0.3
    tab = np.zeros((1, 25, n))
    for lm in range(1, 25):
        L = int(math.isqrt(lm))
        tab[0, lm] = cl[lm - 1] * r ** L * np.exp(-r * r)
    rho = np.zeros((31, 31, 31))
    O.sphere_density_terms([x, x, x], c, [R], r_min, tab, 1, rho)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    want = np.zeros_like(rho)
    for idx in np.ndindex(rho.shape):
        dx, dy, dz = X[idx] - c[0, 0], Y[idx] - c[0, 1], Z[idx] - c[0, 2]
        if dx * dx + dy * dy + dz * dz < R * R:
            S = O.solid_harmonics(dx, dy, dz)
            want[idx] = (cl * S[1:]).sum() * math.exp(-(dx * dx + dy * dy + dz * dz))
    assert np.abs(rho - want).max() <= 3e-5 * np.abs(want).max()


def test_density_terms_window_is_centred():
    """a table that is 1 at one mesh index k and 0 elsewhere: at a node half
    way between r_k and r_(k+1) the interpolant uses the window k-1..k+2 and
    returns the Lagrange weight of its second node at u = 1.5, 9/16 (a window
    starting at k would give 5/16)"""
    R, r_min, n, k = 2.0, 0.1, 30, 12
    r = O.radial_mesh(R, r_min, n)
    rk = math.sqrt(r[k] * r[k + 1])   # t half way
    x = np.array([-2.5, -1.0, 0.0, rk, 2.5])
    xs = [x, np.array([-2.5, -1.0, 0.0, 1.0, 2.5]), np.array([-2.5, -1.0, 0.0, 1.0, 2.5])]
    tab = np.zeros((1, 25, n))
    tab[0, 0, k] = 1.0
    rho = np.zeros((5, 5, 5))
    O.sphere_density_terms(xs, np.zeros((1, 3)), [R], r_min, tab, 0, rho)
    y00 = 0.5 / math.sqrt(math.pi)
    assert abs(rho[2, 2, 3] - 9.0 / 16.0 * y00) <= 1e-12
