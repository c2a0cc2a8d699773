"""CPU oracle for the LASTO Hartree step -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C (``oracle.c``, ``sphere.c``, ``basis.c``) behind ctypes. Only ``tests/``, the smoke check
and the benchmark's CPU-baseline leg may import this package. The GPU path
(``paper_0806_1723_amd``) never imports it and shares no code with it.

``build()`` compiles ``liboracle.so`` with gcc (no fast-math, so the
arithmetic is plain IEEE FP64); importing builds it if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("oracle.c", "sphere.c", "basis.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

PI = np.pi


def build(force: bool = True) -> str:
    """Compile the oracle library in place; returns its path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
            build(force=True)
        L = C.CDLL(_LIB)
        d, i = C.c_double, C.c_int
        P = C.c_void_p
        L.oracle_mesh_graded_1d.argtypes = [d, d, i, P, i, d, d, d, d, P, P, P]
        L.oracle_mesh_graded_1d.restype = i
        L.oracle_solid_harmonics.argtypes = [d, d, d, P]
        L.oracle_solid_harmonics.restype = None
        L.oracle_pseudo_density.argtypes = [P, i, P, i, P, i, i, P, P, P, P, P, P, P, P, P, P, P, i, P]
        L.oracle_pseudo_density.restype = i
        L.oracle_moments.argtypes = [P, i, P, i, P, i, P, i, P, P]
        L.oracle_moments.restype = None
        L.oracle_boundary_values.argtypes = [P, i, P, i, P, i, i, P, i, P, P]
        L.oracle_boundary_values.restype = None
        L.oracle_apply.argtypes = [P, i, P, i, P, i, P, P]
        L.oracle_apply.restype = None
        L.oracle_solve.argtypes = [P, i, P, i, P, i, P, P, d, i, i, i, d, i, P, P]
        L.oracle_solve.restype = i
        L.oracle_rel_residual.argtypes = [P, i, P, i, P, i, P, P]
        L.oracle_rel_residual.restype = d
        L.oracle_interp.argtypes = [P, i, P, i, P, i, P, i, P, P]
        L.oracle_interp.restype = i
        L.oracle_rb_sweep.argtypes = [P, i, P, i, P, i, P, P, i, P]
        L.oracle_rb_sweep.restype = None
        L.oracle_hierarchy_sizes.argtypes = [P, i, P, i, P, i, d, i, P, i]
        L.oracle_hierarchy_sizes.restype = i
        L.oracle_sphere_rule.argtypes = [i, i, P, P]
        L.oracle_sphere_rule.restype = i
        L.oracle_sphere_project.argtypes = [i, i, i, P, P]
        L.oracle_sphere_project.restype = i
        L.oracle_radial_node.argtypes = [d, d, i, i]
        L.oracle_radial_node.restype = d
        L.oracle_sphere_radial.argtypes = [i, P, P, i, d, P, P, P]
        L.oracle_sphere_radial.restype = i
        L.oracle_sphere_energy.argtypes = [i, P, i, d, P, P, P]
        L.oracle_sphere_energy.restype = i
        L.oracle_energy_grid.argtypes = [P, i, P, i, P, i, P, P, i, P, P]
        L.oracle_energy_grid.restype = d
        L.oracle_sphere_density_terms.argtypes = [P, i, P, i, P, i, i, P, P, i, d, P, i, P]
        L.oracle_sphere_density_terms.restype = i
        L.oracle_density_points.argtypes = [i, P, i, P, P, P, i, P, P, i, P, P]
        L.oracle_density_points.restype = i
        L.oracle_interstitial_density.argtypes = [P, i, P, i, P, i, i, P, P, i, P, P, P, i, P, P, P]
        L.oracle_interstitial_density.restype = i
        L.oracle_basis_points.argtypes = [i, P, i, P, P, P, i, P, P, P, P]
        L.oracle_basis_points.restype = i
        L.oracle_matrix_elements.argtypes = [P, i, P, i, P, i, P, i, P, P, i, P, P, P, P, P]
        L.oracle_matrix_elements.restype = i
        L.oracle_set_threads.argtypes = [i]
        L.oracle_set_threads.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = i
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ API
def mesh_graded_1d(lo, hi, n, planes, hmin, hmax, gmax=1.2, hmin_step=0.0):
    """Graded 1-D node coordinates (Section 3's adaptive mesh, grading rule of
    the oracle header). Returns (x, g, hmin_used)."""
    planes = _f64(planes).ravel()
    x = np.zeros(n)
    g = np.zeros(1)
    hm = np.zeros(1)
    rc = lib().oracle_mesh_graded_1d(lo, hi, n, _p(planes), len(planes), hmin, hmax, gmax,
                                     hmin_step, _p(x), _p(g), _p(hm))
    if rc != 0:
        raise ValueError("oracle_mesh_graded_1d failed (%d)" % rc)
    return x, float(g[0]), float(hm[0])


def mesh_for(axes):
    """Coordinates for the three AxisSpec of a workload."""
    out = []
    for a in axes:
        x, _, _ = mesh_graded_1d(a.lo, a.hi, a.n, a.planes, a.hmin, a.hmax, a.gmax, a.hmin_step)
        out.append(x)
    return out


def solid_harmonics(x, y, z) -> np.ndarray:
    S = np.zeros(25)
    lib().oracle_solid_harmonics(float(x), float(y), float(z), _p(S))
    return S


def pseudo_density(xs, atoms_arr, rho_inter=None, renormalize=True) -> np.ndarray:
    x, y, z = (_f64(a) for a in xs)
    A = atoms_arr
    n = len(A["q"])
    out = np.zeros((len(z), len(y), len(x)))
    ri = None if rho_inter is None else _f64(rho_inter)
    centers = _f64(A["centers"])
    clm = _f64(A["clm"])
    assert clm.shape == (n, 24)
    keep = [centers, _f64(A["q"]), _f64(A["width"]), _f64(A["radius"]), _f64(A["alpha"]),
            np.ascontiguousarray(A["lmax"], dtype=np.int32), clm,
            np.ascontiguousarray(A["kind"], dtype=np.int32), _f64(A["rho_R"]), _f64(A["drho_R"])]
    rc = lib().oracle_pseudo_density(_p(x), len(x), _p(y), len(y), _p(z), len(z), n,
                                     *[_p(k) for k in keep],
                                     None if ri is None else _p(ri), int(renormalize), _p(out))
    if rc != 0:
        raise ValueError("oracle_pseudo_density failed")
    return out


def moments(xs, rho, lmax_bc=4, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    x, y, z = (_f64(a) for a in xs)
    rho = _f64(rho)
    Q = np.zeros((lmax_bc + 1) ** 2)
    c = _f64(center)
    lib().oracle_moments(_p(x), len(x), _p(y), len(y), _p(z), len(z), _p(rho), lmax_bc, _p(c), _p(Q))
    return Q


def boundary_values(xs, Q, v, bc_mode=1, lmax_bc=4, center=(0.0, 0.0, 0.0)):
    """Writes the six faces of v (in place)."""
    x, y, z = (_f64(a) for a in xs)
    Qa = _f64(Q)
    c = _f64(center)
    assert v.dtype == np.float64 and v.flags.c_contiguous
    lib().oracle_boundary_values(_p(x), len(x), _p(y), len(y), _p(z), len(z), bc_mode, _p(Qa),
                                 lmax_bc, _p(c), _p(v))
    return v


def apply(xs, u) -> np.ndarray:
    x, y, z = (_f64(a) for a in xs)
    u = _f64(u)
    out = np.zeros_like(u)
    lib().oracle_apply(_p(x), len(x), _p(y), len(y), _p(z), len(z), _p(u), _p(out))
    return out


def solve(xs, rho, v, rtol=1e-12, max_cycles=200, nu1=2, nu2=2, theta=4.0, coarse_max=5):
    """In-place V-cycle solve of eq. (3.2); v holds face values and the guess.
    Returns (cycles, rel_resid, history)."""
    x, y, z = (_f64(a) for a in xs)
    rho = _f64(rho)
    assert v.dtype == np.float64 and v.flags.c_contiguous
    rel = np.zeros(1)
    hist = np.zeros(128)
    cyc = lib().oracle_solve(_p(x), len(x), _p(y), len(y), _p(z), len(z), _p(rho), _p(v), rtol,
                             max_cycles, nu1, nu2, theta, coarse_max, _p(rel), _p(hist))
    return cyc, float(rel[0]), hist[:min(cyc, 128)].copy()


def rel_residual(xs, rho, v) -> float:
    x, y, z = (_f64(a) for a in xs)
    return lib().oracle_rel_residual(_p(x), len(x), _p(y), len(y), _p(z), len(z), _p(_f64(rho)), _p(_f64(v)))


def interp(xs, v, pts) -> np.ndarray:
    x, y, z = (_f64(a) for a in xs)
    pts = _f64(pts).reshape(-1, 3)
    out = np.zeros(len(pts))
    rc = lib().oracle_interp(_p(x), len(x), _p(y), len(y), _p(z), len(z), _p(_f64(v)), len(pts), _p(pts), _p(out))
    if rc != 0:
        raise ValueError("oracle_interp needs >= 4 nodes per axis")
    return out


def rb_sweep(xs, u, rho, first=0) -> np.ndarray:
    """One red-black Gauss-Seidel sweep on A u = 4 pi rho (colour `first` first)."""
    x, y, z = (_f64(a) for a in xs)
    u = _f64(u)
    out = np.zeros_like(u)
    lib().oracle_rb_sweep(_p(x), len(x), _p(y), len(y), _p(z), len(z), _p(u), _p(_f64(rho)), int(first), _p(out))
    return out


def hierarchy_sizes(xs, theta=4.0, coarse_max=5):
    x, y, z = (_f64(a) for a in xs)
    s = np.zeros(64 * 3, dtype=np.int32)
    nl = lib().oracle_hierarchy_sizes(_p(x), len(x), _p(y), len(y), _p(z), len(z), theta, coarse_max, _p(s), 64)
    return s[:3 * nl].reshape(nl, 3)


def sphere_points(centers, radii, dirs) -> np.ndarray:
    """C_a + R_a d_k for every atom a and direction k, atom-major."""
    centers = _f64(centers).reshape(-1, 3)
    radii = _f64(radii).ravel()
    dirs = _f64(dirs).reshape(-1, 3)
    return (centers[:, None, :] + radii[:, None, None] * dirs[None, :, :]).reshape(-1, 3)


def hartree_step(xs, atoms_arr, dirs, bc_mode=1, lmax_bc=4, rtol=1e-12, max_cycles=200,
                 rho_inter=None, renormalize=True, guess=None):
    """The whole path on the CPU: pseudo-density -> moments -> face values ->
    solve -> values on the sphere boundaries. Returns a dict."""
    rho = pseudo_density(xs, atoms_arr, rho_inter, renormalize)
    center = (0.5 * (xs[0][0] + xs[0][-1]), 0.5 * (xs[1][0] + xs[1][-1]), 0.5 * (xs[2][0] + xs[2][-1]))
    Q = moments(xs, rho, lmax_bc, center)
    v = np.zeros_like(rho) if guess is None else _f64(guess).copy()
    boundary_values(xs, Q, v, bc_mode, lmax_bc, center)
    cyc, rel, hist = solve(xs, rho, v, rtol, max_cycles)
    pts = sphere_points(atoms_arr["centers"], atoms_arr["radius"], dirs)
    vs = interp(xs, v, pts).reshape(len(atoms_arr["q"]), -1)
    return dict(rho=rho, Q=Q, v=v, cycles=cyc, rel=rel, hist=hist, sphere=vs, center=center)


# ------------------------------------------------------- inside the spheres
NLM = 25


def sphere_rule(n_theta, n_phi):
    """Directions [n_theta*n_phi][3] and weights of the product rule on the
    unit sphere used for eq. (3.6) (sphere.c)."""
    np_ = n_theta * n_phi
    d = np.zeros((np_, 3))
    w = np.zeros(np_)
    if lib().oracle_sphere_rule(n_theta, n_phi, _p(d), _p(w)) != 0:
        raise ValueError("bad sphere rule")
    return d, w


def sphere_project(values, n_theta, n_phi):
    """eq. (3.6): values [n_atoms][n_theta*n_phi] -> V_LM(R) [n_atoms][25]."""
    v = _f64(values).reshape(-1, n_theta * n_phi)
    out = np.zeros((len(v), NLM))
    if lib().oracle_sphere_project(len(v), n_theta, n_phi, _p(v), _p(out)) != 0:
        raise ValueError("bad sphere rule")
    return out


def radial_mesh(R, r_min, n):
    """Atom mesh r_k, k = 0..n-1 (sphere.c)."""
    return np.array([lib().oracle_radial_node(float(R), float(r_min), int(n), k) for k in range(n)])


def sphere_radial(radii, Z, r_min, vlm_R, rho_lm):
    """Interior solution of eq. (3.4): vlm_R [n_atoms][25], rho_lm
    [n_atoms][25][n_rad] -> V_LM(r_k) [n_atoms][25][n_rad]."""
    rho_lm = _f64(rho_lm)
    na, _, n = rho_lm.shape
    out = np.zeros_like(rho_lm)
    rc = lib().oracle_sphere_radial(na, _p(_f64(radii)), _p(_f64(Z)), n, float(r_min), _p(_f64(vlm_R)),
                                    _p(rho_lm), _p(out))
    if rc != 0:
        raise ValueError("oracle_sphere_radial needs n_rad >= 4")
    return out


def sphere_energy(radii, r_min, vlm, rho_lm):
    """Per atom sum_LM int_0^R V_LM rho_LM r^2 dr."""
    vlm, rho_lm = _f64(vlm), _f64(rho_lm)
    na, _, n = rho_lm.shape
    out = np.zeros(na)
    if lib().oracle_sphere_energy(na, _p(_f64(radii)), n, float(r_min), _p(vlm), _p(rho_lm), _p(out)) != 0:
        raise ValueError("oracle_sphere_energy needs n_rad >= 4")
    return out


def energy_grid(xs, v, rho, centers, radii):
    """sum over nodes outside every sphere of vol_n v_n rho_n."""
    x, y, z = (_f64(a) for a in xs)
    centers = _f64(centers).reshape(-1, 3)
    return lib().oracle_energy_grid(_p(x), len(x), _p(y), len(y), _p(z), len(z), _p(_f64(v)), _p(_f64(rho)),
                                    len(centers), _p(centers), _p(_f64(radii)))


# ------------------------------------------------ interstitial output density
def _shells(shells):
    n = np.ascontiguousarray([s[0] for s in shells], dtype=np.int32)
    l = np.ascontiguousarray([s[1] for s in shells], dtype=np.int32)
    z = _f64([s[2] for s in shells])
    return n, l, z


def density_points(centers, shells, coef, occ, pts):
    """rho_out = sum_k f_k psi_k^2 at points [npts][3] (basis.c); shells =
    [(n, l, zeta), ...] on every atom; coef [n_basis][n_occ]."""
    centers = _f64(centers).reshape(-1, 3)
    n, l, z = _shells(shells)
    coef = _f64(coef)
    occ = _f64(occ)
    pts = _f64(pts).reshape(-1, 3)
    out = np.zeros(len(pts))
    rc = lib().oracle_density_points(len(centers), _p(centers), len(n), _p(n), _p(l), _p(z), len(occ), _p(coef),
                                     _p(occ), len(pts), _p(pts), _p(out))
    if rc != 0:
        raise ValueError("bad shells")
    return out


def interstitial_density(xs, centers, radii, shells, coef, occ):
    """rho_out on the grid nodes [nz][ny][nx], zero inside the spheres."""
    x, y, zz = (_f64(a) for a in xs)
    centers = _f64(centers).reshape(-1, 3)
    n, l, z = _shells(shells)
    coef = _f64(coef)
    occ = _f64(occ)
    out = np.zeros((len(zz), len(y), len(x)))
    rc = lib().oracle_interstitial_density(_p(x), len(x), _p(y), len(y), _p(zz), len(zz), len(centers), _p(centers),
                                           _p(_f64(radii)), len(n), _p(n), _p(l), _p(z), len(occ), _p(coef),
                                           _p(occ), _p(out))
    if rc != 0:
        raise ValueError("bad shells")
    return out


def basis_points(centers, shells, pts, vpts=None):
    """phi and (-1/2 Laplacian + V) phi at points: two [npts][n_basis] arrays."""
    centers = _f64(centers).reshape(-1, 3)
    n, l, z = _shells(shells)
    pts = _f64(pts).reshape(-1, 3)
    vp = np.zeros(len(pts)) if vpts is None else _f64(vpts).ravel()
    nb = len(centers) * int(sum(2 * q + 1 for q in l))
    phi = np.zeros((len(pts), nb))
    tphi = np.zeros((len(pts), nb))
    rc = lib().oracle_basis_points(len(centers), _p(centers), len(n), _p(n), _p(l), _p(z), len(pts), _p(pts), _p(vp),
                                   _p(phi), _p(tphi))
    if rc != 0:
        raise ValueError("bad shells")
    return phi, tphi


def matrix_elements(xs, v, centers, radii, shells):
    """Interstitial S and H by grid quadrature (basis.c): two [n_basis][n_basis]."""
    x, y, zz = (_f64(a) for a in xs)
    centers = _f64(centers).reshape(-1, 3)
    n, l, z = _shells(shells)
    nb = len(centers) * int(sum(2 * q + 1 for q in l))
    S = np.zeros((nb, nb))
    H = np.zeros((nb, nb))
    rc = lib().oracle_matrix_elements(_p(x), len(x), _p(y), len(y), _p(zz), len(zz), _p(_f64(v)), len(centers),
                                      _p(centers), _p(_f64(radii)), len(n), _p(n), _p(l), _p(z), _p(S), _p(H))
    if rc != 0:
        raise ValueError("bad shells")
    return S, H


def sphere_density_terms(xs, centers, radii, r_min, rho_lm, lmin, rho):
    """Adds sum_(L >= lmin) rho_LM(r) y_LM inside each sphere to rho (in place)."""
    x, y, z = (_f64(a) for a in xs)
    centers = _f64(centers).reshape(-1, 3)
    rho_lm = _f64(rho_lm)
    assert rho.dtype == np.float64 and rho.flags.c_contiguous
    rc = lib().oracle_sphere_density_terms(_p(x), len(x), _p(y), len(y), _p(z), len(z), len(centers), _p(centers),
                                           _p(_f64(radii)), rho_lm.shape[2], float(r_min), _p(rho_lm), int(lmin),
                                           _p(rho))
    if rc != 0:
        raise ValueError("bad n_rad or lmin")
    return rho


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())
