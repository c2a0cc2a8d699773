"""Seeded synthetic workloads for the Hartree step (geometry and random
coefficients only).

This module is shared by the tests, the benchmark and the smoke check. It
holds none of the method's arithmetic: it draws atom positions, charges,
multipole coefficients and mesh parameters, and nothing else. Both the GPU
path and the CPU oracle turn these numbers into meshes, densities and
potentials with their own code.

Cluster shapes follow the Pd clusters the paper studies (Section 4, Fig. 7
shows Pd2/Pd4/Pd8); the larger shapes (icosahedron, cuboctahedron, Mackay
icosahedron, random close-packed clusters) and the per-atom charges are a
synthetic stand-in for real Pd sphere densities, which are not available.
Lengths are in bohr (a0), the paper's atomic units (Section 2).

Per-atom draw order: position jitter, then q, then the multipole
coefficients c_lm (l = 1: m = -1, 0, 1; l = 2: m = -2..2), then any
perturbations.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

GAUSS_WIDTH = 0.5        # w in exp(-r^2/w^2) of the monopole pseudo-density
ALPHA = 1.0              # radial factor r^l exp(-alpha r^2) of the l >= 1 terms
SPHERE_RADIUS = 2.5      # muffin-tin radius used for the interpolation points
NN_DIST = 5.2            # nearest-neighbour distance of the Pd-like clusters
PD_Z = 46.0              # nuclear charge of the sphere densities (palladium)
CORE_ZETA = 46.0         # exponent of their hydrogen-like core, exp(-2 zeta r)
N_RAD = 429              # radial points per sphere (Section 4)
R_MIN = 1e-5             # first radial point (bohr)
# the LASTO basis of Table 1 (n, l, zeta): 4d, 5d, 5s, 5p, 6s, 6p, 4f
LASTO_SHELLS = [(4, 2, 2.2), (5, 2, 2.6), (5, 0, 1.0), (5, 1, 1.0), (6, 0, 2.0), (6, 1, 2.0), (4, 3, 1.6)]
STATES_PER_ATOM = 5      # doubly occupied states per atom (10 valence electrons)


@dataclass
class Atom:
    center: np.ndarray          # (3,) bohr
    q: float                    # charge of the monopole pseudo-density
    width: float = GAUSS_WIDTH
    radius: float = SPHERE_RADIUS
    lmax: int = 2
    clm: np.ndarray = field(default_factory=lambda: np.zeros(0))  # (lmax+1)^2-1
    alpha: float = ALPHA
    kind: int = 0               # 0 Gaussian monopole, 1 paper quartic
    rho_R: float = 0.0          # kind 1: spherical density at R
    drho_R: float = 0.0         # kind 1: its radial derivative at R


@dataclass
class AxisSpec:
    """Parameters of one axis of the tensor-product mesh (not the nodes)."""
    lo: float
    hi: float
    n: int
    planes: np.ndarray          # atom coordinates on this axis (may repeat)
    hmin: float
    hmax: float
    gmax: float = 1.2
    hmin_step: float = 0.0      # > 0: raise hmin in these steps until feasible


@dataclass
class Workload:
    name: str
    atoms: List[Atom]
    axes: List[AxisSpec]        # x, y, z
    n_batch: int = 1
    batch_atoms: Optional[List[List[Atom]]] = None   # per-batch perturbed atoms
    precision: str = "fp64"
    rtol: float = 1e-10


# ----------------------------------------------------------------- geometry
def icosahedron_vertices() -> np.ndarray:
    """12 vertices: cyclic permutations of (0, +-1, +-phi), unit radius."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v += [(0.0, s1, s2 * phi), (s1, s2 * phi, 0.0), (s2 * phi, 0.0, s1)]
    v = np.array(v)
    return v / np.linalg.norm(v[0])


def icosahedron_faces(v: np.ndarray) -> List[tuple]:
    edge = min(np.linalg.norm(v[i] - v[j]) for i in range(12) for j in range(i + 1, 12))
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                d = [np.linalg.norm(v[a] - v[b]) for a, b in ((i, j), (j, k), (i, k))]
                if all(abs(x - edge) < 1e-9 for x in d):
                    faces.append((i, j, k))
    assert len(faces) == 20
    return faces


def ico13(nn: float = NN_DIST) -> np.ndarray:
    """Centre + 12 vertices at radius nn (minimum pairwise distance nn)."""
    return np.vstack([np.zeros(3), icosahedron_vertices() * nn])


def mackay_icosahedron(shells: int, nn: float = NN_DIST) -> np.ndarray:
    """Mackay icosahedron: centre plus shells k = 1..shells; shell k holds the
    points (a V0 + b V1 + c V2) nn with a + b + c = k on every face (flat
    faces, k subdivisions per edge). 1, 13, 55, 147, 309 atoms."""
    v = icosahedron_vertices()
    faces = icosahedron_faces(v)
    pts = [np.zeros(3)]
    for k in range(1, shells + 1):
        shell = []
        for (i, j, l) in faces:
            for a in range(k + 1):
                for b in range(k + 1 - a):
                    c = k - a - b
                    p = (a * v[i] + b * v[j] + c * v[l]) * nn
                    if not any(np.linalg.norm(p - s) < 1e-6 for s in shell):
                        shell.append(p)
        pts += shell
    return np.array(pts)


def cuboctahedron55(nn: float = NN_DIST) -> np.ndarray:
    """fcc points (a,b,c) nn/sqrt(2), a+b+c even, max|.| <= 2, sum|.| <= 4."""
    pts = []
    for a in range(-2, 3):
        for b in range(-2, 3):
            for c in range(-2, 3):
                if (a + b + c) % 2 == 0 and abs(a) + abs(b) + abs(c) <= 4:
                    pts.append((a, b, c))
    p = np.array(pts, dtype=np.float64) * nn / np.sqrt(2.0)
    assert len(p) == 55
    return p


def random_cluster(rng: np.random.Generator, n: int, dmin: float = 5.0,
                   max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition in a ball of radius 2.6 (n/0.22)^(1/3) - 2.6
    with minimum pairwise distance dmin, then centred at the origin."""
    rad = 2.6 * (n / 0.22) ** (1.0 / 3.0) - 2.6
    pts: List[np.ndarray] = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not finish")
        p = rng.uniform(-rad, rad, 3)
        if np.linalg.norm(p) > rad:
            continue
        if all(np.linalg.norm(p - s) >= dmin for s in pts):
            pts.append(p)
    P = np.array(pts)
    return P - P.mean(axis=0)


# ----------------------------------------------------------------- atoms
def n_clm(lmax: int) -> int:
    return (lmax + 1) ** 2 - 1


def make_atoms(rng: np.random.Generator, pos: np.ndarray, lmax: int = 2,
               jitter: float = 0.0, q=10.0, clm_sigma: float = 0.1) -> List[Atom]:
    """Draw per atom: jitter (3 normals), q (if a range), c_lm normals."""
    atoms = []
    for p in pos:
        c = np.array(p, dtype=np.float64)
        if jitter > 0.0:
            c = c + rng.normal(0.0, jitter, 3)
        if isinstance(q, tuple):
            qa = float(rng.uniform(q[0], q[1]))
        else:
            qa = float(q)
        clm = rng.normal(0.0, clm_sigma, n_clm(lmax))
        atoms.append(Atom(center=c, q=qa, lmax=lmax, clm=clm))
    return atoms


def perturb_atoms(atoms: List[Atom], seed: int, rel: float = 0.01) -> List[Atom]:
    """SCF-like perturbation: q and every c_lm times (1 + rel xi), xi ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    out = []
    for a in atoms:
        q = a.q * (1.0 + rel * rng.normal())
        clm = a.clm * (1.0 + rel * rng.normal(size=a.clm.shape))
        out.append(Atom(center=a.center.copy(), q=q, width=a.width, radius=a.radius,
                        lmax=a.lmax, clm=clm, alpha=a.alpha))
    return out


def uniform_axes(L: float, n: int) -> List[AxisSpec]:
    return [AxisSpec(-L / 2, L / 2, n, np.zeros(0), 0.0, 0.0) for _ in range(3)]


def graded_axes(L: float, n: int, atoms: List[Atom], hmin: float, hmax: float,
                gmax: float = 1.2, hmin_step: float = 0.0) -> List[AxisSpec]:
    pos = np.array([a.center for a in atoms])
    return [AxisSpec(-L / 2, L / 2, n, pos[:, d].copy(), hmin, hmax, gmax, hmin_step)
            for d in range(3)]


# ----------------------------------------------------------------- configs
def _scale(n_default: int, n: int) -> float:
    """Spacing scale of a reduced-size variant of a config: (N0-1)/(N-1)."""
    return (n_default - 1) / (n - 1)


def config(cid: int, n_override: Optional[int] = None, sample: int = 0) -> Workload:
    """The five synthetic workloads. ``n_override`` gives a reduced (or
    enlarged) variant of the same geometry with hmin and hmax scaled by
    (N0-1)/(N-1).

    1: one atom, uniform 33^3 in a 20-bohr cube, plain FP64.
    2: 13-atom icosahedron, graded 129^3 in a 40-bohr box.
    3: 55-atom jittered cuboctahedron, graded 257^3 in a 56-bohr box, mixed.
    4: random 13..55-atom cluster (sample s, seed 40000+s), graded 129^3, L=48.
    5: 309-atom Mackay icosahedron, graded 513^3 in an 80-bohr box, 8 RHS.
    """
    if cid == 1:
        rng = np.random.default_rng(1)
        n = n_override or 33
        atoms = make_atoms(rng, np.zeros((1, 3)))
        return Workload("one atom, uniform %d^3, L=20" % n, atoms, uniform_axes(20.0, n))
    if cid == 2:
        rng = np.random.default_rng(2)
        n = n_override or 129
        atoms = make_atoms(rng, ico13())
        return Workload("13-atom icosahedron, graded %d^3, L=40" % n, atoms,
                        graded_axes(40.0, n, atoms, 0.12 * _scale(129, n), 0.6 * _scale(129, n)))
    if cid == 3:
        rng = np.random.default_rng(3)
        n = n_override or 257
        atoms = make_atoms(rng, cuboctahedron55(), jitter=0.05)
        return Workload("55-atom cuboctahedron, graded %d^3, L=56" % n, atoms,
                        graded_axes(56.0, n, atoms, 0.12 * _scale(257, n), 0.6 * _scale(257, n)),
                        precision="mixed")
    if cid == 4:
        rng = np.random.default_rng(40000 + sample)
        n = n_override or 129
        na = int(rng.integers(13, 56))
        pos = random_cluster(rng, na)
        atoms = make_atoms(rng, pos, q=(8.0, 12.0))
        return Workload("random %d-atom cluster #%d, graded %d^3, L=48" % (na, sample, n),
                        atoms, graded_axes(48.0, n, atoms, 0.12 * _scale(129, n), 0.6 * _scale(129, n),
                                           1.2, 0.01))
    if cid == 5:
        rng = np.random.default_rng(5)
        n = n_override or 513
        atoms = make_atoms(rng, mackay_icosahedron(4))
        batch = [perturb_atoms(atoms, 500 + b) for b in range(8)]
        return Workload("309-atom Mackay icosahedron, graded %d^3, L=80, 8 RHS" % n,
                        atoms, graded_axes(80.0, n, atoms, 0.12 * _scale(513, n), 0.6 * _scale(513, n)),
                        n_batch=8,
                        batch_atoms=batch, precision="mixed")
    raise ValueError("config id must be 1..5")


def default_directions() -> np.ndarray:
    """64 unit vectors: 8 Gauss-Legendre nodes in cos(theta) times 8 azimuths
    phi_b = 2 pi (b + 1/2) / 8, theta-major."""
    t, _ = np.polynomial.legendre.leggauss(8)
    out = []
    for ct in t:
        st = np.sqrt(max(0.0, 1.0 - ct * ct))
        for b in range(8):
            ph = 2.0 * np.pi * (b + 0.5) / 8.0
            out.append((st * np.cos(ph), st * np.sin(ph), ct))
    return np.array(out)


def atom_arrays(atoms: List[Atom], lmax_pad: int = 4):
    """Flat float64 arrays in the C-ABI atom-table order.

    centers [n,3], q [n], width [n], radius [n], alpha [n], lmax [n] (int32),
    clm [n, (lmax_pad+1)^2-1] zero-padded, kind [n] (int32), rho_R [n], drho_R [n].
    """
    n = len(atoms)
    nc = n_clm(lmax_pad)
    clm = np.zeros((n, nc))
    for i, a in enumerate(atoms):
        clm[i, :len(a.clm)] = a.clm
    return dict(
        centers=np.array([a.center for a in atoms], dtype=np.float64).reshape(n, 3),
        q=np.array([a.q for a in atoms], dtype=np.float64),
        width=np.array([a.width for a in atoms], dtype=np.float64),
        radius=np.array([a.radius for a in atoms], dtype=np.float64),
        alpha=np.array([a.alpha for a in atoms], dtype=np.float64),
        lmax=np.array([a.lmax for a in atoms], dtype=np.int32),
        clm=clm,
        kind=np.array([a.kind for a in atoms], dtype=np.int32),
        rho_R=np.array([a.rho_R for a in atoms], dtype=np.float64),
        drho_R=np.array([a.drho_R for a in atoms], dtype=np.float64),
    )


# ------------------------------------------------------- sphere densities
def radial_points(R: float, n: int = N_RAD, r_min: float = R_MIN) -> np.ndarray:
    """Where a sphere's radial density is sampled: r_k = R exp((k - (n-1)) D),
    D = ln(R / r_min)/(n - 1) (logarithmic, Section 4)."""
    D = np.log(R / r_min) / (n - 1)
    return R * np.exp((np.arange(n) - (n - 1)) * D)


def muffin_tin_radii(atoms: List[Atom]) -> np.ndarray:
    """Sphere radii for the interior solve: each atom's radius, cut to just
    under half its nearest-neighbour distance so that no two spheres overlap
    (the jittered clusters bring some pairs below 2 x 2.5 bohr)."""
    c = np.array([a.center for a in atoms], dtype=np.float64).reshape(-1, 3)
    R = np.array([a.radius for a in atoms], dtype=np.float64)
    if len(c) > 1:
        d = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))
        np.fill_diagonal(d, np.inf)
        R = np.minimum(R, 0.5 * d.min(axis=1) * (1.0 - 1e-9))
    return R


def sphere_density(atoms: List[Atom], n: int = N_RAD, r_min: float = R_MIN, Z: float = PD_Z,
                   zeta: float = CORE_ZETA, radii=None) -> np.ndarray:
    """Synthetic all-electron density inside each sphere as rho_LM(r_k)
    [n_atoms][25][n] (real orthonormal y_LM, index L*L + L + M): a
    hydrogen-like core of Z electrons, Z (zeta^3/pi) exp(-2 zeta r), plus the
    atom's Gaussian of q electrons (its pseudo-density's monopole) on
    y_00 = 1/sqrt(4 pi); for L >= 1 the atom's own c_lm r^l exp(-alpha r^2).
    With a nucleus of charge Z the core is neutral, so the sphere's net
    monopole is q like the pseudo-density's. radii: the spheres' radii
    (default each atom's own)."""
    out = np.zeros((len(atoms), 25, n))
    for a, at in enumerate(atoms):
        r = radial_points(at.radius if radii is None else radii[a], n, r_min)
        core = Z * zeta ** 3 / np.pi * np.exp(-2.0 * zeta * r)
        gauss = at.q * (np.pi * at.width ** 2) ** -1.5 * np.exp(-(r / at.width) ** 2)
        out[a, 0] = np.sqrt(4.0 * np.pi) * (core + gauss)
        for t in range(len(at.clm)):
            lm = t + 1
            l = int(np.sqrt(lm))
            out[a, lm] = at.clm[t] * r ** l * np.exp(-at.alpha * r * r)
    return out


# ------------------------------------------------------ basis coefficients
def basis_coefficients(n_atoms: int, seed: int, shells=None, states_per_atom: int = STATES_PER_ATOM):
    """Synthetic real coefficients of the occupied states, [n_basis][n_occ],
    and their occupations (2 each). Each basis function's column of draws
    N(0, 1/n_basis) is divided by its norm sqrt((2n)!/(2 zeta)^(2n+1)), so
    every function contributes on a like scale (the paper's basis functions
    are not normalised)."""
    from math import factorial
    shells = LASTO_SHELLS if shells is None else shells
    rng = np.random.default_rng(seed)
    scale = []
    for n, l, z in shells:
        nrm = np.sqrt(factorial(2 * n) / (2.0 * z) ** (2 * n + 1))
        scale += [1.0 / nrm] * (2 * l + 1)
    scale = np.tile(np.array(scale), n_atoms)
    n_occ = states_per_atom * n_atoms
    coef = rng.normal(0.0, 1.0 / np.sqrt(len(scale)), size=(len(scale), n_occ)) * scale[:, None]
    return coef, np.full(n_occ, 2.0)


# ------------------------------------------------- the paper's own setting
# Fig. 4 read at R = 2.3 a0 (Section 3): the Pd pseudo-charge inside the
# sphere, the true density and its slope at R; Section 4: the dimer, a
# uniform 0.05 a0 mesh.
FIG4_R = 2.3
FIG4_Q = -1.62
FIG4_RHO_R = 0.0353
FIG4_DRHO_R = -0.089
PD2_SEPARATION = 4.7     # bohr, near the dimer's equilibrium distance
PAPER_SPACING = 0.05


def paper_dimer(n: int = 257) -> Workload:
    """The paper's own setting: a Pd dimer along z in a cube of 256 x 0.05 =
    12.8 a0 on a uniform mesh (0.05 a0 at n = 257; a reduced n keeps the box
    and widens the spacing), kind-1 quartic pseudo-densities from the Fig. 4
    readings, no analytic l >= 1 terms (the sphere tables supply them)."""
    L = PAPER_SPACING * 256
    pos = np.array([[0.0, 0.0, -PD2_SEPARATION / 2], [0.0, 0.0, PD2_SEPARATION / 2]])
    atoms = [Atom(center=p.copy(), q=FIG4_Q, radius=FIG4_R, lmax=0, clm=np.zeros(0), kind=1, rho_R=FIG4_RHO_R,
                  drho_R=FIG4_DRHO_R) for p in pos]
    return Workload("Pd2 dimer, uniform %d^3 (%.3f a0), L=%.1f" % (n, L / (n - 1), L), atoms, uniform_axes(L, n))
