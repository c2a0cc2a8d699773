"""The paper's own setting end to end on the GPU: a Pd dimer on a uniform
mesh (0.05 a0 at 257^3), kind-1 quartic pseudo-densities from the Fig. 4
readings, the tabulated non-spherical density inside the spheres, the
interstitial density outside, zero Dirichlet faces (eq. (3.3)), the solve
(multigrid and fast diagonalisation), the interior solve and the energy
integral; against the oracle at 65^3 and through the oracle's residual at
257^3."""
import sys

import numpy as np
import pytest

from paper_0806_1723_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a device"
    return t


@pytest.fixture(scope="module")
def L():
    from paper_0806_1723_amd import lasto
    lasto.load()
    return lasto


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def inputs(n):
    w = I.paper_dimer(n)
    A = I.atom_arrays(w.atoms)
    c, r = A["centers"], A["radius"]
    rng = np.random.default_rng(101)
    tab = I.sphere_density(I.make_atoms(rng, c), radii=r)    # synthetic sphere tables
    coef, occ = I.basis_coefficients(len(r), seed=102)
    return w, A, c, r, tab, coef, occ


def test_paper_setting_matches_oracle_65(torch, L, oracle_mod):
    n = 65
    say("paper setting, Pd2 at %d^3, zero faces" % n)
    w, A, c, r, tab, coef, occ = inputs(n)
    xs = oracle_mod.mesh_for(w.axes)
    # oracle
    ri = oracle_mod.interstitial_density(xs, c, r, I.LASTO_SHELLS, coef, occ)
    rho_o = oracle_mod.pseudo_density(xs, A, rho_inter=ri)
    oracle_mod.sphere_density_terms(xs, c, r, I.R_MIN, tab, 1, rho_o)
    v_o = np.zeros_like(rho_o)
    oracle_mod.boundary_values(xs, np.zeros(25), v_o, 0, 4)
    _, rel, _ = oracle_mod.solve(xs, rho_o, v_o, rtol=1e-12)
    assert rel <= 1e-12
    d, _ = oracle_mod.sphere_rule(8, 9)
    vals = oracle_mod.interp(xs, v_o, oracle_mod.sphere_points(c, r, d)).reshape(2, -1)
    wR = oracle_mod.sphere_project(vals, 8, 9)
    Z = np.full(2, I.PD_Z)
    wl = oracle_mod.sphere_radial(r, Z, I.R_MIN, wR, tab)
    e_o = (oracle_mod.energy_grid(xs, v_o, rho_o, c, r), oracle_mod.sphere_energy(r, I.R_MIN, wl, tab).sum())
    # GPU
    g = L.Grid(*xs)
    S = L.Spheres(g, c, r, Z=Z)
    ri_g = g.interstitial_density(c, r, I.LASTO_SHELLS, dev(torch, coef), occ)
    rho = g.pseudo_density(w.atoms, rho_interstitial=ri_g)
    S.density_terms(dev(torch, tab), rho, lmin=1)
    assert np.abs(rho.cpu().numpy() - rho_o).max() <= 1e-12 * np.abs(rho_o).max()
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-12, bc=0)
    vf = g.empty()
    finfo = g.fdm_solve(rho, vf, bc=0)
    for name, vv, inf in (("multigrid", v, info), ("direct", vf, finfo)):
        err = np.abs(vv.cpu().numpy() - v_o).max() / np.abs(v_o).max()
        say("  %s: rel resid %.2e, max rel diff to the oracle %.2e" % (name, inf["rel_resid"], err))
        assert err <= 1e-9
    tl = dev(torch, tab)
    v_lm = S.radial(S.project(v), tl)
    e = S.energy(v, rho, v_lm, tl)
    assert np.abs(v_lm.cpu().numpy() - wl).max() <= 1e-9 * np.abs(wl).max()
    say("  energy parts %s vs %s" % (e, e_o))
    assert abs(e[0] - e_o[0]) <= 1e-9 * abs(e_o[0]) and abs(e[1] - e_o[1]) <= 1e-9 * abs(e_o[1])
    S.close()
    g.close()


def test_paper_setting_257(torch, L, oracle_mod):
    """0.05 a0 spacing as in Section 4: the whole step on the GPU; the oracle's
    operator confirms both solves' residuals, and they agree"""
    n = 257
    say("paper setting, Pd2 at %d^3 (0.05 a0), zero faces" % n)
    w, A, c, r, tab, coef, occ = inputs(n)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    S = L.Spheres(g, c, r, Z=np.full(2, I.PD_Z))
    ri = g.interstitial_density(c, r, I.LASTO_SHELLS, dev(torch, coef), occ)
    rho = g.pseudo_density(w.atoms, rho_interstitial=ri)
    tl = dev(torch, tab)
    S.density_terms(tl, rho, lmin=1)
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-10, bc=0, precision=1)
    vf = g.empty()
    finfo = g.fdm_solve(rho, vf, bc=0)
    rho_h = rho.cpu().numpy()
    r_mg = oracle_mod.rel_residual(xs, rho_h, v.cpu().numpy())
    r_fd = oracle_mod.rel_residual(xs, rho_h, vf.cpu().numpy())
    d = (v - vf).abs().max().item() / vf.abs().max().item()
    say("  multigrid rel %.2e (oracle %.2e, %.2f ms); direct rel %.2e (oracle %.2e, %.2f ms); max rel diff %.2e"
        % (info["rel_resid"], r_mg, info["ms_total"], finfo["rel_resid"], r_fd, finfo["ms_total"], d))
    # the direct solve's rounding floor grows with the operator's spread of
    # eigenvalues (4/h^2 at h = 0.05 against (pi/12.8)^2): a few 1e-12
    assert r_mg <= 1e-10 and r_fd <= 1e-11
    assert d <= 1e-8
    v_lm = S.radial(S.project(vf), tl)
    e = S.energy(vf, rho, v_lm, tl)
    say("  energy integral parts %s" % (e,))
    assert np.isfinite(e).all()
    S.close()
    g.close()
