"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element at sizes the oracle finishes in
seconds (spanning several tiles, with ragged tails), and through properties
at the full 257^3 size."""
import dataclasses
import math
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


def graded(rng, n, lo=-6.0, hi=6.0):
    h = rng.uniform(0.4, 1.6, n - 1)
    x = np.concatenate([[0.0], np.cumsum(h)])
    return lo + (hi - lo) * x / x[-1]


def dual(x):
    m = np.zeros_like(x)
    m[1:-1] = 0.5 * (x[2:] - x[:-2])
    m[0] = 0.5 * (x[1] - x[0])
    m[-1] = 0.5 * (x[-1] - x[-2])
    return m


def wnorm(xs, a):
    vol = np.einsum("k,j,i->kji", dual(xs[2]), dual(xs[1]), dual(xs[0]))
    return math.sqrt(float((vol * a * a)[1:-1, 1:-1, 1:-1].sum()))


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


# ------------------------------------------------------------- kernels
SHAPES = [(131, 37, 41), (4, 4, 4), (70, 9, 19)]


@pytest.mark.parametrize("shape", SHAPES)
def test_apply_matches_oracle(torch, L, oracle_mod, shape):
    say("apply %s" % (shape,))
    rng = np.random.default_rng(11)
    xs = [graded(rng, n) for n in shape]
    u = rng.normal(size=shape[::-1])
    g = L.Grid(*xs)
    Au = g.apply(to_dev(torch, u)).cpu().numpy()
    want = oracle_mod.apply(xs, u)
    I_ = (slice(1, -1),) * 3
    assert np.abs(Au[I_] - want[I_]).max() <= 1e-13 * np.abs(want[I_]).max()
    g.close()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("first", [0, 1])
def test_rb_sweep_matches_oracle(torch, L, oracle_mod, shape, first):
    say("rb_sweep %s first=%d" % (shape, first))
    rng = np.random.default_rng(12 + first)
    xs = [graded(rng, n) for n in shape]
    u = rng.normal(size=shape[::-1])
    rho = rng.normal(size=shape[::-1])
    g = L.Grid(*xs)
    ud = to_dev(torch, u)
    out = g.rb_sweep(ud, to_dev(torch, rho), first_colour=first)
    got = out.cpu().numpy()
    want = oracle_mod.rb_sweep(xs, u, rho, first)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # faces untouched, deterministic
    assert np.array_equal(got[0], u[0]) and np.array_equal(got[:, :, -1], u[:, :, -1])
    out2 = g.rb_sweep(ud, to_dev(torch, rho), first_colour=first)
    assert torch.equal(out, out2)
    g.close()


# ------------------------------------------------------------- source
@pytest.mark.parametrize("cid,n", [(1, 33), (2, 65), (2, 129)])
def test_pseudo_density_and_moments_match_oracle(torch, L, oracle_mod, cid, n):
    say("pseudo_density config %d n=%d" % (cid, n))
    w = I.config(cid, n_override=n)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    rho, Q = g.pseudo_density(w.atoms, moments=True)
    got = rho.cpu().numpy()
    A = I.atom_arrays(w.atoms)
    want = oracle_mod.pseudo_density(xs, A)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    Qw = oracle_mod.moments(xs, want, 4)
    assert np.abs(Q - Qw).max() <= 1e-11 * np.abs(Qw).max()
    g.close()


def test_quartic_and_interstitial_density(torch, L, oracle_mod):
    say("pseudo_density kind 1 + interstitial")
    rng = np.random.default_rng(13)
    xs = [graded(rng, n, -5, 5) for n in (45, 38, 51)]
    atoms = [I.Atom(center=np.array([0.3, -0.2, 0.1]), q=-1.6, radius=2.3, kind=1, rho_R=0.035, drho_R=-0.089,
                    lmax=2, clm=rng.normal(0, 0.1, 8)),
             I.Atom(center=np.array([-2.0, 1.5, 1.0]), q=3.0, width=0.6, radius=1.2, lmax=4,
                    clm=rng.normal(0, 0.1, 24))]
    inter = rng.uniform(0, 0.01, size=(51, 38, 45))
    g = L.Grid(*xs)
    got = g.pseudo_density(atoms, rho_interstitial=to_dev(torch, inter)).cpu().numpy()
    want = oracle_mod.pseudo_density(xs, I.atom_arrays(atoms), rho_inter=inter)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    got2 = g.pseudo_density(atoms, renormalize=False).cpu().numpy()
    want2 = oracle_mod.pseudo_density(xs, I.atom_arrays(atoms), renormalize=False)
    assert np.abs(got2 - want2).max() <= 1e-12 * np.abs(want2).max()
    g.close()


# --------------------------------------------------------------- solve
def oracle_solution(oracle_mod, xs, atoms, bc=1, rtol=1e-12):
    A = I.atom_arrays(atoms)
    rho = oracle_mod.pseudo_density(xs, A)
    Q = oracle_mod.moments(xs, rho, 4)
    v = np.zeros_like(rho)
    oracle_mod.boundary_values(xs, Q, v, bc, 4)
    cyc, rel, _ = oracle_mod.solve(xs, rho, v, rtol=rtol)
    assert rel <= rtol
    return rho, v


SOLVE_CASES = [
    (1, 33, dict()),
    (1, 25, dict()),                         # 25^3 <= 16384 nodes: the whole cycle in one workgroup
    (1, 25, dict(precision=1, method=1)),
    (1, 17, dict(precision=1)),              # every FP32 level of the cycle fits in LDS
    (1, 17, dict(precision=1, method=1)),
    (2, 65, dict()),
    (2, 65, dict(method=1)),
    (2, 65, dict(precision=1)),
    (2, 65, dict(precision=1, method=1)),
    (2, 129, dict()),
    (2, 129, dict(precision=1)),
    (2, 129, dict(precision=1, method=1)),
    # more sweeps below the finest level than on it (coarse = 2 keeps levels
    # between the finest and the exact solve, where nu_coarse applies)
    (3, 129, dict(precision=1, nu1=3, nu2=3, nu_coarse=4, inner_first=4, inner_iters=8, inner_rate=0.05, coarse=2)),
    (3, 129, dict(nu1=2, nu2=2, nu_coarse=3, coarse=2)),
    (4, 65, dict()),
    (4, 65, dict(precision=1, method=1)),
    # the red-black tail instead of the exact coarsest solve
    (1, 33, dict(coarse=1)),
    (2, 65, dict(coarse=1)),
    (2, 129, dict(precision=1, coarse=1)),
    # the exact solve at the level of at most 16384 nodes, in LDS
    (2, 65, dict(coarse=2)),
    (2, 129, dict(coarse=2)),
    (2, 129, dict(precision=1, coarse=2)),
    # the benchmark's forms on the 55-atom cluster: V(3,3), FP32 PCG with 4
    # then 5 steps per FP64 refinement, and the FP64 PCG
    (3, 129, dict(precision=1, method=0, inner_iters=5, inner_first=4, nu1=3, nu2=3)),
    (3, 129, dict(nu1=3, nu2=3)),
]

# the benchmark's two timed forms (mixed with adaptive inner steps, FP64),
# both from the analytic start, and the fixed-step mixed form from zero
BENCH_FORMS = [dict(precision=1, method=0, nu1=3, nu2=3, inner_first=4, inner_iters=8, inner_rate=0.05, guess=2),
               dict(nu1=3, nu2=3, guess=2),
               dict(precision=1, method=0, inner_iters=5, inner_first=4, nu1=3, nu2=3)]


def start_atoms(form, atoms):
    """the atom tables a form's start needs (guess 2 and 3)"""
    return dict(atoms=atoms) if form.get("guess", 0) >= 2 else {}


@pytest.mark.parametrize("cid,n,opts", SOLVE_CASES)
def test_solve_matches_oracle(torch, L, oracle_mod, cid, n, opts):
    say("solve config %d n=%d %s" % (cid, n, opts))
    w = I.config(cid, n_override=n)
    xs = oracle_mod.mesh_for(w.axes)
    rho_o, v_o = oracle_solution(oracle_mod, xs, w.atoms)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-12, **opts)
    assert info["rel_resid"] <= 1e-12
    got = v.cpu().numpy()
    faces = np.ones(got.shape, bool)
    faces[1:-1, 1:-1, 1:-1] = False
    assert np.abs(got[faces] - v_o[faces]).max() <= 1e-12 * np.abs(v_o[faces]).max()
    err = wnorm(xs, got - v_o) / wnorm(xs, v_o)
    say("  rel W-norm error vs oracle %.3e, iters %d" % (err, info["iters"]))
    assert err <= 1e-9
    # the oracle's own operator confirms the residual
    assert oracle_mod.rel_residual(xs, rho_o, got) <= 2e-12
    g.close()


@pytest.mark.parametrize("form", BENCH_FORMS)
def test_bench_form_at_the_headline_tolerance_matches_oracle(torch, L, oracle_mod, form):
    """The benchmark's forms stopped at its tolerance (1e-10) on the
    55-atom cluster at 129^3: the solution matches the oracle's (solved to
    1e-12) to 1e-9 in the relative W-norm, and the oracle's own operator
    confirms the residual."""
    say("bench form at 1e-10, config 3 n=129 %s" % form)
    w = I.config(3, n_override=129)
    xs = oracle_mod.mesh_for(w.axes)
    rho_o, v_o = oracle_solution(oracle_mod, xs, w.atoms)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-10, **form, **start_atoms(form, w.atoms))
    got = v.cpu().numpy()
    err = wnorm(xs, got - v_o) / wnorm(xs, v_o)
    say("  iters %d vcycles %d refinements %d rel %.2e, error vs oracle %.3e" % (
        info["iters"], info["vcycles"], info["refinements"], info["rel_resid"], err))
    assert info["rel_resid"] <= 1e-10
    assert err <= 1e-9
    assert oracle_mod.rel_residual(xs, rho_o, got) <= 1.05e-10
    g.close()


@pytest.mark.parametrize("batch", [1, 2])
def test_graph_replays_match_eager_launches(torch, L, batch):
    """With graphs = 1 the inner FP32 PCG steps and the FP64 CG's V-cycles
    are captured into HIP graphs and replayed: the same bits as launching
    every kernel from the host, for the mixed and the FP64 CG forms solved
    five times in a row on one grid (the first use eager, the second
    capturing, then replays), with eager work of the program's own between
    the solves, each compared with a solve launched from the host."""
    say("graph replays vs eager launches, config 3 n=%d x %d" % (65 if batch > 1 else 129, batch))
    n = 65 if batch > 1 else 129
    w = I.config(3, n_override=n)
    xs = L.mesh_for(w.axes)
    g = L.Grid(*xs, n_batch=batch)
    atoms = [w.atoms] + [I.perturb_atoms(w.atoms, 70 + b) for b in range(batch - 1)] if batch > 1 else w.atoms
    rho = g.pseudo_density(atoms)
    for form in BENCH_FORMS[:2]:
        ref = g.empty()
        iref = g.poisson_solve(rho, ref, rtol=1e-10, **form, **start_atoms(form, atoms))
        for rep in range(5):
            v = g.empty()
            info = g.poisson_solve(rho, v, rtol=1e-10, graphs=1, **form, **start_atoms(form, atoms))
            assert torch.equal(v, ref), (form, rep)
            assert (info["iters"], info["vcycles"], info["rel_resid"]) == \
                (iref["iters"], iref["vcycles"], iref["rel_resid"])
            assert info["alg_bytes"] == iref["alg_bytes"]
            # eager work of the program's own between the replays
            g.apply(v)
            g.pseudo_density(atoms, rho_out=rho)
            torch.cuda.synchronize()
    g.close()


def test_adaptive_inner_steps_take_fewer_cycles(torch, L):
    """inner_rate > 0: each refinement plans its FP32 step count from the
    current residual and the inner solve's measured convergence. From the
    analytic start the mixed solve then needs fewer V-cycles than the fixed
    4 + 5 steps from zero, and at least one fewer than the fixed steps from
    the same start; every form reaches 1e-10."""
    say("adaptive inner steps, config 3 n=129")
    w = I.config(3, n_override=129)
    xs = L.mesh_for(w.axes)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    base = dict(precision=1, method=0, nu1=3, nu2=3)
    fixed0 = g.poisson_solve(rho, g.empty(), rtol=1e-10, guess=1, inner_first=4, inner_iters=5, **base)
    fixed2 = g.poisson_solve(rho, g.empty(), rtol=1e-10, guess=2, atoms=w.atoms, inner_first=4, inner_iters=5,
                             **base)
    adapt2 = g.poisson_solve(rho, g.empty(), rtol=1e-10, guess=2, atoms=w.atoms, inner_first=4, inner_iters=8,
                             inner_rate=0.05, **base)
    for name, i in (("fixed, zero start", fixed0), ("fixed, analytic start", fixed2),
                    ("adaptive, analytic start", adapt2)):
        say("  %s: %d V-cycles, %d refinements, rel %.2e, q %.3f" % (name, i["vcycles"], i["refinements"],
                                                                    i["rel_resid"], i["inner_rate"]))
        assert i["rel_resid"] <= 1e-10
    assert adapt2["vcycles"] < fixed0["vcycles"] and adapt2["vcycles"] < fixed2["vcycles"]
    assert 0.0 < adapt2["inner_rate"] < 1.0
    with pytest.raises(L.LastoError):
        g.poisson_solve(rho, g.empty(), precision=1, inner_rate=1.0)
    g.close()


@pytest.mark.parametrize("cid,n", [(2, 129), (3, 129), (1, 33), (3, 257)])
def test_exact_coarsest_solve_engaged_and_no_slower_to_converge(torch, L, oracle_mod, cid, n):
    """the cycle's exact coarsest solve runs on the level the options name:
    by GEMMs on the first level below the finest with at most 3e6 nodes
    (when that level is larger than 16384 nodes), in LDS on the first level
    of at most 16384 nodes; either takes no more V-cycles than the red-black
    tail it replaces, to the same tolerance and solution"""
    say("coarsest solve config %d n=%d" % (cid, n))
    w = I.config(cid, n_override=n)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    sizes = [s[0] * s[1] * s[2] for s in g.levels()]
    top = next(l for l, s in enumerate(sizes) if s <= 16384)
    gemm = next(l for l, s in enumerate(sizes) if l >= 1 and s <= 3000000)
    gemm = gemm if sizes[gemm] > 16384 else top
    assert top >= 1
    out = {}
    for prec in (0, 1):
        for coarse in (0, 2, 1):
            v = g.empty()
            info = g.poisson_solve(rho, v, rtol=1e-10, precision=prec, coarse=coarse)
            out[prec, coarse] = (info, v)
            say("  precision %d coarse %d: iters %d vcycles %d level %d" % (
                prec, coarse, info["iters"], info["vcycles"], info["coarse_level"]))
        ref, vref = out[prec, 1]
        assert ref["coarse_level"] == -1 and ref["rel_resid"] <= 1e-10
        # (an FP32 cycle whose LDS tail starts above the LDS level keeps the tail)
        assert out[prec, 0][0]["coarse_level"] == gemm or (gemm == top and prec == 1 and
                                                           out[prec, 0][0]["coarse_level"] == -1)
        assert out[prec, 2][0]["coarse_level"] == top or (prec == 1 and out[prec, 2][0]["coarse_level"] == -1)
        for coarse in (0, 2):
            info, v = out[prec, coarse]
            assert info["rel_resid"] <= 1e-10
            assert info["vcycles"] <= ref["vcycles"]
            d = (v - vref).cpu().numpy()
            assert wnorm(xs, d) <= 1e-8 * wnorm(xs, vref.cpu().numpy())
    g.close()


def test_solve_ragged_noncubic_zero_faces(torch, L, oracle_mod):
    say("solve ragged 70x45x97, bc=0")
    rng = np.random.default_rng(14)
    xs = [graded(rng, n, -8, 8) for n in (70, 45, 97)]
    rho = np.zeros((97, 45, 70))
    rho[1:-1, 1:-1, 1:-1] = rng.normal(size=(95, 43, 68))
    g = L.Grid(*xs)
    v = g.empty()
    info = g.poisson_solve(to_dev(torch, rho), v, rtol=1e-12, bc=0)
    got = v.cpu().numpy()
    want = np.zeros_like(rho)
    cyc, rel, _ = oracle_mod.solve(xs, rho, want, rtol=1e-12)
    err = wnorm(xs, got - want) / wnorm(xs, want)
    assert err <= 1e-9 and info["rel_resid"] <= 1e-12
    assert np.all(got[0] == 0) and np.all(got[:, :, -1] == 0)
    g.close()


# -------------------------------------------------------------- batches
BATCH_OPTS = [dict(), dict(precision=1), dict(method=1), dict(precision=1, method=1), dict(coarse=1),
              dict(precision=1, coarse=1), dict(coarse=2), dict(precision=1, coarse=2)]


@pytest.mark.parametrize("opts", BATCH_OPTS)
def test_batched_solve_matches_oracle_per_copy(torch, L, oracle_mod, opts):
    """Three right-hand sides (SCF-like perturbations of the 13-atom cluster)
    stacked in one grid: every copy matches the oracle's solve of that copy."""
    say("batched solve, 3 x config 2 n=65 %s" % opts)
    w = I.config(2, n_override=65)
    xs = oracle_mod.mesh_for(w.axes)
    batch = [w.atoms] + [I.perturb_atoms(w.atoms, 700 + b) for b in range(2)]
    g = L.Grid(*xs, n_batch=3)
    rho, Q = g.pseudo_density(batch, moments=True)
    assert tuple(rho.shape) == (3, 65, 65, 65) and Q.shape == (3, 25)
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-12, **opts)
    say("  iters %d vcycles %d per-copy rel %s" % (info["iters"], info["vcycles"], info["batch_rel_resid"]))
    assert len(info["batch_rel_resid"]) == 3 and max(info["batch_rel_resid"]) <= 1e-12
    got = v.cpu().numpy()
    for b, atoms in enumerate(batch):
        rho_o, v_o = oracle_solution(oracle_mod, xs, atoms)
        assert np.abs(rho[b].cpu().numpy() - rho_o).max() <= 1e-12 * np.abs(rho_o).max()
        assert np.abs(Q[b] - oracle_mod.moments(xs, rho_o, 4)).max() <= 1e-11 * np.abs(Q[b]).max()
        err = wnorm(xs, got[b] - v_o) / wnorm(xs, v_o)
        say("  copy %d: rel W-norm error vs oracle %.3e" % (b, err))
        assert err <= 1e-9
        assert oracle_mod.rel_residual(xs, rho_o, got[b]) <= 2e-12
    # the batch's sphere values are each copy's own
    centers = np.array([a.center for a in w.atoms])
    radii = np.array([a.radius for a in w.atoms])
    sph = g.sphere_interp(v, centers, radii)
    assert sph.shape == (3, 13, 64)
    pts = oracle_mod.sphere_points(centers, radii, I.default_directions())
    for b in range(3):
        want = oracle_mod.interp(xs, got[b], pts).reshape(13, 64)
        assert np.abs(sph[b] - want).max() <= 1e-13 * np.abs(want).max()
    g.close()


def test_mackay_cluster_batch_matches_oracle_per_copy(torch, L, oracle_mod):
    """The 309-atom Mackay icosahedron with its 8 SCF-like perturbations
    (1 % multiplicative noise on q and c_lm) on one batched grid, at 65^3 per
    copy, in the benchmark's mixed form: each copy's source, moments and
    solution match the oracle's run of that copy, and the sphere values are
    each copy's own."""
    say("batched solve, 8 x config 5 (309 atoms) n=65, bench mixed form")
    w = I.config(5, n_override=65)
    xs = oracle_mod.mesh_for(w.axes)
    assert len(w.atoms) == 309 and len(w.batch_atoms) == 8
    g = L.Grid(*xs, n_batch=8)
    rho, Q = g.pseudo_density(w.batch_atoms, moments=True)
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-12, **BENCH_FORMS[0], **start_atoms(BENCH_FORMS[0], w.batch_atoms))
    say("  iters %d vcycles %d per-copy rel %s" % (info["iters"], info["vcycles"], info["batch_rel_resid"]))
    assert max(info["batch_rel_resid"]) <= 1e-12
    got = v.cpu().numpy()
    centers = np.array([a.center for a in w.atoms])
    radii = np.array([a.radius for a in w.atoms])
    sph = g.sphere_interp(v, centers, radii)
    pts = oracle_mod.sphere_points(centers, radii, I.default_directions())
    for b, atoms in enumerate(w.batch_atoms):
        rho_o, v_o = oracle_solution(oracle_mod, xs, atoms)
        assert np.abs(rho[b].cpu().numpy() - rho_o).max() <= 1e-12 * np.abs(rho_o).max()
        assert np.abs(Q[b] - oracle_mod.moments(xs, rho_o, 4)).max() <= 1e-11 * np.abs(Q[b]).max()
        err = wnorm(xs, got[b] - v_o) / wnorm(xs, v_o)
        say("  copy %d: rel W-norm error vs oracle %.3e" % (b, err))
        assert err <= 1e-9
        want = oracle_mod.interp(xs, got[b], pts).reshape(309, 64)
        assert np.abs(sph[b] - want).max() <= 1e-13 * np.abs(want).max()
    g.close()


def test_batched_operator_and_sweep_match_oracle(torch, L, oracle_mod):
    say("batched apply / rb_sweep (2 copies, ragged)")
    rng = np.random.default_rng(31)
    xs = [graded(rng, n) for n in (37, 21, 18)]
    u = rng.normal(size=(2, 18, 21, 37))
    rho = rng.normal(size=(2, 18, 21, 37))
    g = L.Grid(*xs, n_batch=2)
    Au = g.apply(to_dev(torch, u)).cpu().numpy()
    sw = g.rb_sweep(to_dev(torch, u), to_dev(torch, rho)).cpu().numpy()
    I_ = (slice(1, -1),) * 3
    for b in range(2):
        want = oracle_mod.apply(xs, u[b])
        assert np.abs(Au[b][I_] - want[I_]).max() <= 1e-13 * np.abs(want[I_]).max()
        want = oracle_mod.rb_sweep(xs, u[b], rho[b], 0)
        assert np.abs(sw[b] - want).max() <= 1e-12 * np.abs(want).max()
    g.close()


def test_analytic_guess_matches_closed_form(torch, L):
    """lasto_analytic_guess: the monopole field of every atom at each
    interior node (Gaussian: -q erf(r/w)/r, with its r -> 0 limit; quartic:
    the uniform ball of radius R), faces untouched."""
    from scipy.special import erf
    rng = np.random.default_rng(11)
    xs = [graded(rng, n) for n in (37, 29, 33)]
    g = L.Grid(*xs)
    node = np.array([xs[0][18], xs[1][14], xs[2][16]])   # an atom exactly on a node
    atoms = [I.Atom(center=node, q=9.0, width=0.6),
             I.Atom(center=np.array([1.3, -2.2, 0.7]), q=10.5, width=0.85),
             I.Atom(center=np.array([-4.0, 3.1, -1.9]), q=8.0, width=0.5),
             I.Atom(center=np.array([2.9, 2.4, -3.3]), q=11.0, radius=1.7, kind=1),
             I.Atom(center=np.array([-2.5, -3.6, 3.8]), q=7.5, radius=2.1, kind=1)]
    v0 = rng.standard_normal((33, 29, 37))
    v = to_dev(torch, v0)
    g.analytic_guess(atoms, v)
    got = v.cpu().numpy()
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    want = np.zeros_like(v0)
    for a in atoms:
        r = np.sqrt((X - a.center[0]) ** 2 + (Y - a.center[1]) ** 2 + (Z - a.center[2]) ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            if a.kind == 0:
                f = np.where(r > 1e-12 * a.width, erf(r / a.width) / r, 2.0 / (math.sqrt(math.pi) * a.width))
            else:
                R = a.radius
                f = np.where(r < R, (3 * R * R - r * r) / (2 * R ** 3), 1.0 / r)
        want -= a.q * f
    faces = np.ones(v0.shape, bool)
    faces[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(got[faces], v0[faces])
    err = np.abs(got - want)[~faces].max() / np.abs(want[~faces]).max()
    say("  analytic guess max rel error %.2e" % err)
    # the far field (-q/r beyond 6w or R) is summed in FP32 partial sums of
    # at most 32 atoms, near fields in FP64: the guess only starts the
    # iteration, and its own distance from the discrete solution (no l >= 1
    # terms, no discretisation) is ~1e-3
    assert err <= 40 * 2.0 ** -24
    g.close()


@pytest.mark.parametrize("nb,shared", [(8, True), (3, True), (2, False)])
def test_batched_analytic_guess_matches_each_copy(torch, L, nb, shared):
    """Copies whose atoms differ only in charge share one pass over the
    node-atom pairs (groups of 8, 4, 2, then single copies); every copy's
    guess equals, bit for bit, the guess of a grid holding that copy alone,
    and so does a batch whose copies differ in geometry."""
    say("batched analytic guess, %d copies, shared geometry %s" % (nb, shared))
    w = I.config(2, n_override=57)
    xs = L.mesh_for(w.axes)
    if shared:
        batch = [I.perturb_atoms(w.atoms, 90 + b, rel=0.05) for b in range(nb)]
    else:
        batch = [w.atoms, [dataclasses.replace(a, center=a.center + 0.3) for a in w.atoms]]
    gb = L.Grid(*xs, n_batch=nb)
    vb = gb.analytic_guess(batch, gb.empty())
    g1 = L.Grid(*xs)
    for b in range(nb):
        v1 = g1.analytic_guess(batch[b], g1.empty())
        assert torch.equal(v1, vb[b]), b
    g1.close()
    gb.close()


def test_analytic_guess_many_atoms_matches_closed_form(torch, L):
    """More atoms than one staging chunk of the guess kernel (512): 700
    Gaussian atoms scattered over the box, some of them off the mesh."""
    from scipy.special import erf
    rng = np.random.default_rng(12)
    xs = [graded(rng, n) for n in (35, 27, 31)]
    g = L.Grid(*xs)
    lo = np.array([x[0] for x in xs]) - 1.0
    hi = np.array([x[-1] for x in xs]) + 1.0
    atoms = [I.Atom(center=lo + (hi - lo) * rng.random(3), q=float(rng.uniform(0.5, 2.0)),
                    width=float(rng.uniform(0.3, 0.7))) for _ in range(700)]
    v = to_dev(torch, np.zeros((31, 27, 35)))
    g.analytic_guess(atoms, v)
    got = v.cpu().numpy()[1:-1, 1:-1, 1:-1]
    Z, Y, X = np.meshgrid(xs[2][1:-1], xs[1][1:-1], xs[0][1:-1], indexing="ij")
    want = np.zeros_like(got)
    for a in atoms:
        r = np.sqrt((X - a.center[0]) ** 2 + (Y - a.center[1]) ** 2 + (Z - a.center[2]) ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            f = np.where(r > 1e-12 * a.width, erf(r / a.width) / r, 2.0 / (math.sqrt(math.pi) * a.width))
        want -= a.q * f
    err = np.abs(got - want).max() / np.abs(want).max()
    say("  analytic guess, 700 atoms: max rel error %.2e" % err)
    # FP32 partial sums of 32 same-sign terms: (32 + a few ulp per term) * 2^-24
    assert err <= 40 * 2.0 ** -24
    g.close()


def test_levels_match_oracle_hierarchy(torch, L, oracle_mod):
    w = I.config(3)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    got = np.array(g.levels())
    want = oracle_mod.hierarchy_sizes(xs)
    assert np.array_equal(got, want)
    g.close()


def test_sphere_interp_matches_oracle(torch, L, oracle_mod):
    say("sphere interp config 2 n=129")
    w = I.config(2)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    res = L.hartree_step(g, w.atoms)
    v = res["v"].cpu().numpy()
    A = I.atom_arrays(w.atoms)
    pts = oracle_mod.sphere_points(A["centers"], A["radius"], I.default_directions())
    want = oracle_mod.interp(xs, v, pts).reshape(len(w.atoms), 64)
    assert np.abs(res["sphere"] - want).max() <= 1e-13 * np.abs(want).max()
    # explicit directions; radius 0 puts the point exactly on a node, where
    # the interpolant returns that node's value
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0]])
    c = np.array([[xs[0][60], xs[1][70], xs[2][64]]])
    got = g.sphere_interp(res["v"], c, [0.0], d)
    assert got[0, 0] == v[64, 70, 60] and got[0, 1] == v[64, 70, 60]
    g.close()


# --------------------------------------------------- full-size properties
def test_full_size_257_properties(torch, L, oracle_mod):
    """The 55-atom 257^3 workload: the oracle's operator confirms the GPU
    residual for the FP64 and the mixed solve, the two agree, the discrete
    Gauss law holds, and sampled density values match the oracle."""
    say("full size 257^3 config 3")
    w = I.config(3)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    v64 = g.empty()
    i64 = g.poisson_solve(rho, v64, rtol=1e-10)
    v32 = g.empty()
    i32 = g.poisson_solve(rho, v32, rtol=1e-10, precision=1)
    vmg = g.empty()
    img = g.poisson_solve(rho, vmg, rtol=1e-10, precision=1, method=1)
    say("  fp64 iters %d (%.1f ms), mixed PCG refinements %d vcycles %d (%.1f ms), "
        "mixed MG refinements %d vcycles %d (%.1f ms)" %
        (i64["iters"], i64["ms_total"], i32["refinements"], i32["vcycles"], i32["ms_total"],
         img["refinements"], img["vcycles"], img["ms_total"]))
    rho_h = rho.cpu().numpy()
    a = v64.cpu().numpy()
    b = v32.cpu().numpy()
    c = vmg.cpu().numpy()
    assert oracle_mod.rel_residual(xs, rho_h, a) <= 1.2e-10
    assert oracle_mod.rel_residual(xs, rho_h, b) <= 1.2e-10
    assert oracle_mod.rel_residual(xs, rho_h, c) <= 1.2e-10
    assert wnorm(xs, a - b) / wnorm(xs, a) <= 1e-8
    assert wnorm(xs, a - c) / wnorm(xs, a) <= 1e-8
    # sampled density values against the oracle's full evaluation
    want = oracle_mod.pseudo_density(xs, I.atom_arrays(w.atoms))
    rng = np.random.default_rng(15)
    idx = tuple(rng.integers(0, 257, size=(3, 20000)))
    assert np.abs(rho_h[idx] - want[idx]).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(rho_h - want).max() <= 1e-12 * np.abs(want).max()
    # Gauss: flux through the faces = 4 pi * interior charge (to the tolerance)
    mx, my, mz = (dual(x) for x in xs)
    hx, hy, hz = (np.diff(x) for x in xs)
    s = slice(1, -1)
    flux = ((a[s, s, 0] - a[s, s, 1]) / hx[0] * np.outer(mz[s], my[s])).sum()
    flux += ((a[s, s, -1] - a[s, s, -2]) / hx[-1] * np.outer(mz[s], my[s])).sum()
    flux += ((a[s, 0, s] - a[s, 1, s]) / hy[0] * np.outer(mz[s], mx[s])).sum()
    flux += ((a[s, -1, s] - a[s, -2, s]) / hy[-1] * np.outer(mz[s], mx[s])).sum()
    flux += ((a[0, s, s] - a[1, s, s]) / hz[0] * np.outer(my[s], mx[s])).sum()
    flux += ((a[-1, s, s] - a[-2, s, s]) / hz[-1] * np.outer(my[s], mx[s])).sum()
    vol = np.einsum("k,j,i->kji", mz, my, mx)
    q_in = (vol * rho_h)[s, s, s].sum()
    assert abs(flux - 4 * math.pi * q_in) <= 1e-6 * 4 * math.pi * abs(q_in)
    g.close()


# ------------------------------------------------------------ edge cases
def test_failure_paths(torch, L, oracle_mod):
    say("failure paths")
    w = I.config(2, n_override=57)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    # too few iterations: NOT_CONVERGED with info filled and a finite iterate
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-12, max_iters=1, allow_fail=True)
    assert info["status"] == L.ERR_NOT_CONVERGED and info["iters"] == 1 and 0 < info["rel_resid"] < 1
    assert torch.isfinite(v).all()
    # injected NaN: DIVERGED, iterate still finite
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-12, debug_nan_iter=2, allow_fail=True)
    assert info["status"] == L.ERR_DIVERGED
    assert torch.isfinite(v).all()
    # NaN in the source: ERR_ARG
    bad = rho.clone()
    bad[5, 5, 5] = float("nan")
    with pytest.raises(L.LastoError) as e:
        g.poisson_solve(bad, g.empty())
    assert e.value.status == L.ERR_ARG
    # bad options
    with pytest.raises(L.LastoError):
        g.poisson_solve(rho, g.empty(), nu1=0)
    with pytest.raises(L.LastoError):
        g.poisson_solve(rho, g.empty(), precision=1, method=2)
    with pytest.raises(L.LastoError):
        g.poisson_solve(rho, g.empty(), precision=1, inner_iters=0)
    # faces as given (bc = 2) are kept
    v = g.empty()
    v[0].fill_(1.25)
    g.poisson_solve(rho, v, bc=2, rtol=1e-10)
    assert bool((v[0] == 1.25).all())
    # a point outside the box
    with pytest.raises(L.LastoError):
        g.sphere_interp(v, np.array([[100.0, 0, 0]]), [1.0])
    # guess = 1 ignores the interior given
    v1 = g.empty()
    v1.fill_(7.0)
    g.poisson_solve(rho, v1, guess=1, rtol=1e-12)
    v2 = g.empty()
    g.poisson_solve(rho, v2, rtol=1e-12)
    assert float((v1 - v2).abs().max()) <= 1e-9 * float(v2.abs().max())
    # a problem the faces alone solve (rho = 0, zero faces): OK, the zero
    # interior, no iteration, in every form
    zero = torch.zeros_like(rho)
    for opts in (dict(), dict(precision=1), dict(method=1)):
        v3 = g.empty()
        v3.fill_(3.0)
        info = g.poisson_solve(zero, v3, bc=0, **opts)
        assert info["rel_resid"] == 0.0 and info["iters"] == 0
        assert float(v3.abs().max()) == 0.0
    g.close()


def test_mixed_form_falls_back_to_fp64(torch, L, oracle_mod):
    """The fallback of the mixed form, forced from the host: a NaN injected
    into the FP32 inner solve's right-hand side (its correction never reaches
    v), and a refinement budget too small for the tolerance. Both finish as
    FP64 MG-PCG from the current iterate and match the oracle; with the
    fallback off the first returns DIVERGED with a finite v."""
    say("mixed-form fallback, config 2 n=65")
    w = I.config(2, n_override=65)
    xs = oracle_mod.mesh_for(w.axes)
    rho_o, v_o = oracle_solution(oracle_mod, xs, w.atoms)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    for opts in (dict(debug_nan_iter=1), dict(max_iters=10, inner_iters=1), dict(debug_nan_iter=0, method=1)):
        v = g.empty()
        info = g.poisson_solve(rho, v, rtol=1e-12, precision=1, **opts)
        err = wnorm(xs, v.cpu().numpy() - v_o) / wnorm(xs, v_o)
        say("  %s: fallback %d iters %d refinements %d rel %.2e err %.2e" % (
            opts, info["fallback_used"], info["iters"], info["refinements"], info["rel_resid"], err))
        assert info["fallback_used"] & 2 and info["rel_resid"] <= 1e-12 and err <= 1e-9
    v = g.empty()
    info = g.poisson_solve(rho, v, rtol=1e-12, precision=1, debug_nan_iter=1, fallback=0, allow_fail=True)
    assert info["status"] == L.ERR_DIVERGED and info["fallback_used"] == 0
    assert torch.isfinite(v).all()
    # without trouble the mixed form needs no fallback
    info = g.poisson_solve(rho, g.empty(), rtol=1e-12, precision=1)
    assert info["fallback_used"] == 0
    g.close()


@pytest.mark.parametrize("nb", [1, 2])
def test_analytic_start_option_and_phase_report(torch, L, oracle_mod, nb):
    """guess = 2 starts from the analytic superposition inside the solve:
    the same iterate as lasto_analytic_guess followed by a solve of v as
    given, fewer iterations than the zero start, the oracle's solution; the
    info reports the phases and the finest level's algorithmic bytes."""
    say("guess 2, config 2 n=65, %d copies" % nb)
    w = I.config(2, n_override=65)
    xs = oracle_mod.mesh_for(w.axes)
    batch = [w.atoms] + [I.perturb_atoms(w.atoms, 900 + b) for b in range(nb - 1)]
    atoms = batch if nb > 1 else w.atoms
    g = L.Grid(*xs, n_batch=nb)
    rho = g.pseudo_density(atoms)
    v2 = g.empty()
    i2 = g.poisson_solve(rho, v2, rtol=1e-12, guess=2, atoms=atoms)
    v0 = g.empty()
    g.boundary_values(rho, v0)
    g.analytic_guess(atoms, v0)
    i0 = g.poisson_solve(rho, v0, rtol=1e-12)
    assert torch.equal(v0, v2) and i0["iters"] == i2["iters"]
    iz = g.poisson_solve(rho, g.empty(), rtol=1e-12, guess=1)
    say("  iters analytic %d zero %d; ms bc %.3f guess %.3f cycles %.3f total %.3f; %.0f B per node per V-cycle"
        % (i2["iters"], iz["iters"], i2["ms_bc"], i2["ms_guess"], i2["ms_cycles"], i2["ms_total"],
           i2["alg_bytes"] / (i2["vcycles"] * nb * 63 ** 3)))
    assert i2["iters"] < iz["iters"]
    assert i2["ms_bc"] > 0 and i2["ms_guess"] > 0 and i2["ms_cycles"] > 0
    assert i2["ms_bc"] + i2["ms_guess"] + i2["ms_cycles"] <= i2["ms_total"]
    # FP64 V(2,2) MG-PCG at the finest level, per node and iteration: the
    # cycle (8 half-sweeps 92 B, red residual 16 B, restriction and
    # prolongation 14 B plus the coarse level's share) and the Krylov streams
    # (update of p, A p, update of x and r: 96 B), about 220 B
    assert 190 <= i2["alg_bytes"] / (i2["vcycles"] * nb * 63 ** 3) <= 260
    got = v2.cpu().numpy()
    for b, a in enumerate(batch):
        _, v_o = oracle_solution(oracle_mod, xs, a)
        gb = got[b] if nb > 1 else got
        assert wnorm(xs, gb - v_o) / wnorm(xs, v_o) <= 1e-9
    # the atom tables are required
    with pytest.raises(L.LastoError):
        g.poisson_solve(rho, g.empty(), guess=2)
    g.close()


def test_scratch_users_leave_the_solver_clean(torch, L, oracle_mod):
    """lasto_rb_sweep borrows the solver's vectors: a solve after it on the
    same grid gives the same bits as before it."""
    say("solve, rb_sweep, solve on one grid")
    w = I.config(2, n_override=57)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    v1 = g.empty()
    g.poisson_solve(rho, v1, rtol=1e-11)
    rng = np.random.default_rng(17)
    u = to_dev(torch, rng.normal(size=rho.shape) * 50.0)
    g.rb_sweep(u, rho)
    v2 = g.empty()
    g.poisson_solve(rho, v2, rtol=1e-11)
    assert torch.equal(v1, v2)
    g.close()


def test_profile_counts_sweeps(torch, L, oracle_mod):
    w = I.config(2, n_override=65)
    xs = oracle_mod.mesh_for(w.axes)
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    info = g.poisson_solve(rho, g.empty(), profile=1)
    # V(2,2): four sweeps of two half-sweeps each on the finest level
    assert info["smooth_launches"] == 8 * info["vcycles"]
    assert info["smooth_ms"] > 0
    # 24 B per interior node per sweep, less 4 B for the sweep from zero
    n_int = 63 ** 3
    assert abs(info["smooth_bytes"] - info["vcycles"] * n_int * (4 * 24 - 4)) < 1e-6 * info["smooth_bytes"]
    info = g.poisson_solve(rho, g.empty())
    assert info["smooth_launches"] == 0
    g.close()
