"""The fused smoothing pass (several red-black half-sweeps of the multigrid
smoother in one pass over a level, lasto_smooth with fused = 1) against one
launch per half-sweep, which must give the same bits, and against the
oracle's red-black sweeps; then solves with the fused pass forced on every
level against solves without it."""
import math
import sys

import numpy as np
import pytest

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


# (shape nx, ny, nz; right-hand sides; level): ragged x tiles (131: 66 colour
# entries, three 32-entry tiles), fewer rows than a tile (9), the smallest
# grid, a batch (copy faces inside the stacked planes), and a coarse level
CASES = [((131, 37, 41), 1, 0), ((70, 9, 19), 1, 0), ((4, 4, 4), 1, 0), ((37, 21, 18), 2, 0),
         ((65, 57, 61), 1, 1)]


def level_coords(g, xs, level):
    idx = g.level_nodes(level)
    return [xs[d][idx[d]] for d in range(3)]


def zero_faces(a):
    a = a.copy()
    a[..., 0, :, :] = 0.0
    a[..., -1, :, :] = 0.0
    a[..., :, 0, :] = 0.0
    a[..., :, -1, :] = 0.0
    a[..., :, :, 0] = 0.0
    a[..., :, :, -1] = 0.0
    return a


@pytest.fixture(scope="module")
def grids(L):
    made = {}
    yield made
    for g, _ in made.values():
        g.close()


def grid_for(L, grids, shape, nb):
    key = (shape, nb)
    if key not in grids:
        rng = np.random.default_rng(7 + sum(shape) + nb)
        xs = [graded(rng, n) for n in shape]
        grids[key] = (L.Grid(*xs, n_batch=nb), xs)
    return grids[key]


def mismatch(a, b):
    """where and by how much two results differ (for the failure message)"""
    d = np.abs(a - b)
    idx = np.argwhere(d > 0)
    rel = d.max() / max(np.abs(a).max(), 1e-300)
    lo, hi = idx.min(axis=0), idx.max(axis=0)
    return "fused pass differs from the half-sweeps at %d nodes, max |diff| %.3e (rel %.3e), index range %s..%s" % (
        len(idx), d.max(), rel, lo.tolist(), hi.tolist())


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", [0, 1])
def test_fused_pass_matches_one_launch_per_half_sweep(torch, L, grids, case, precision):
    shape, nb, level = case
    g, xs = grid_for(L, grids, shape, nb)
    lshape = g.levels()[level]
    full = (nb,) + tuple(lshape[::-1]) if nb > 1 else tuple(lshape[::-1])
    rng = np.random.default_rng(100 + level + 3 * precision)
    f0 = zero_faces(rng.normal(size=full))
    u0 = zero_faces(rng.normal(size=full))
    for nsw in ((2, 4, 6) if precision else (2, 4)):
        for first in (0, 1):
            for zero_in in (0, 1):
                say("smooth %s nb=%d level=%d prec=%d nsweeps=%d first=%d zero_in=%d"
                    % (shape, nb, level, precision, nsw, first, zero_in))
                f = torch.from_numpy(f0).cuda()
                outs, dots = [], []
                for fused in (0, 1):
                    u = torch.from_numpy(u0).cuda()
                    d = g.smooth(level, f, u, nsw, first, bool(zero_in), bool(fused), precision, dot=not zero_in)
                    outs.append(u.cpu().numpy())
                    dots.append(d)
                assert np.array_equal(outs[0], outs[1]), mismatch(outs[0], outs[1])
                if not zero_in:
                    assert abs(dots[1] - dots[0]) <= 1e-12 * abs(dots[0])
                    # the dot is <f, u>_W over the interior nodes of the result
                    lx = level_coords(g, xs, level)
                    vol = np.einsum("k,j,i->kji", dual(lx[2]), dual(lx[1]), dual(lx[0]))
                    fu = (f0 * outs[1]).reshape((nb,) + tuple(lshape[::-1]))
                    want = sum(float((vol * fu[b])[1:-1, 1:-1, 1:-1].sum()) for b in range(nb))
                    # (FP32: f and the x volume factors are rounded to FP32)
                    tol = 1e-10 if precision == 0 else 1e-6
                    assert abs(dots[1] - want) <= tol * np.abs(vol[None] * fu).sum()


@pytest.mark.parametrize("case", CASES)
def test_fused_pass_matches_oracle_sweeps(torch, L, oracle_mod, grids, case):
    """nsweeps half-sweeps from first_colour are nsweeps / 2 red-black sweeps
    of the oracle (on A u = 4 pi rho, so rho = f / (4 pi)), faces zero."""
    shape, nb, level = case
    g, xs = grid_for(L, grids, shape, nb)
    lshape = g.levels()[level]
    lx = level_coords(g, xs, level)
    full = (nb,) + tuple(lshape[::-1])
    rng = np.random.default_rng(200 + level)
    f0 = zero_faces(rng.normal(size=full))
    u0 = zero_faces(rng.normal(size=full))
    for nsw in (2, 4):
        for first in (0, 1):
            for zero_in in (0, 1):
                say("smooth vs oracle %s nb=%d level=%d nsweeps=%d first=%d zero_in=%d"
                    % (shape, nb, level, nsw, first, zero_in))
                f = torch.from_numpy(f0.reshape(full if nb > 1 else full[1:])).cuda()
                u = torch.from_numpy(u0.reshape(full if nb > 1 else full[1:])).cuda()
                g.smooth(level, f, u, nsw, first, bool(zero_in), True, 0)
                got = u.cpu().numpy().reshape(full)
                for b in range(nb):
                    w = np.zeros_like(u0[b]) if zero_in else u0[b].copy()
                    for _ in range(nsw // 2):
                        w = oracle_mod.rb_sweep(lx, w, f0[b] / (4.0 * math.pi), first)
                    I_ = (slice(1, -1),) * 3
                    scale = max(np.abs(w[I_]).max(), 1e-300)
                    assert np.abs(got[b][I_] - w[I_]).max() <= 1e-12 * scale


def test_smooth_rejects_bad_arguments(torch, L, grids):
    g, _ = grid_for(L, grids, (37, 21, 18), 2)
    f = g.empty()
    u = g.empty()
    for args in [dict(nsweeps=3), dict(nsweeps=8), dict(first_colour=2), dict(level=99), dict(precision=2)]:
        kw = dict(level=0, nsweeps=2, first_colour=0, precision=0)
        kw.update(args)
        with pytest.raises(L.LastoError):
            g.smooth(kw["level"], f, u, kw["nsweeps"], kw["first_colour"], precision=kw["precision"])
    with pytest.raises(L.LastoError):
        g.smooth(0, f, u, 2, 0, zero_in=True, dot=True)
    with pytest.raises(L.LastoError):   # a fused FP64 pass takes at most 4 half-sweeps
        g.smooth(0, f, u, 6, 0, precision=0)
    with pytest.raises(L.LastoError):
        g.smooth(0, f, f, 2, 0)


@pytest.mark.parametrize("opts", [dict(precision=1, inner_iters=6, nu1=3, nu2=3),
                                  dict(precision=0, nu1=2, nu2=2),
                                  dict(precision=1, method=1, inner_iters=4, nu1=1, nu2=3),
                                  dict(precision=0, nu1=3, nu2=1, coarse=1)])
@pytest.mark.parametrize("fuse", [2, 4, 6])
def test_solve_with_fused_passes_everywhere(torch, L, oracle_mod, opts, fuse):
    """The solve with the fused passes forced on every level that sweeps
    converges like the one-launch-per-half-sweep solve (the same V-cycles up
    to the order of the <r, z> sums) to the same solution."""
    from paper_0806_1723_amd import inputs as I
    w = I.config(2, n_override=65)
    xs = oracle_mod.mesh_for(w.axes)
    say("solve fused_sweeps=%d %s" % (fuse, opts))
    g = L.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    res = []
    for fs in (1, fuse):
        v = g.empty()
        info = g.poisson_solve(rho, v, rtol=1e-10, fused_sweeps=fs, **opts)
        res.append((v.cpu().numpy(), info))
    (v1, i1), (v2, i2) = res
    say("  vcycles %d / %d, rel %.2e / %.2e" % (i1["vcycles"], i2["vcycles"], i1["rel_resid"], i2["rel_resid"]))
    assert i2["rel_resid"] <= 1e-10 and i1["rel_resid"] <= 1e-10
    assert abs(i2["vcycles"] - i1["vcycles"]) <= 1
    vol = np.einsum("k,j,i->kji", dual(xs[2]), dual(xs[1]), dual(xs[0]))
    err = math.sqrt(float((vol * (v2 - v1) ** 2).sum())) / math.sqrt(float((vol * v1 ** 2).sum()))
    assert err <= 1e-9
    g.close()
