"""GPU parity and behaviour of the learned-guess network: its BF16 matrix-core
kernels against the CPU reference (oracle/net_ref.py) on identical BF16
operands, training by the library's own backward pass, and the learned guess
judged by plain multigrid."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CH = (16, 32, 48, 64)


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


@pytest.fixture(scope="module")
def R():
    from oracle import net_ref
    return net_ref


def _features(torch, rng, shape):
    """random BF16 features as int16 bit patterns on the device, and their values"""
    a = torch.from_numpy(rng.normal(size=shape + (8,)).astype(np.float32)).to(torch.bfloat16)
    bits = a.view(torch.int16).contiguous().to("cuda")
    return bits, a.to(torch.float64).numpy()


def _net_with_biases(L, rng, shape, ch=CH, seed=3):
    net = L.Net(shape, ch=ch, seed=seed)
    p = net.params().astype(np.float64)
    from oracle import net_ref as R
    o = 0
    for ci, co, _ in R.layer_specs(ch):
        o += 27 * ci * co
        p[o:o + co] = rng.normal(scale=0.05, size=co)
        o += co
    p[o:o + ch[0]] = rng.normal(scale=0.3, size=ch[0])
    p[o + ch[0]] = 0.1
    net.set_params(p.astype(np.float32))
    return net, net.params().astype(np.float64)


# (93, 94, 95): levels of 0.83 M and 0.11 M nodes, where the stride-1
# convolutions take their LDS-staged form (8 and 32 input channels)
@pytest.mark.parametrize("shape,ch", [((20, 27, 37), CH), ((9, 16, 8), CH), ((93, 94, 95), (16, 32, 16, 16))])
def test_net_forward_matches_reference(torch, L, R, shape, ch):
    say("net forward %s ch %s" % (shape, ch))
    rng = np.random.default_rng(21)
    net, p = _net_with_biases(L, rng, shape, ch=ch)
    x_bits, x = _features(torch, rng, shape)
    y = net.forward(x_bits).cpu().numpy().astype(np.float64)
    want = R.forward(x, p, ch, bf16=True).numpy()
    err = np.linalg.norm(y - want) / np.linalg.norm(want)
    exact = R.forward(x, p, ch, bf16=False).numpy()
    rounding = np.linalg.norm(want - exact) / np.linalg.norm(exact)
    say("  rel L2 %.3e, max %.3e of %.3e (rounded reference vs unrounded FP64: %.3e)" % (
        err, np.abs(y - want).max(), np.abs(want).max(), rounding))
    # Both sides round every activation to BF16, the GPU from FP32
    # accumulators and the reference from FP64: where the two pre-rounding
    # values straddle a rounding boundary they round apart, and such
    # differences cascade through the net's eleven rounded stages. The GPU
    # then stays closer to the rounded reference than that reference is to
    # unrounded arithmetic (0.6x at every shape measured).
    assert err <= 0.75 * rounding + 1e-6
    assert err <= 5e-3
    assert np.abs(y - want).max() <= 2e-2 * np.abs(want).max()
    net.close()


def test_net_gradients_match_reference(torch, L, R):
    shape = (12, 17, 21)
    say("net gradients %s" % (shape,))
    rng = np.random.default_rng(22)
    net, p = _net_with_biases(L, rng, shape)
    x_bits, x = _features(torch, rng, shape)
    t = rng.normal(size=shape).astype(np.float32)
    wt = (rng.uniform(0.5, 1.5, size=shape) / np.prod(shape)).astype(np.float32)
    net.forward(x_bits)
    loss = net.backward(x_bits, torch.from_numpy(t).cuda(), torch.from_numpy(wt).cuda())
    g = net.grads().astype(np.float64)
    L_ref, g_ref = R.loss_and_grads(x, p, CH, t.astype(np.float64), wt.astype(np.float64), bf16=True)
    assert abs(loss - L_ref) <= 1e-3 * abs(L_ref)
    # per parameter tensor (BF16 rounding of the backward's intermediates bounds the agreement)
    o = 0
    scale = np.linalg.norm(g_ref)
    for k, (ci, co, _) in enumerate(R.layer_specs(CH)):
        for name, size in (("W", 27 * ci * co), ("b", co)):
            a, b = g[o:o + size], g_ref[o:o + size]
            err = np.linalg.norm(a - b)
            say("  layer %d %s: rel %.3e" % (k, name, err / max(np.linalg.norm(b), 1e-300)))
            assert err <= 3e-2 * np.linalg.norm(b) + 1e-6 * scale
            o += size
    a, b = g[o:], g_ref[o:]
    assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b) + 1e-6 * scale
    net.close()


def test_net_training_lowers_the_loss(torch, L):
    shape = (17, 17, 17)
    say("net training %s" % (shape,))
    rng = np.random.default_rng(23)
    net = L.Net(shape, ch=(16, 16, 16, 16), seed=4)
    x_bits, x = _features(torch, rng, shape)
    # a smooth target the features determine: a blurred feature channel
    t = torch.from_numpy(np.tanh(x[..., 0] + 0.5 * x[..., 4]).astype(np.float32)).cuda()
    wt = torch.full(shape, 1.0 / np.prod(shape), dtype=torch.float32, device="cuda")
    losses = [net.train_step(x_bits, t, wt, 3e-3) for _ in range(60)]
    say("  loss %.4e -> %.4e" % (losses[0], losses[-1]))
    assert losses[-1] < 0.5 * losses[0]
    assert all(np.isfinite(losses))
    # deterministic: the same steps from the same start give the same loss
    net2 = L.Net(shape, ch=(16, 16, 16, 16), seed=4)
    losses2 = [net2.train_step(x_bits, t, wt, 3e-3) for _ in range(60)]
    assert losses2 == losses
    net.close()
    net2.close()


def test_net_checkpoint_resumes_training_bit_for_bit(torch, L, tmp_path):
    """lasto_net_save / lasto_net_load: five Adam steps, a checkpoint, five
    more; a fresh net (other seed and scales) loaded from the checkpoint takes
    the same five steps with the same losses and parameters bit for bit, and
    has the checkpoint's step count and scales. Foreign files and other
    channel counts are refused."""
    shape = (17, 19, 18)
    say("net checkpoint %s" % (shape,))
    rng = np.random.default_rng(24)
    ch = (16, 32, 16, 16)
    x_bits, x = _features(torch, rng, shape)
    t = torch.from_numpy(np.tanh(x[..., 0] - 0.3 * x[..., 4]).astype(np.float32)).cuda()
    wt = torch.full(shape, 1.0 / np.prod(shape), dtype=torch.float32, device="cuda")
    a = L.Net(shape, ch=ch, seed=11, rho_scale=0.2, pot_scale=0.03, h_ref=0.3, out_scale=2.0)
    first = [a.train_step(x_bits, t, wt, 3e-3) for _ in range(5)]
    path = str(tmp_path / "net.ckpt")
    a.save(path)
    rest = [a.train_step(x_bits, t, wt, 2e-3) for _ in range(5)]
    pa = a.params()
    b = L.Net(shape, ch=ch, seed=99)
    b.load_checkpoint(path)
    assert b.adam_steps() == 5
    assert (b.cfg.seed, b.cfg.rho_scale, b.cfg.pot_scale, b.cfg.h_ref, b.cfg.out_scale) == (11, 0.2, 0.03, 0.3, 2.0)
    rest_b = [b.train_step(x_bits, t, wt, 2e-3) for _ in range(5)]
    assert rest_b == rest and all(np.isfinite(first))
    assert np.array_equal(b.params(), pa) and b.adam_steps() == 10
    # refused: other channel counts, a file that is not a checkpoint
    c = L.Net(shape, ch=(16, 16, 16, 16), seed=1)
    with pytest.raises(L.LastoError):
        c.load_checkpoint(path)
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a checkpoint" * 8)
    with pytest.raises(L.LastoError):
        b.load_checkpoint(str(junk))
    for n in (a, b, c):
        n.close()


def test_learned_guess_on_a_batch_matches_each_copy_alone(torch, L):
    """The learned guess on a batched grid (three SCF-like perturbations of a
    random config-4 cluster at 34^3) judges every copy on its own, with the
    same bits as a grid holding that copy alone; the solve's guess = 3 runs
    the same judge and reports how many learned starts it kept. (The node
    colours of the stacked sweeps follow the stacked plane index, so with an
    even plane count every copy sweeps red first, as a grid of its own does.)"""
    from paper_0806_1723_amd import inputs as I
    from paper_0806_1723_amd import learned
    n = 34
    say("learned guess on a batch, config 4 n=%d x 3" % n)
    w = I.config(4, n_override=n, sample=3)
    xs = L.mesh_for(w.axes)
    batch = [w.atoms] + [I.perturb_atoms(w.atoms, 50 + b, rel=0.2) for b in range(2)]
    net = L.Net((n, n, n), ch=(16, 16, 16, 16), seed=3, **learned.NET_SCALES)

    def start(g, atoms):
        rho = g.pseudo_density(atoms)
        v = g.empty()
        g.boundary_values(rho, v)
        g.analytic_guess(atoms, v)
        return rho, v

    gb = L.Grid(*xs, n_batch=3)
    rho_b, v_b = start(gb, batch)
    rb = gb.learned_guess(net, rho_b, v_b)
    acc = 0
    for b in range(3):
        g1 = L.Grid(*xs)
        rho1, v1 = start(g1, batch[b])
        r1 = g1.learned_guess(net, rho1, v1)
        say("  copy %d: plain %.3e learned %.3e accepted %s" % (b, r1["rel_before"], r1["rel_after"], r1["accepted"]))
        assert torch.equal(v1, v_b[b])
        assert (r1["rel_before"], r1["rel_after"]) == (rb["rel_before"][b], rb["rel_after"][b])
        acc += r1["accepted"]
        g1.close()
    assert rb["accepted"] == acc
    v3 = gb.empty()
    info = gb.poisson_solve(rho_b, v3, rtol=1e-10, guess=3, atoms=batch, guess_net=net)
    assert info["guess_accepted"] == acc and bool(info["fallback_used"] & 1) == (acc < 3)
    assert max(info["batch_rel_resid"]) <= 1e-10
    v_b2 = v_b.clone()
    gb.poisson_solve(rho_b, v_b2, rtol=1e-10)
    assert float((v3 - v_b2).abs().max()) <= 1e-8 * float(v_b2.abs().max())
    gb.close()
    net.close()


def test_learned_guess_lowers_the_residual_of_the_analytic_guess(torch, L):
    """Trained on config-4 problems (random clusters, 65^3 graded), the net's
    correction lowers the smoothed residual of the analytic guess on held-out
    problems, and the solve from it needs fewer cycles than the solve from the
    faces alone. (Against the analytic guess itself its cycle count is within
    one either way: with the exact coarsest solve, 36 against 35 cycles over
    these three problems; with the red-black tail it was no more.)"""
    from paper_0806_1723_amd import learned
    n = 65
    say("learned guess, config 4 at %d^3" % n)
    train_p = [learned.make_problem(4, s, n) for s in range(10)]
    test_p = [learned.make_problem(4, 1000 + s, n) for s in range(3)]
    net = L.Net((n, n, n), ch=(16, 32, 32, 32), seed=7, **learned.NET_SCALES)
    hist = learned.train(net, train_p, steps=800, lr=2e-3)
    say("  training loss %.3e -> %.3e" % (np.mean(hist[:10]), np.mean(hist[-10:])))
    # the last 10 steps revisit the first 10 steps' problems
    assert np.mean(hist[-10:]) < 0.6 * np.mean(hist[:10])
    better, iters = 0, []
    for p in test_p:
        r = learned.compare(net, p, rtol=1e-10, method=1)
        say("  %s: %s" % (p.name, r))
        better += r["learned"]["rel_learned"] < r["learned"]["rel_plain"]
        iters.append((r["zero"]["iters"], r["analytic"]["iters"], r["learned"]["iters"]))
        assert r["learned"]["rel_resid"] <= 1e-10
        # the learned guess borrowed the solver's vectors: the same solve again gives the same bits
        v1, v2 = p.v_star.clone(), p.v_guess.clone()
        p.grid.poisson_solve(p.rho, v2, rtol=1e-10, bc=2)
        assert torch.equal(v1, v2)
    assert better >= 2
    say("  cycles (zero, analytic, learned): %s" % iters)
    assert all(i[2] < i[0] for i in iters)
    assert sum(i[2] for i in iters) <= sum(i[1] for i in iters) + len(iters)
    net.close()


def test_learned_correction_saves_cycles(torch, L):
    """The learned coarse correction: a net trained on the solver's own
    iterates (residual -> error, config-4 clusters at 65^3) applied before
    each stationary V-cycle cuts the cycles to 1e-10 on held-out clusters by
    more than the extra red-black sweep of its judge could."""
    from paper_0806_1723_amd import learned
    n = 65
    say("learned correction, config 4 at %d^3" % n)
    train_p = [learned.make_problem(4, s, n) for s in range(12)]
    test_p = [learned.make_problem(4, 1000 + s, n) for s in range(2)]
    net = L.Net((n, n, n), ch=(16, 32, 32, 32), seed=9, **learned.CORRECTION_SCALES)
    pairs = [pp for p in train_p for pp in learned.correction_pairs(net, p, (1, 2, 3))]
    hist = learned.train_pairs(net, pairs, steps=1200, lr=2e-3)
    say("  training loss %.3e -> %.3e" % (np.mean(hist[:36]), np.mean(hist[-36:])))
    assert np.mean(hist[-36:]) < 0.1 * np.mean(hist[:36])
    for p in test_p:
        plain = learned.corrected_cycles(p, None)
        corr = learned.corrected_cycles(p, net)
        say("  %s: plain %s, learned %s" % (p.name, plain, corr))
        assert plain["rel_resid"] <= 1e-10 and corr["rel_resid"] <= 1e-10
        assert corr["cycles"] <= plain["cycles"] - 2
        assert corr["accepted"] >= corr["cycles"] // 2
    net.close()


def test_learned_guess_on_a_coarse_level(torch, L):
    """A learned-guess net on a coarse level of the hierarchy: its features
    are taken at that level's nodes and its output is interpolated linearly to
    the finest level. A net whose output is a constant c (all weights zero,
    head bias c) must propose the finest-level start v + out_scale c at every
    interior node; its judged residual matches that candidate's, swept once,
    computed here from lasto_rb_sweep and lasto_apply. A net trained on that
    level then helps the solve from its start reach the tolerance."""
    from paper_0806_1723_amd import learned
    n, lev = 65, 2
    say("learned guess on coarse level %d, config 4 at %d^3" % (lev, n))
    p = learned.make_problem(4, 7, n)
    g = p.grid
    nx, ny, nz = g.levels()[lev]
    net = L.Net((nz, ny, nx), ch=(16, 16, 16, 16), seed=5, **learned.NET_SCALES)
    prm = np.zeros(net.nparam, dtype=np.float32)
    prm[-1] = 0.7
    net.set_params(prm)
    v = p.v_guess.clone()
    r = g.learned_guess(net, p.rho, v)
    shift = learned.NET_SCALES["out_scale"] * float(np.float32(0.7))   # the net's output is FP32
    shifted = p.v_guess.clone()
    shifted[1:-1, 1:-1, 1:-1] += shift
    cand = g.rb_sweep(shifted, p.rho)
    plain = g.rb_sweep(p.v_guess, p.rho)
    m = []
    for c in g.coords:
        mm = np.zeros_like(c)
        mm[1:-1] = 0.5 * (c[2:] - c[:-2])
        m.append(mm)
    vol = np.einsum("k,j,i->kji", m[2], m[1], m[0])
    b = 4 * np.pi * p.rho.cpu().numpy()
    vbc = p.v_guess.clone()
    vbc[1:-1, 1:-1, 1:-1] = 0.0

    def wres(u):
        rr = (b - g.apply(u).cpu().numpy())[1:-1, 1:-1, 1:-1]
        return float(np.sqrt((vol[1:-1, 1:-1, 1:-1] * rr * rr).sum()))

    r0 = wres(vbc)
    rc, rp = wres(cand) / r0, wres(plain) / r0
    say("  constant net: judged plain %.6e learned %.6e; host %.6e %.6e" % (r["rel_before"], r["rel_after"], rp, rc))
    assert abs(r["rel_after"] - rc) <= 1e-9 * rc and abs(r["rel_before"] - rp) <= 1e-9 * rp
    assert r["accepted"] == (rc < rp)
    # (the interpolation weights of a constant sum to one up to rounding)
    want = cand if r["accepted"] else plain
    assert float((v - want).abs().max()) <= 1e-13 * float(want.abs().max())
    # trained on the coarse level: the solve from its start reaches the tolerance
    train_p = [learned.make_problem(4, s, n) for s in range(8)]
    # (the first coarse level: at 65^3 about 43^3 nodes, the resolution the
    # 129^3 benchmark's guess net has on its second)
    net2 = L.Net((48, 48, 48), ch=(16, 32, 32, 32), seed=7, **learned.NET_SCALES)
    hist = learned.train(net2, train_p, steps=1500, lr=2e-3, level=1)
    say("  coarse-level training loss %.3e -> %.3e" % (np.mean(hist[:8]), np.mean(hist[-8:])))
    assert np.mean(hist[-8:]) < 0.8 * np.mean(hist[:8])
    res = learned.compare(net2, p, rtol=1e-10, level=1)
    say("  %s" % res)
    assert res["learned"]["rel_resid"] <= 1e-10 and res["err_vs_label"] <= 1e-8
    for q in train_p:
        q.grid.close()
    g.close()
    net.close()
    net2.close()


def test_learned_coarse_correction_inside_the_cycle(torch, L):
    """The learned coarse correction (config-4 clusters at 65^3, the net on
    the first coarse level, the exact coarsest solve one level below): it is
    proposed at every visit of its level, kept only where it lowers that
    level's residual, and the flexible CG, the mixed form and the stationary
    cycles reach the same solution (the label) with it. A net whose proposals
    are far off is always refused, and the solve then takes the plain cycle's
    course."""
    from paper_0806_1723_amd import learned
    n, level = 65, 1
    say("learned coarse correction, config 4 at %d^3, level %d" % (n, level))
    train_p = [learned.make_problem(4, s, n) for s in range(8)]
    test_p = [learned.make_problem(4, 1000 + s, n) for s in range(2)]
    cap = max(max(p.grid.levels()[level]) for p in train_p + test_p)
    net = L.Net((cap, cap, cap), ch=(16, 32, 32, 32), seed=13, **learned.COARSE_SCALES)
    pairs = [pp for p in train_p for pp in learned.coarse_pairs(net, p, level)]
    hist = learned.train_coarse(net, pairs, steps=800, lr=2e-3)
    k = len(pairs)
    say("  %d pairs, training loss %.3e -> %.3e" % (k, np.mean(hist[:k]), np.mean(hist[-k:])))
    assert np.mean(hist[-k:]) < 0.5 * np.mean(hist[:k])
    for p in test_p:
        for opts in (dict(), dict(precision=1), dict(method=1)):
            r = learned.compare_coarse(net, p, level, **opts)
            say("  %s %s: %s" % (p.name[:24], opts, r))
            for kind in ("plain", "learned"):
                assert r[kind]["rel_resid"] <= 1e-10 and r[kind]["err_vs_label"] <= 1e-8
            assert r["plain"]["applied"] == 0
            assert r["learned"]["applied"] >= r["learned"]["vcycles"] and r["learned"]["accepted"] >= 1
            assert r["learned"]["accepted"] <= r["learned"]["applied"]
    # far-off proposals are refused every time: the plain cycle's course
    bad = L.Net((cap, cap, cap), ch=(16, 16, 16, 16), seed=2, rho_scale=1.0, pot_scale=0.01, h_ref=1.0,
                out_scale=1e6)
    p = test_p[0]
    r = learned.compare_coarse(bad, p, level)
    say("  refused net: %s" % r)
    assert r["learned"]["accepted"] == 0 and r["learned"]["applied"] >= r["learned"]["vcycles"]
    assert abs(r["learned"]["iters"] - r["plain"]["iters"]) <= 1 and r["learned"]["rel_resid"] <= 1e-10
    # the level must lie above the exact coarsest solve
    with pytest.raises(L.LastoError):
        p.grid.poisson_solve(p.rho, p.v_guess.clone(), bc=2, coarse_net=net, coarse_net_level=level)
    for q in train_p + test_p:
        q.grid.close()
    net.close()
    bad.close()


def test_net_features_match_their_definition(torch, L, R):
    """lasto_net_features: channel 0 rho * rho_scale, 1..3 log(m_d / h_ref)
    of the dual widths, 4 v * pot_scale, 5 the face flag, 6 and 7 zero, each
    rounded to BF16 (the width channels within one BF16 step, or 1e-6 where
    the logarithm is near zero: the kernel takes them in FP32)."""
    rng = np.random.default_rng(21)
    xs = [np.concatenate([[0.0], np.cumsum(rng.uniform(0.1, 0.9, n - 1))]) for n in (23, 17, 19)]
    g = L.Grid(*xs)
    shape = (19, 17, 23)
    net = L.Net(shape, ch=(16, 16, 16, 16), seed=5, rho_scale=0.3, pot_scale=0.02, h_ref=0.25)
    rho_h = rng.normal(size=shape) * 4.0
    v_h = rng.normal(size=shape) * 50.0
    rho = torch.from_numpy(rho_h).to("cuda")
    v = torch.from_numpy(v_h).to("cuda")
    got = R.bf16_bits_to_float(net.features(g, rho, v).cpu().numpy())
    m = []
    for x in xs:
        d = np.zeros_like(x)
        d[1:-1] = 0.5 * (x[2:] - x[:-2])
        d[0] = 0.5 * (x[1] - x[0])
        d[-1] = 0.5 * (x[-1] - x[-2])
        m.append(d)
    Z, Y, X = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), np.arange(shape[2]), indexing="ij")
    face = (X == 0) | (Y == 0) | (Z == 0) | (X == shape[2] - 1) | (Y == shape[1] - 1) | (Z == shape[0] - 1)
    want = np.zeros(shape + (8,))
    want[..., 0] = rho_h * 0.3
    want[..., 1] = np.log(m[0][X] / 0.25)
    want[..., 2] = np.log(m[1][Y] / 0.25)
    want[..., 3] = np.log(m[2][Z] / 0.25)
    want[..., 4] = v_h * 0.02
    want[..., 5] = face.astype(float)
    exact = R.round_bf16(want)
    for c in (0, 4, 5, 6, 7):
        assert np.array_equal(got[..., c], exact[..., c]), c
    for c in (1, 2, 3):
        # one BF16 step, or the FP32 rounding of m / h_ref where the log is near 0
        step = np.abs(exact[..., c]) * 2.0 ** -7 + 1e-6
        assert (np.abs(got[..., c] - exact[..., c]) <= step).all(), c
    g.close()
