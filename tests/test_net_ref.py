"""Pins of the CPU reference of the learned-guess network (oracle/net_ref.py):
finite differences of its loss, its up-sampling, and its level sizes. The
network itself has no counterpart in the paper: parity unpinned for its
weights and outputs, which is why only the reference's arithmetic is pinned."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import net_ref as R

CH = (16, 16, 16, 16)


def _random_problem(rng, shape=(9, 8, 11)):
    nz, ny, nx = shape
    x = rng.normal(size=(nz, ny, nx, 8))
    p = rng.normal(scale=0.2, size=R.param_count(CH))
    t = rng.normal(size=shape)
    w = rng.uniform(0.5, 1.5, size=shape)
    return x, p, t, w


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    x, p, t, w = _random_problem(rng)
    L, g = R.loss_and_grads(x, p, CH, t, w, bf16=False)
    idx = rng.choice(len(p), size=40, replace=False)
    for k in idx:
        e = 1e-6 * max(1.0, abs(p[k]))
        pp, pm = p.copy(), p.copy()
        pp[k] += e
        pm[k] -= e
        fp = float((w * (R.forward(x, pp, CH, bf16=False).numpy() - t) ** 2).sum())
        fm = float((w * (R.forward(x, pm, CH, bf16=False).numpy() - t) ** 2).sum())
        fd = (fp - fm) / (2 * e)
        assert abs(fd - g[k]) <= 1e-5 * max(1.0, abs(g[k])) + 1e-7 * abs(L), (k, fd, g[k])


def test_upsampling_reproduces_linear_functions_and_levels():
    # index-space linear interpolation is exact on functions linear in the index
    for nc, n in ((5, 9), (5, 10), (3, 5)):
        M = R.up_matrix(nc, n).numpy()
        c = 2.0 * np.arange(nc) + 1.0
        f = M @ c
        lim = n if n == 2 * nc - 1 else n - 1      # past the last coarse node the value is held
        assert np.allclose(f[:lim], np.arange(n)[:lim] + 1.0)
        assert np.allclose(M.sum(axis=1), 1.0)
    # stride-2 levels have (n + 1) // 2 nodes
    x = np.zeros((9, 8, 11, 8))
    p = np.zeros(R.param_count(CH))
    _, inter = R.forward(x, p, CH, bf16=False, keep=True)
    assert inter["e1"].shape[2:] == (5, 4, 6)
    assert inter["e3"].shape[2:] == (2, 1, 2)


def test_bf16_rounding_is_nearest_even():
    # 1 + 2^-8 lies halfway between two BF16 neighbours (1 and 1 + 2^-7): ties go to even (1)
    a = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -9)])
    assert list(R.round_bf16(a)) == [1.0, 1.0 + 2.0 ** -6, -1.0]
    bits = np.array([0x3F80, 0xBF80, 0x4000], dtype=np.int64).astype(np.int16)
    assert list(R.bf16_bits_to_float(bits)) == [1.0, -1.0, 2.0]


def test_stage_helpers_are_the_forward_pass_and_its_adjoints():
    """The one-stage helpers the kernel tests use: conv_pre with a ReLU, the
    up-sampling plus skip and the head rebuild the whole forward pass; each
    adjoint satisfies <A x, g> = <x, A^T g> (stride 1 and 2, odd and even
    sizes); a direct triple loop pins one output of conv_pre."""
    rng = np.random.default_rng(9)
    x, p, _, _ = _random_problem(rng)
    y, inter = R.forward(x, p, CH, bf16=False, keep=True)
    layers, hw, hb = R.unflatten(p, CH)
    specs = R.layer_specs(CH)
    a = torch.as_tensor(x).permute(3, 0, 1, 2)
    e0 = torch.relu(R.conv_pre(a, layers[0][0], layers[0][1], 1))
    assert torch.allclose(e0, inter["e0"][0], rtol=0, atol=1e-12)
    e1 = torch.relu(R.conv_pre(e0, layers[1][0], layers[1][1], 2))
    assert torch.allclose(e1, inter["e1"][0], rtol=0, atol=1e-12)
    u0 = R.upsample(inter["d0"][0], tuple(e0.shape[1:])) + inter["e0"][0]
    assert torch.allclose(u0, inter["u0"][0], rtol=0, atol=1e-12)
    assert torch.allclose(R.head(u0, hw, float(hb)), y, rtol=0, atol=1e-12)
    # one output node of conv_pre by the definition
    W, b = layers[1]
    out = R.conv_pre(e0, W, b, 2)
    co, z, yy, xx = 3, 2, 1, 3
    s = float(b[co])
    for ci in range(e0.shape[0]):
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    iz, iy, ix = 2 * z + dz - 1, 2 * yy + dy - 1, 2 * xx + dx - 1
                    if 0 <= iz < e0.shape[1] and 0 <= iy < e0.shape[2] and 0 <= ix < e0.shape[3]:
                        s += float(W[co, ci, dz, dy, dx]) * float(e0[ci, iz, iy, ix])
    assert abs(float(out[co, z, yy, xx]) - s) <= 1e-12 * max(1.0, abs(s))
    # adjoints by the inner-product identity
    for shape, stride in (((16, 9, 8, 11), 1), ((16, 9, 8, 11), 2), ((16, 10, 7, 6), 2)):
        xin = torch.as_tensor(rng.normal(size=shape))
        Wt = torch.as_tensor(rng.normal(size=(12, 16, 3, 3, 3)))
        Ax = R.conv_pre(xin, Wt, None, stride)
        gout = torch.as_tensor(rng.normal(size=tuple(Ax.shape)))
        lhs = float((Ax * gout).sum())
        rhs = float((xin * R.conv_adjoint(gout, Wt, stride, shape)).sum())
        assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    c = torch.as_tensor(rng.normal(size=(4, 3, 4, 5)))
    fine = torch.as_tensor(rng.normal(size=(4, 5, 7, 10)))
    lhs = float((R.upsample(c, (5, 7, 10)) * fine).sum())
    rhs = float((c * R.upsample_adjoint(fine, (3, 4, 5))).sum())
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
