"""Every BF16 matrix-core kernel of the learned net, one at a time, against
the CPU reference (oracle/net_ref.py, float64) on exactly the operands the
kernel read (the GPU's own stored BF16 tensors, lasto_net_tensor).

Bound per output element: the kernels accumulate n exact BF16 x BF16
products in FP32, so |acc - exact| <= gamma_n sum |a||b| with gamma_n =
n u / (1 - n u), u = 2^-24; an output stored in BF16 adds at most
u_bf16 = 2^-8 of its magnitude (nearest-even rounding of 8 significant bits).
n is the terms summed: 27 cin (+1 for the bias) for a convolution, 27 cout
for its adjoint, the nodes for a weight gradient."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
UBF = 2.0 ** -8


def say(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def gamma(n):
    return n * U32 / (1.0 - n * U32)


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


def check(name, got, exact, absdot, n, bf16_out, extra=None):
    """|got - exact| <= gamma_n absdot (+ the BF16 rounding of the output)."""
    got = np.asarray(got, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    acc = gamma(n) * np.asarray(absdot, dtype=np.float64)
    bound = acc * (1.0 + UBF) + UBF * np.abs(exact) if bf16_out else acc
    if extra is not None:
        bound = bound + extra
    bound = bound + 1e-30
    err = np.abs(got - exact)
    worst = float((err / bound).max())
    say("  %-28s max |err| %.3e of max %.3e; worst err/bound %.3f" % (name, err.max(), np.abs(exact).max(), worst))
    assert worst <= 1.0, name
    return worst


CASES = [((20, 27, 37), (16, 32, 48, 64)),
         # levels of 0.83 M and 0.11 M nodes: the stride-1 convolutions' LDS-staged form
         ((93, 94, 95), (16, 32, 16, 16))]


@pytest.mark.parametrize("shape,ch", CASES)
def test_each_net_kernel_within_its_rounding_bound(torch, L, R, shape, ch):
    say("net kernels one by one %s ch %s" % (shape, ch))
    import torch.nn.functional as F
    rng = np.random.default_rng(31)
    net = L.Net(shape, ch=ch, seed=5)
    # random biases and head so that every term of the epilogues is exercised
    p = net.params().astype(np.float64)
    o = 0
    for ci, co, _ in R.layer_specs(ch):
        o += 27 * ci * co
        p[o:o + co] = rng.normal(scale=0.05, size=co)
        o += co
    p[o:o + ch[0]] = rng.normal(scale=0.3, size=ch[0])
    p[o + ch[0]] = 0.1
    net.set_params(p.astype(np.float32))
    p = net.params().astype(np.float64)
    layers, hw, hb = R.unflatten(p, ch)
    Wb = [torch.as_tensor(R.round_bf16(W.numpy())) for W, _ in layers]   # the packed BF16 weights
    bs = [b for _, b in layers]
    specs = R.layer_specs(ch)
    a = torch.from_numpy(rng.normal(size=shape + (8,)).astype(np.float32)).to(torch.bfloat16)
    x_bits = a.view(torch.int16).contiguous().to("cuda")
    x = torch.as_tensor(a.to(torch.float64).numpy()).permute(3, 0, 1, 2).contiguous()
    y = net.forward(x_bits).cpu().numpy().astype(np.float64)

    def T(name):
        bits = net.tensor(name).cpu().numpy()
        return torch.as_tensor(R.bf16_bits_to_float(bits)).permute(3, 0, 1, 2).contiguous()

    # ---- forward: each convolution from its stored input
    ins = {0: x, 1: T("e0"), 2: T("e1"), 3: T("e2"), 4: T("e3"), 5: T("m3"), 6: T("u2"), 7: T("u1")}
    outs = {0: "e0", 1: "e1", 2: "e2", 3: "e3", 4: "m3", 5: "d2", 6: "d1", 7: "d0"}
    for i in range(8):
        ci, co, stride = specs[i]
        pre = R.conv_pre(ins[i], Wb[i], bs[i], stride)
        absd = R.conv_pre(ins[i].abs(), Wb[i].abs(), bs[i].abs(), stride)
        check("conv %d (stride %d) %d->%d" % (i, stride, ci, co), T(outs[i]).numpy(), F.relu(pre).numpy(),
              absd.numpy(), 27 * ci + 1, True)
    # ---- up-sampling plus skip: u_l = up(d_l) + e_l (weights 1 and 1/2, exact)
    for l, (dn, en, un) in enumerate((("d0", "e0", "u0"), ("d1", "e1", "u1"), ("d2", "e2", "u2"))):
        d, e = T(dn), T(en)
        up = R.upsample(d, tuple(e.shape[1:]))
        absd = R.upsample(d.abs(), tuple(e.shape[1:])) + e.abs()
        check("upsample + skip, level %d" % l, T(un).numpy(), (up + e).numpy(), absd.numpy(), 9, True)
    # ---- head (FP32 weights and output)
    u0 = T("u0")
    check("head", y, R.head(u0, hw, float(hb)).numpy(),
          R.head(u0.abs(), hw.abs(), abs(float(hb))).numpy(), ch[0] + 1, False)

    # ---- backward
    t = (np.tanh(x[0].numpy()) * 0.5).astype(np.float32)
    wt = (rng.uniform(0.5, 1.5, size=shape) / np.prod(shape)).astype(np.float32)
    net.backward(x_bits, torch.from_numpy(t).cuda(), torch.from_numpy(wt).cuda())
    g = net.grads().astype(np.float64)
    # head: du0 = bf16(w (2 wt (y - t))) with four FP32 roundings before the BF16 one
    dy = 2.0 * wt.astype(np.float64) * (y - t.astype(np.float64))
    du0 = torch.einsum("c,zyx->czyx", hw, torch.as_tensor(dy))
    check("head backward", T("du0").numpy(), du0.numpy(), 0.0 * du0.numpy(), 1, True,
          extra=4 * U32 * (1 + UBF) * np.abs(du0.numpy()))
    # up-sampling adjoints, masked by the ReLU of the up-sampled d_l
    for l, (dun, dn, gn) in enumerate((("du0", "d0", "g7"), ("du1", "d1", "g6"), ("du2", "d2", "g5"))):
        fine, d = T(dun), T(dn)
        adj = R.upsample_adjoint(fine, tuple(d.shape[1:]))
        absd = R.upsample_adjoint(fine.abs(), tuple(d.shape[1:]))
        mask = (d > 0).to(torch.float64)
        check("upsample adjoint, level %d" % l, T(gn).numpy(), (adj * mask).numpy(), (absd * mask).numpy(), 27, True)
    # data adjoints of the convolutions: du_{l} from layers 7, 6; then the
    # masked, skip-added gradients of e3, e2, e1, e0 and m3
    def adjoint(i, gout, in_shape):
        stride = specs[i][2]
        return (R.conv_adjoint(gout, Wb[i], stride, in_shape), R.conv_adjoint(gout.abs(), Wb[i].abs(), stride, in_shape))

    for i, gn, outn, addn, maskn in ((7, "g7", "du1", None, None), (6, "g6", "du2", None, None),
                                     (5, "g5", "g4", None, "m3"), (4, "g4", "g3", None, "e3"),
                                     (3, "g3", "g2", "du2", "e2"), (2, "g2", "g1", "du1", "e1"),
                                     (1, "g1", "g0", "du0", "e0")):
        gout = T(gn)
        in_shape = tuple(ins[i].shape)
        adj, absd = adjoint(i, gout, in_shape)
        if addn is not None:
            add = T(addn)
            adj, absd = adj + add, absd + add.abs()
        if maskn is not None:
            m = (T(maskn) > 0).to(torch.float64)
            adj, absd = adj * m, absd * m
        check("conv %d adjoint -> %s" % (i, outn), T(outn).numpy(), adj.numpy(), absd.numpy(),
              27 * specs[i][1] + 1, True)
    # weight and bias gradients: sums over the output nodes of input x gradient
    o = 0
    gouts = {i: T("g%d" % i) for i in range(8)}
    for i in range(8):
        ci, co, stride = specs[i]
        inp = ins[i]
        W = Wb[i].clone().requires_grad_(True)
        out = F.conv3d(inp[None], W, None, stride=stride, padding=1)
        (gW,) = torch.autograd.grad(out, W, gouts[i][None])
        Wa = Wb[i].abs().clone().requires_grad_(True)
        outa = F.conv3d(inp.abs()[None], Wa, None, stride=stride, padding=1)
        (aW,) = torch.autograd.grad(outa, Wa, gouts[i].abs()[None])
        # (each of 64 node shares summed, then the shares)
        nodes = int(np.prod(gouts[i].shape[1:])) + 64
        got_W = g[o:o + 27 * ci * co].reshape(3, 3, 3, ci, co).transpose(4, 3, 0, 1, 2)
        check("conv %d weight gradient" % i, got_W, gW.numpy(), aW.numpy(), nodes, False)
        o += 27 * ci * co
        gb = gouts[i].sum(dim=(1, 2, 3))
        ab = gouts[i].abs().sum(dim=(1, 2, 3))
        check("conv %d bias gradient" % i, g[o:o + co], gb.numpy(), ab.numpy(), nodes, False)
        o += co
    # head gradients: sum over nodes of u0 dy (dy with its own FP32 roundings) and of dy
    dyt = torch.as_tensor(dy)
    gw = torch.einsum("czyx,zyx->c", u0, dyt)
    aw = torch.einsum("czyx,zyx->c", u0.abs(), dyt.abs())
    # (per-thread sums, 256 threads per share, 64 shares; dy's own three roundings)
    nodes = int(np.prod(shape)) + 256 + 64 + 4
    check("head weight gradient", g[o:o + ch[0]], gw.numpy(), aw.numpy(), nodes, False)
    check("head bias gradient", g[o + ch[0]], float(dyt.sum()), float(dyt.abs().sum()), nodes, False)
    net.close()
