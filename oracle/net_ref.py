"""CPU reference of the learned-guess U-Net -- TEST INFRASTRUCTURE ONLY.

Plain PyTorch CPU ops in float64 (a 3-D convolution as the library step),
written from the network's definition, not from the GPU code: it shares no
code with paper_0806_1723_amd/csrc. It serves the GPU parity tests of the
network kernels (forward values and parameter gradients on identical BF16
operands) and is itself pinned by finite differences.

The network (the learned form has no counterpart in the paper; it is the
learned initial guess grown beside the multigrid solver):
    e0 = relu(conv(x))              x: 8 features per node
    e1 = relu(conv_s2(e0)); e2 = relu(conv_s2(e1)); e3 = relu(conv_s2(e2))
    m3 = relu(conv(e3))
    d2 = relu(conv(m3)); u2 = up(d2) + e2
    d1 = relu(conv(u2)); u1 = up(d1) + e1
    d0 = relu(conv(u1)); u0 = up(d0) + e0
    y  = w . u0 + b
conv: 3x3x3, zero padding; conv_s2: the same sampled at every other node (a
level of an n-node axis has (n + 1) // 2 nodes); up: linear in index space
(even fine node i takes coarse i / 2, odd the mean of (i - 1) / 2 and
(i + 1) / 2, the last coarse node standing in past the end).

Parameter vector (FP32 on the GPU): per convolution W[27][cin][cout] (tap
t = 9 (dz+1) + 3 (dy+1) + (dx+1)) then b[cout], in forward order, then the
head w[c0] and b.

bf16=True rounds what the GPU stores in BF16 (weights of the convolutions,
every activation) to nearest-even BF16 in the forward pass; the backward pass
treats that rounding as the identity.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

IN_FEATURES = 8


def layer_specs(ch):
    """(cin, cout, stride) of the eight convolutions."""
    c0, c1, c2, c3 = ch
    return [(IN_FEATURES, c0, 1), (c0, c1, 2), (c1, c2, 2), (c2, c3, 2),
            (c3, c3, 1), (c3, c2, 1), (c2, c1, 1), (c1, c0, 1)]


def param_count(ch):
    n = sum(27 * ci * co + co for ci, co, _ in layer_specs(ch))
    return n + ch[0] + 1


def unflatten(p, ch):
    """Flat parameter vector -> list of (W [co, ci, 3, 3, 3] torch layout, b), head w, head b."""
    p = torch.as_tensor(np.asarray(p, dtype=np.float64))
    out, o = [], 0
    for ci, co, _ in layer_specs(ch):
        W = p[o:o + 27 * ci * co].reshape(3, 3, 3, ci, co)      # [dz][dy][dx][ci][co]
        o += 27 * ci * co
        b = p[o:o + co]
        o += co
        out.append((W.permute(4, 3, 0, 1, 2).contiguous(), b))  # [co][ci][kz][ky][kx]
    hw = p[o:o + ch[0]]
    hb = p[o + ch[0]]
    return out, hw, hb


def flatten_grads(layer_grads, hw_grad, hb_grad):
    parts = []
    for gW, gb in layer_grads:
        parts.append(gW.permute(2, 3, 4, 1, 0).reshape(-1))    # back to [dz][dy][dx][ci][co]
        parts.append(gb.reshape(-1))
    parts.append(hw_grad.reshape(-1))
    parts.append(hb_grad.reshape(-1))
    return torch.cat(parts).numpy()


class _RoundBF16(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a):
        return a.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


def _r(a, on):
    return _RoundBF16.apply(a) if on else a


def up_matrix(nc, n):
    """[n, nc] linear up-sampling in index space."""
    M = np.zeros((n, nc))
    for i in range(n):
        a = i // 2
        if i % 2:
            b = min(a + 1, nc - 1)
            M[i, a] += 0.5
            M[i, b] += 0.5
        else:
            M[i, a] = 1.0
    return torch.as_tensor(M)


def upsample(a, shape):
    """a: [C, cz, cy, cx] -> [C, nz, ny, nx]: the tensor product of the three
    axes' up-sampling matrices, applied one axis at a time."""
    nz, ny, nx = shape
    _, cz, cy, cx = a.shape
    Mz, My, Mx = up_matrix(cz, nz), up_matrix(cy, ny), up_matrix(cx, nx)
    t = torch.einsum("Xx,czyx->czyX", Mx, a)
    t = torch.einsum("Yy,czyX->czYX", My, t)
    return torch.einsum("Zz,czYX->cZYX", Mz, t)


def forward(x, p, ch, bf16=True, keep=False):
    """x: [nz, ny, nx, 8] float64 (the BF16 features' values); p: flat
    parameters. Returns y [nz, ny, nx] (and the intermediates when keep)."""
    layers, hw, hb = unflatten(p, ch)
    a = torch.as_tensor(x).permute(3, 0, 1, 2)[None]          # [1, 8, nz, ny, nx]

    def conv(i, inp):
        W, b = layers[i]
        stride = layer_specs(ch)[i][2]
        out = F.conv3d(inp, _r(W, bf16), b, stride=stride, padding=1)
        return _r(F.relu(out), bf16)

    e0 = conv(0, a)
    e1 = conv(1, e0)
    e2 = conv(2, e1)
    e3 = conv(3, e2)
    m3 = conv(4, e3)
    d2 = conv(5, m3)
    u2 = _r(upsample(d2[0], e2.shape[2:])[None] + e2, bf16)
    d1 = conv(6, u2)
    u1 = _r(upsample(d1[0], e1.shape[2:])[None] + e1, bf16)
    d0 = conv(7, u1)
    u0 = _r(upsample(d0[0], e0.shape[2:])[None] + e0, bf16)
    y = torch.einsum("c,czyx->zyx", hw, u0[0]) + hb
    if keep:
        return y, dict(e0=e0, e1=e1, e2=e2, e3=e3, m3=m3, d2=d2, u2=u2, d1=d1, u1=u1, d0=d0, u0=u0)
    return y


def loss_and_grads(x, p, ch, target, weight, bf16=True):
    """L = sum weight (y - target)^2 and dL/dp (flat, float64)."""
    layers, hw, hb = unflatten(p, ch)
    leaves = []
    for W, b in layers:
        W.requires_grad_(True)
        b.requires_grad_(True)
        leaves += [W, b]
    hw.requires_grad_(True)
    hb = hb.clone().requires_grad_(True)
    a = torch.as_tensor(x).permute(3, 0, 1, 2)[None]

    def conv(i, inp):
        W, b = layers[i]
        stride = layer_specs(ch)[i][2]
        return _r(F.relu(F.conv3d(inp, _r(W, bf16), b, stride=stride, padding=1)), bf16)

    e0 = conv(0, a)
    e1 = conv(1, e0)
    e2 = conv(2, e1)
    e3 = conv(3, e2)
    m3 = conv(4, e3)
    d2 = conv(5, m3)
    u2 = _r(upsample(d2[0], e2.shape[2:])[None] + e2, bf16)
    d1 = conv(6, u2)
    u1 = _r(upsample(d1[0], e1.shape[2:])[None] + e1, bf16)
    d0 = conv(7, u1)
    u0 = _r(upsample(d0[0], e0.shape[2:])[None] + e0, bf16)
    y = torch.einsum("c,czyx->zyx", hw, u0[0]) + hb
    t = torch.as_tensor(np.asarray(target, dtype=np.float64))
    w = torch.as_tensor(np.asarray(weight, dtype=np.float64))
    L = (w * (y - t) ** 2).sum()
    L.backward()
    lg = [(W.grad, b.grad) for W, b in layers]
    return L.item(), flatten_grads(lg, hw.grad, hb.grad)


def bf16_bits_to_float(bits):
    """int16 BF16 bit patterns -> float64 values."""
    u = np.asarray(bits).astype(np.int64) & 0xFFFF
    return (u << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def round_bf16(a):
    """Nearest-even BF16 values of a (float64 array)."""
    return torch.as_tensor(np.asarray(a, dtype=np.float64)).to(torch.float32).to(torch.bfloat16).to(
        torch.float64).numpy()


# ------------------------------------------------- one stage at a time
# Each stage of the network on given operands (the values the GPU stored), in
# float64, so that every kernel is checked on exactly the inputs it read.
def conv_pre(inp, W, b, stride):
    """One convolution before its ReLU: inp [C, nz, ny, nx], W [co, ci, 3, 3,
    3], b [co] (or None) -> [co, ...]; stride 1 or 2, zero padding 1."""
    out = F.conv3d(torch.as_tensor(inp)[None], torch.as_tensor(W), None if b is None else torch.as_tensor(b),
                   stride=stride, padding=1)
    return out[0]


def conv_adjoint(gout, W, stride, in_shape):
    """The adjoint of conv_pre (no bias) with respect to its input: the
    vector-Jacobian product of the convolution, by autograd."""
    x = torch.zeros((1,) + tuple(in_shape), dtype=torch.float64, requires_grad=True)
    out = F.conv3d(x, torch.as_tensor(W), None, stride=stride, padding=1)
    (g,) = torch.autograd.grad(out, x, torch.as_tensor(gout)[None])
    return g[0]


def upsample_adjoint(fine, coarse_shape):
    """The adjoint of upsample: [C, nz, ny, nx] -> [C, cz, cy, cx]."""
    c = torch.zeros((fine.shape[0],) + tuple(coarse_shape), dtype=torch.float64, requires_grad=True)
    out = upsample(c, tuple(fine.shape[1:]))
    (g,) = torch.autograd.grad(out, c, torch.as_tensor(fine))
    return g


def head(u0, hw, hb):
    """y = w . u0 + b per node: u0 [c0, nz, ny, nx]."""
    return torch.einsum("c,czyx->zyx", torch.as_tensor(hw), torch.as_tensor(u0)) + hb
