"""Training and use of the learned initial guess (orchestration only: every
step runs in the library's kernels through the C ABI; torch holds buffers).

The paper's solver has no learned part. This is the learned form grown beside
it: a U-Net (lasto_net_*) maps features of a source and its analytic
monopole guess (lasto_analytic_guess, with the multipole faces of
lasto_boundary_values) to a correction of that guess. Its training labels
are the method's own FP64 multigrid solutions of the same problems
(config 4: random 13..55-atom clusters on graded meshes), and plain
multigrid judges every learned guess (lasto_learned_guess).
"""
from __future__ import annotations

import dataclasses
import time
from typing import List

import numpy as np

from . import inputs as I
from . import lasto

# feature and output scales of the net (fixed, from the statistics of the
# config-4 problems: densities up to ~15, potentials ~ -100, corrections ~ 0.1)
NET_SCALES = dict(rho_scale=0.1, pot_scale=0.01, h_ref=0.25, out_scale=0.1)
# the correction net reads the residual at unit RMS and returns the error in
# units of out_scale * RMS (smooth errors are ~ (L / pi)^2 ~ 200 times the residual)
CORRECTION_SCALES = dict(rho_scale=1.0, pot_scale=0.01, h_ref=0.25, out_scale=100.0)


@dataclasses.dataclass
class Problem:
    name: str
    atoms: list
    grid: "lasto.Grid"
    rho: object          # device float64 [nz, ny, nx]
    v_guess: object      # faces + analytic guess inside
    v_star: object       # FP64 multigrid solution to 1e-10 (the label)
    solve_info: dict


def make_problem(cid: int, sample: int, n: int, rtol: float = 1e-10) -> Problem:
    """One seeded problem: grid, pseudo-density, faces, analytic guess, label."""
    w = I.config(cid, n_override=n, sample=sample)
    xs = lasto.mesh_for(w.axes)
    g = lasto.Grid(*xs)
    rho = g.pseudo_density(w.atoms)
    v = g.empty()
    g.boundary_values(rho, v, bc=1)
    g.analytic_guess(w.atoms, v)
    v_star = v.clone()
    info = g.poisson_solve(rho, v_star, rtol=rtol, bc=2)
    return Problem(w.name, w.atoms, g, rho, v, v_star, info)


def use_level(net: "lasto.Net", grid: "lasto.Grid", level: int):
    """Run the net on level `level` of the grid (0: the finest; a coarse level
    for a learned guess whose output is interpolated to the finest)."""
    nx, ny, nz = grid.levels()[level]
    net.set_grid((nz, ny, nx))


def training_pair(net: "lasto.Net", p: Problem, weighting: str = "volume", level: int = 0):
    """Features, target (the correction in units of out_scale) and weights
    over interior nodes (zero on faces): "volume" weighs each node by its
    dual-cell volume (the W-norm of the error, which the far field's smooth
    error dominates), "uniform" weighs nodes alike. A net on a coarse level
    learns the correction at that level's nodes (each a fine node)."""
    import torch
    lev = level
    use_level(net, p.grid, lev)
    x = net.features(p.grid, p.rho, p.v_guess)
    t = ((p.v_star - p.v_guess) / net.cfg.out_scale).to(torch.float32)
    coords = p.grid.coords
    if lev > 0:
        ix, iy, iz = (torch.from_numpy(a.astype(np.int64)).to(t.device) for a in p.grid.level_nodes(lev))
        t = t.index_select(0, iz).index_select(1, iy).index_select(2, ix).contiguous()
        coords = [c[idx.cpu().numpy()] for c, idx in zip(coords, (ix, iy, iz))]
    wt = torch.zeros_like(t)
    if weighting == "volume":
        m = [np.zeros_like(c) for c in coords]
        for c, mm in zip(coords, m):
            mm[1:-1] = 0.5 * (c[2:] - c[:-2])
        vol = np.einsum("k,j,i->kji", m[2], m[1], m[0])
        wt.copy_(torch.from_numpy(vol.astype(np.float32)))
    else:
        wt[1:-1, 1:-1, 1:-1] = 1.0
    wt /= wt.sum()
    t[0, :, :] = 0
    t[-1, :, :] = 0
    t[:, 0, :] = 0
    t[:, -1, :] = 0
    t[:, :, 0] = 0
    t[:, :, -1] = 0
    return x, t.contiguous(), wt.contiguous()


def train(net: "lasto.Net", problems: List[Problem], steps: int, lr: float = 2e-3, log_every: int = 0,
          weighting: str = "volume", level: int = 0, pairs=None):
    """Adam over the problems (or the given pairs) in turn; returns the loss history."""
    if pairs is None:
        pairs = [training_pair(net, p, weighting, level) for p in problems]
    hist = []
    for s in range(steps):
        x, t, wt = pairs[s % len(pairs)]
        net.set_grid(tuple(t.shape))
        a = lr * 0.5 * (1.0 + np.cos(np.pi * s / max(steps, 1)))   # cosine decay
        hist.append(net.train_step(x, t, wt, max(a, lr * 1e-3)))
        if log_every and (s + 1) % log_every == 0:
            print("train step %d loss %.4e" % (s + 1, np.mean(hist[-log_every:])), flush=True)
    return hist


def compare(net: "lasto.Net", p: Problem, rtol: float = 1e-10, level: int = 0, **opts) -> dict:
    """Time-to-tolerance and iterations from the faces alone (zero guess), the
    analytic guess, and the learned guess, same solver and tolerance. Each
    timing covers the faces, the guess and the solve."""
    import torch
    out = {}
    g, rho = p.grid, p.rho

    def timed(kind):
        v = g.empty()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.boundary_values(rho, v, bc=1)
        lg = None
        if kind != "zero":
            g.analytic_guess(p.atoms, v)
        if kind == "learned":
            use_level(net, g, level)
            lg = g.learned_guess(net, rho, v)
        info = g.poisson_solve(rho, v, rtol=rtol, bc=2, **opts)
        torch.cuda.synchronize()
        r = dict(iters=info["iters"], vcycles=info["vcycles"], ms=(time.perf_counter() - t0) * 1e3,
                 rel_resid=info["rel_resid"])
        if lg is not None:
            r.update(accepted=lg["accepted"], rel_plain=lg["rel_before"], rel_learned=lg["rel_after"])
        return r, v

    for kind in ("zero", "analytic", "learned"):
        out[kind], v = timed(kind)
    out["err_vs_label"] = float((v - p.v_star).abs().max() / p.v_star.abs().max())
    return out


def _vol_weights(grid, like):
    import torch
    m = [np.zeros_like(c) for c in grid.coords]
    for c, mm in zip(grid.coords, m):
        mm[1:-1] = 0.5 * (c[2:] - c[:-2])
    vol = np.einsum("k,j,i->kji", m[2], m[1], m[0])
    wt = torch.from_numpy(vol.astype(np.float32)).to(like.device)
    return (wt / wt.sum()).contiguous()


def correction_pairs(net: "lasto.Net", p: Problem, cycles=(1, 2, 3)):
    """Training pairs of the correction net from the solver's own iterates:
    after k stationary V-cycles from the analytic guess, the features of the
    iterate and its error (v* - v_k) in units of out_scale times the residual
    RMS."""
    import torch
    pairs = []
    for k in cycles:
        v = p.v_guess.clone()
        p.grid.poisson_solve(p.rho, v, rtol=1e-14, bc=2, method=1, max_iters=k, allow_fail=True)
        x, s = net.correction_features(p.grid, p.rho, v)
        t = ((p.v_star - v) / (net.cfg.out_scale * s)).to(torch.float32).contiguous()
        pairs.append((x, t, _vol_weights(p.grid, t)))
    return pairs


def train_pairs(net: "lasto.Net", pairs, steps: int, lr: float = 2e-3):
    hist = []
    for s in range(steps):
        x, t, wt = pairs[s % len(pairs)]
        a = lr * 0.5 * (1.0 + np.cos(np.pi * s / max(steps, 1)))
        hist.append(net.train_step(x, t, wt, max(a, lr * 1e-3)))
    return hist


def corrected_cycles(p: Problem, net_c, rtol: float = 1e-10, max_cycles: int = 60) -> dict:
    """Stationary V-cycles from the analytic guess, with (net_c given) or
    without a learned correction before each cycle; cycles to rtol."""
    import torch
    v = p.v_guess.clone()
    acc, rel = 0, 1.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(1, max_cycles + 1):
        if net_c is not None:
            acc += p.grid.learned_correction(net_c, p.rho, v)["accepted"]
        info = p.grid.poisson_solve(p.rho, v, rtol=rtol, bc=2, method=1, max_iters=1, allow_fail=True)
        rel = info["rel_resid"]
        if rel <= rtol:
            break
    torch.cuda.synchronize()
    return dict(cycles=c, accepted=acc, rel_resid=rel, ms=(time.perf_counter() - t0) * 1e3)


# ------------------------------------------- learned coarse correction
# The coarse net reads a coarse level's restricted residual at unit RMS and
# returns the correction in units of out_scale times that RMS (smooth
# corrections are ~ (L / pi)^2 / (4 pi) ~ 20 .. 200 times the residual).
COARSE_SCALES = dict(rho_scale=1.0, pot_scale=0.01, h_ref=1.0, out_scale=100.0)


def coarse_pairs(net: "lasto.Net", p: Problem, level: int, cycles=(0, 1, 2, 3), nu1: int = 2):
    """Training pairs of the coarse net at `level` from the solver's own
    iterates (k stationary V-cycles from the analytic guess): the restricted
    residual the cycle's descent produces there and the exact correction of
    that level (lasto_coarse_pair), with uniform weights over the level's
    interior nodes."""
    import torch
    pairs = []
    for k in cycles:
        v = p.v_guess.clone()
        if k:
            p.grid.poisson_solve(p.rho, v, rtol=1e-14, bc=2, method=1, max_iters=k, allow_fail=True, coarse=2,
                                 nu1=nu1)
        x, t, _, shape = net.coarse_pair(p.grid, p.rho, v, level, nu1)
        wt = torch.zeros_like(t)
        wt[1:-1, 1:-1, 1:-1] = 1.0
        wt /= wt.sum()
        pairs.append((x, t, wt.contiguous(), shape))
    return pairs


def train_coarse(net: "lasto.Net", pairs, steps: int, lr: float = 2e-3):
    """Adam over the pairs in turn, the net's grid set to each pair's level shape."""
    hist = []
    for s in range(steps):
        x, t, wt, shape = pairs[s % len(pairs)]
        net.set_grid(shape)
        a = lr * 0.5 * (1.0 + np.cos(np.pi * s / max(steps, 1)))
        hist.append(net.train_step(x, t, wt, max(a, lr * 1e-3)))
    return hist


def compare_coarse(net_c: "lasto.Net", p: Problem, level: int, rtol: float = 1e-10, **opts) -> dict:
    """The same solve (faces and analytic guess as given, the exact coarsest
    solve one level further down: coarse = 2) without and with the learned
    coarse correction at `level`: iterations, V-cycles, time, proposals kept."""
    import torch
    out = {}
    for kind in ("plain", "learned"):
        for rep in range(2):   # the second pass timed warm
            v = p.v_guess.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            kw = dict(coarse_net=net_c, coarse_net_level=level) if kind == "learned" else {}
            info = p.grid.poisson_solve(p.rho, v, rtol=rtol, bc=2, coarse=2, **kw, **opts)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
        out[kind] = dict(iters=info["iters"], vcycles=info["vcycles"], ms=ms, rel_resid=info["rel_resid"],
                         applied=info["coarse_applied"], accepted=info["coarse_accepted"],
                         err_vs_label=float((v - p.v_star).abs().max() / p.v_star.abs().max()))
    return out
