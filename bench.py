"""Benchmark of the LASTO Hartree step on one MI355X.

One step = the whole hot path on one synthetic input already resident in HBM:
pseudo-density on the 257^3 graded mesh of the 55-atom cluster, moments and
multipole faces, Poisson solve from a zero guess to 1e-10 relative residual
(FP32 V-cycles inside FP64 refinement), and the 64 sphere values per atom.

Prints ONE JSON line. `value` is the time-to-tolerance of the Poisson solve
(ms, lower is better); the plain FP64 solve of the same problem on the same
GPU is reported beside it. `roofline` is the finest-level red-black sweep
(the dominant kernel), timed with HIP events on its own stream inside the
timed steps. `cpu_baseline` is the C oracle timed on the host cores on a
bounded sample (a few V-cycles of the same 257^3 solve), extrapolated with
its measured contraction to the same tolerance.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--n", type=int, default=0, help="override the mesh size of the config")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-cycles", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (the Poisson solve would "
              "shard by z-slabs with halo exchange, see the design notes)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0806_1723_amd import inputs as I
    from paper_0806_1723_amd import lasto

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lasto.load()
    w = I.config(args.config, n_override=args.n or None)
    xs = lasto.mesh_for(w.axes)
    n = len(xs[0])
    mixed = 1 if w.precision == "mixed" else 0
    g = lasto.Grid(*xs)
    log("bench: %s, levels %s" % (w.name, [l[0] for l in g.levels()]))
    rho = g.empty()
    v = g.empty()
    centers = np.array([a.center for a in w.atoms])
    radii = np.array([a.radius for a in w.atoms])

    def step(profile, precision):
        g.pseudo_density(w.atoms, rho_out=rho)
        v.zero_()
        info = g.poisson_solve(rho, v, rtol=w.rtol, precision=precision, profile=profile)
        sph = g.sphere_interp(v, centers, radii)
        return info, sph

    for _ in range(args.warmup):
        step(1, mixed)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, _ = step(1, mixed)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    solve_ms = statistics.median(i["ms_total"] for i in infos)
    launches = sum(i["smooth_launches"] for i in infos)
    sm_ms = sum(i["smooth_ms"] for i in infos)
    sm_bytes = sum(i["smooth_bytes"] for i in infos)
    achieved = sm_bytes / (sm_ms * 1e-3) / 1e9 if sm_ms > 0 else 0.0
    avg_launch_us = sm_ms * 1e3 / max(launches, 1)
    last = infos[-1]
    log("bench: solve %.3f ms (median), step %.3f ms, iters %d, vcycles %d, refinements %d, rel %.2e"
        % (solve_ms, ms_per_step, last["iters"], last["vcycles"], last["refinements"], last["rel_resid"]))
    log("bench: smoother %d launches, avg %.1f us, %.1f GB/s" % (launches, avg_launch_us, achieved))

    # the plain FP64 solve of the same problem, same GPU, same tolerance
    fp64 = []
    for _ in range(max(3, args.steps)):
        v.zero_()
        fp64.append(g.poisson_solve(rho, v, rtol=w.rtol, precision=0, profile=1))
    fp64_ms = statistics.median(i["ms_total"] for i in fp64[1:])
    f_ms = sum(i["smooth_ms"] for i in fp64[1:])
    f_b = sum(i["smooth_bytes"] for i in fp64[1:])
    f_l = sum(i["smooth_launches"] for i in fp64[1:])
    fp64_gbs = f_b / (f_ms * 1e-3) / 1e9 if f_ms > 0 else 0.0
    log("bench: fp64 solve %.3f ms, iters %d, smoother %.1f GB/s (avg %.1f us)"
        % (fp64_ms, fp64[-1]["iters"], fp64_gbs, f_ms * 1e3 / max(f_l, 1)))

    # algorithmic bytes of one launch (a half-sweep), per interior node of the
    # grid: 12 B (FP64) or 6 B (FP32) for a half-sweep that reads the other
    # colour, f and writes its own colour (24 / 12 B per full sweep)
    interior = (n - 2) ** 3
    sm_bpp = (sm_bytes / launches / interior) if launches else 0.0
    out = {
        "metric": "time-to-1e-10-residual per Poisson solve at 257^3; smoother HBM GB/s vs peak",
        "value": round(solve_ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "atoms": len(w.atoms), "rtol": w.rtol,
                   "form": "fp32 V-cycles in fp64 refinement" if mixed else "fp64",
                   "parallelism": "single GPU"},
        "solve": {"iters": last["iters"], "vcycles": last["vcycles"], "refinements": last["refinements"],
                  "rel_resid": last["rel_resid"]},
        "fp64_solve_ms": round(fp64_ms, 4),
        "fp64_iters": fp64[-1]["iters"],
        "fp64_smoother_gbs": round(fp64_gbs, 1),
        "fp64_smoother_frac": round(fp64_gbs / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_half<%s> (red-black half-sweep, finest level)" % ("float" if mixed else "double"),
                     "bytes_per_point_per_launch": round(sm_bpp, 3), "avg_launch_us": round(avg_launch_us, 2),
                     "launches": launches},
    }

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, xs, rho.cpu().numpy(), args.cpu_cycles)
    g.close()
    print(json.dumps(out), flush=True)


def cpu_baseline(w, xs, rho, cycles):
    """The oracle (plain C FP64 V(2,2) cycles, OpenMP) on the same solve: a
    few cycles timed, then scaled to the cycles its measured contraction
    needs for the same tolerance."""
    import numpy as np
    import oracle
    oracle.lib()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    center = tuple(0.5 * (x[0] + x[-1]) for x in xs)
    Q = oracle.moments(xs, rho, 4, center)
    v = np.zeros_like(rho)
    oracle.boundary_values(xs, Q, v, 1, 4, center)
    t0 = time.perf_counter()
    cyc, rel, hist = oracle.solve(xs, rho, v, rtol=w.rtol, max_cycles=cycles)
    dt = time.perf_counter() - t0
    rate = (hist[-1] / hist[0]) ** (1.0 / max(len(hist) - 1, 1)) if len(hist) > 1 else hist[0]
    need = cyc if rel <= w.rtol else cyc + math.ceil(math.log(w.rtol / rel) / math.log(rate))
    est_ms = dt * 1e3 / cyc * need
    log("bench: oracle %d cycles in %.2f s (%d threads), contraction %.3f, est. %d cycles to %.0e"
        % (cyc, dt, cores, rate, need, w.rtol))
    return {"value": round(est_ms, 1), "unit": "ms", "cores": cores, "kind": "oracle",
            "sample": "%d V(2,2) cycles of the %d^3 solve (%.2f s), extrapolated to %d cycles by the "
                      "measured contraction %.3f" % (cyc, len(xs[0]), dt, need, rate)}


if __name__ == "__main__":
    main()
