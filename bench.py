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
bounded sample: whole FP64 solves of the same 257^3 problem to the same
tolerance, repeated for about ten seconds.
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

# HBM bytes per launch of the dominant kernel (finest-level FP32 half-sweep,
# launch mix of one headline solve: 54 plain, 12 with partials, 6 from zero),
# from two rocprofv3 --pmc runs of `bench.py --steps 1 --warmup 0 --no-cpu
# --no-clean --solve-only` (FETCH_SIZE, then WRITE_SIZE; per-variant means
# over all its FP32 solves), each counter scaled by what it reads for a
# 512 MiB device copy (`bench.py --copy-calibration 512`: FETCH_SIZE x2.000,
# WRITE_SIZE x1.000). Summary: profiles/k_half2_fp32_finest_257_traffic.md.
# The figure belongs to the kernel source it was measured on and to the same
# solve form and start; `traffic` is reported as null when either differs.
COUNTER_TRAFFIC = {"kernel_sha256_16": "d4f5ed99b79fa847", "form": (1, 0, 8, 4, 3, 3, 0.05, 2),
                   "bytes_per_launch": 121.45e6}


def half_sweep_source_digest():
    """First 16 hex digits of the SHA-256 of the half-sweep kernel's source."""
    import hashlib
    path = os.path.join(ROOT, "paper_0806_1723_amd", "csrc", "mg_kernels.hip")
    src = open(path).read()
    a = src.index("template <typename T, int MODE, bool ZERO_IN, bool DOT, bool ZERO_FACES, bool TOP>\n__global__")
    b = src.index("// Resident workgroups of one half-sweep variant")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def smoother_label(t, form):
    """The finest-level smoother kernel a solve form times (profile = 1)."""
    if form.get("fused_sweeps", 0) <= 1:
        return "k_half2<%s, GS, *, *, true, true> (red-black half-sweep, finest level)" % t
    return ("k_gs_block<%s, S, *, *, true> (S red-black half-sweeps in one pass, finest level: the pre-smoothing "
            "from zero and the post-smoothing)" % t)


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
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU time over which the oracle baseline repeats whole solves")
    ap.add_argument("--no-clean", action="store_true", help="skip the 513^3 MALL-free smoother roofline")
    ap.add_argument("--clean-only", action="store_true",
                    help="only the 513^3 MALL-free smoother roofline (one JSON object), for kernel traces")
    ap.add_argument("--train", type=int, default=200, help="config 4: training problems")
    ap.add_argument("--train-steps", type=int, default=2400, help="config 4: Adam steps per net")
    ap.add_argument("--validate", type=int, default=50, help="config 4: labels checked by the oracle")
    ap.add_argument("--train5", type=int, default=32, help="config 5: perturbed copies the guess net trains on")
    ap.add_argument("--fused-sweeps", type=int, default=None,
                    help="opts.fused_sweeps for every solve (default: the library's)")
    ap.add_argument("--solve-only", action="store_true",
                    help="report the solve alone (no sphere, interstitial-density or matrix-element objects)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (the Poisson solve would "
              "shard by z-slabs with halo exchange, see the design notes)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.config == 4:
        bench_learned(args)
        return
    if args.config == 5 and not args.n:
        bench_batched(args)
        return

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
    nb = w.n_batch
    g = lasto.Grid(*xs, n_batch=nb)
    log("bench: %s, levels %s" % (w.name, [l[0] for l in g.levels()]))
    rho = g.empty()
    v = g.empty()
    atoms = w.batch_atoms if nb > 1 else w.atoms
    centers = np.array([a.center for a in w.atoms])
    radii = np.array([a.radius for a in w.atoms])

    # V(3,3) cycles (with the exact coarsest solve, fewer cycles than V(2,2)
    # for less time in both forms). The mixed form takes as many FP32 PCG
    # steps per FP64 refinement as its measured convergence needs to reach
    # the tolerance (adaptive, inner_rate), at most 4 in the first refinement
    # (FP32 rounding bounds its reduction near 2e-5) and 8 in later ones. The
    # start is the analytic monopole superposition of the atoms, computed
    # inside the timed solve (guess = 2); the zero start is reported beside.
    form = dict(precision=mixed, method=0, nu1=3, nu2=3, inner_first=4 if mixed else 0,
                inner_iters=8 if mixed else 5, inner_rate=0.05 if mixed else 0.0)
    if args.fused_sweeps is not None:
        form["fused_sweeps"] = args.fused_sweeps
    start = dict(guess=2, atoms=atoms)
    if args.clean_only:
        g.close()
        print(json.dumps(bench_clean_roofline(args, lasto, I, form)), flush=True)
        return

    def step(profile, precision):
        g.pseudo_density(atoms, rho_out=rho)
        v.zero_()
        opts = dict(form, precision=precision)
        info = g.poisson_solve(rho, v, rtol=w.rtol, profile=profile, **opts, **start)
        sph = g.sphere_interp(v, centers, radii)
        return info, sph

    for _ in range(args.warmup):
        step(0, mixed)
    torch.cuda.synchronize()
    # The first timed step launches every finest-level sweep with a pair of
    # dispatch-stamped events (the roofline's kernel time); the stamps delay
    # the next dispatch by a few microseconds each, so the solve time is the
    # median of the other steps (all of them when only one is timed).
    infos = []
    t0 = time.perf_counter()
    for si in range(args.steps):
        info, _ = step(1 if si == 0 else 0, mixed)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    solve_ms = statistics.median(i["ms_total"] for i in (infos[1:] if len(infos) > 1 else infos))
    launches = infos[0]["smooth_launches"]
    sm_ms = infos[0]["smooth_ms"]
    sm_bytes = infos[0]["smooth_bytes"]
    achieved = sm_bytes / (sm_ms * 1e-3) / 1e9 if sm_ms > 0 else 0.0
    avg_launch_us = sm_ms * 1e3 / max(launches, 1)
    last = infos[-1]
    # the solutions of the timed forms (first right-hand side), for their
    # error against the oracle's solve of the same problem
    kept = {"mixed" if mixed else "fp64": (v[0] if nb > 1 else v).cpu().numpy()}
    log("bench: solve %.3f ms (median), step %.3f ms, iters %d, vcycles %d, refinements %d, rel %.2e"
        % (solve_ms, ms_per_step, last["iters"], last["vcycles"], last["refinements"], last["rel_resid"]))
    log("bench: smoother %d launches, avg %.1f us, %.1f GB/s" % (launches, avg_launch_us, achieved))

    # the plain FP64 solve of the same problem, same GPU, same tolerance
    fp64 = []
    for si in range(max(3, args.steps)):
        v.zero_()
        fp64.append(g.poisson_solve(rho, v, rtol=w.rtol, precision=0, nu1=form["nu1"], nu2=form["nu2"],
                                    fused_sweeps=form.get("fused_sweeps", 0), profile=1 if si == 1 else 0, **start))
    fp64_ms = statistics.median(i["ms_total"] for i in fp64[2:])
    kept["fp64"] = (v[0] if nb > 1 else v).cpu().numpy()
    f_ms = fp64[1]["smooth_ms"]
    f_b = fp64[1]["smooth_bytes"]
    f_l = fp64[1]["smooth_launches"]
    fp64_gbs = f_b / (f_ms * 1e-3) / 1e9 if f_ms > 0 else 0.0
    log("bench: fp64 solve %.3f ms, iters %d, smoother %.1f GB/s (avg %.1f us)"
        % (fp64_ms, fp64[-1]["iters"], fp64_gbs, f_ms * 1e3 / max(f_l, 1)))

    # both forms again from the faces alone (zero interior)
    zero = {}
    for name, prec in (("mixed", mixed), ("fp64", 0)):
        zi = []
        for _ in range(max(3, args.steps)):
            v.zero_()
            zi.append(g.poisson_solve(rho, v, rtol=w.rtol, guess=1, **dict(form, precision=prec)))
        zero[name] = dict(ms=round(statistics.median(i["ms_total"] for i in zi[1:]), 4),
                          iters=zi[-1]["iters"], vcycles=zi[-1]["vcycles"], rel_resid=zi[-1]["rel_resid"])
    log("bench: from the zero start: mixed %.3f ms (%d V-cycles), fp64 %.3f ms (%d iterations)" % (
        zero["mixed"]["ms"], zero["mixed"]["vcycles"], zero["fp64"]["ms"], zero["fp64"]["iters"]))

    # the direct solve by fast diagonalisation on the same problem (six FP64
    # GEMMs along the axes; the first call builds the 1-D decompositions)
    fdm = []
    for _ in range(max(3, args.steps)):
        v.zero_()
        fdm.append(g.fdm_solve(rho, v))
    fdm_ms = statistics.median(i["ms_total"] for i in fdm[1:])
    kept["fdm_direct"] = (v[0] if nb > 1 else v).cpu().numpy()
    m3 = [len(x) - 2 for x in xs]
    fdm_flops = 4.0 * nb * float(np.prod(m3)) * sum(m3)
    log("bench: fdm direct solve %.3f ms (first call %.1f ms), rel %.2e, %.1f TFLOP/s in its GEMMs' flops over the "
        "whole call" % (fdm_ms, fdm[0]["ms_total"], fdm[-1]["rel_resid"], fdm_flops / (fdm_ms * 1e-3) / 1e12))

    # algorithmic bytes of one launch (a half-sweep), per interior node of the
    # grid: 12 B (FP64) or 6 B (FP32) for a half-sweep that reads the other
    # colour, f and writes its own colour (24 / 12 B per full sweep)
    interior = (n - 2) ** 3 * nb
    sm_bpp = (sm_bytes / launches / interior) if launches else 0.0
    traffic = None
    form_key = (form["precision"], form["method"], form["inner_iters"], form["inner_first"], form["nu1"], form["nu2"],
                form["inner_rate"], start["guess"])
    if (n == 257 and args.config == 3 and form_key == COUNTER_TRAFFIC["form"] and form.get("fused_sweeps", 0) <= 1
            and half_sweep_source_digest() == COUNTER_TRAFFIC["kernel_sha256_16"]):
        traffic = COUNTER_TRAFFIC["bytes_per_launch"]
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
        "config": {"workload": w.name, "n": n, "atoms": len(w.atoms), "rtol": w.rtol, "right_hand_sides": nb,
                   "form": ("fp32 V-cycles in fp64 refinement, adaptive inner steps" if mixed else "fp64") +
                           ", from the analytic monopole start (timed)",
                   "parallelism": "single GPU"},
        "solve": {"iters": last["iters"], "vcycles": last["vcycles"], "refinements": last["refinements"],
                  "rel_resid": last["rel_resid"], "per_rhs_rel_resid": last["batch_rel_resid"],
                  "ms_per_rhs": round(solve_ms / nb, 4),
                  # the level the cycle solves exactly by fast diagonalisation (its coarsest)
                  "coarsest_exact_level": last["coarse_level"],
                  "coarsest_exact_shape": (list(g.levels()[last["coarse_level"]])
                                           if last["coarse_level"] >= 0 else None)},
        "zero_start": zero,
        "fp64_solve_ms": round(fp64_ms, 4),
        "fp64_iters": fp64[-1]["iters"],
        "fp64_smoother_gbs": round(fp64_gbs, 1),
        "fp64_smoother_frac": round(fp64_gbs / HBM_PEAK_GBS, 4),
        "fdm_direct_solve": {"ms": round(fdm_ms, 4), "first_call_ms": round(fdm[0]["ms_total"], 2),
                             "rel_resid": fdm[-1]["rel_resid"], "gemm_tflop": round(fdm_flops / 1e12, 4),
                             "note": "fast diagonalisation (six FP64 GEMMs), beside the multigrid headline"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": round(sm_bytes / launches) if launches else 0,
                     "kernel": smoother_label("float" if mixed else "double", form),
                     "bytes_per_point_per_launch": round(sm_bpp, 3), "avg_launch_us": round(avg_launch_us, 2),
                     "launches": launches, "events_on": "timed step 1 of %d" % args.steps},
    }

    # the whole iteration's algorithmic bytes at the finest level (every
    # launch's compulsory reads and writes) over the event-timed iteration
    out["solve_phases"] = {
        name: {"ms_bc": round(inf["ms_bc"], 4), "ms_guess": round(inf["ms_guess"], 4),
               "ms_cycles": round(inf["ms_cycles"], 4), "alg_bytes": inf["alg_bytes"],
               "alg_gbs_over_cycles": round(inf["alg_bytes"] / (inf["ms_cycles"] * 1e-3) / 1e9, 1)
               if inf["ms_cycles"] > 0 else None, "fallback_used": inf["fallback_used"]}
        for name, inf in (("mixed" if mixed else "timed", last), ("fp64", fp64[-1]))}
    log("bench: iteration bandwidth (finest-level algorithmic bytes / event-timed cycles): %s"
        % {k: v["alg_gbs_over_cycles"] for k, v in out["solve_phases"].items()})
    if args.config == 3 and not args.n and not args.no_clean:
        out["roofline_clean"] = bench_clean_roofline(args, lasto, I, form)
    out["roofline"]["mall_assisted"] = bool(n <= 257)
    if n <= 257:
        out["roofline"]["note"] = ("the finest level's FP32 arrays (u, f: ~150 MB with padding) fit the 256 MB "
                                   "Infinity Cache; roofline_clean gives the same kernel at 513^3")

    if not args.solve_only:
        out["spheres"] = bench_spheres(args, lasto, I, g, w, xs, v, rho, centers, radii)
        out["interstitial_density"] = bench_interstitial(args, lasto, I, g, w, xs, centers, radii)
        out["matrix_elements"] = bench_matrix_elements(args, lasto, I)

    if not args.no_cpu:
        out["cpu_baseline"], v_oracle = cpu_baseline(w, xs, (rho[0] if nb > 1 else rho).cpu().numpy(),
                                                     args.cpu_seconds)
        # relative W-norm (dual-volume) difference over the interior
        vol = np.einsum("k,j,i->kji", *[dual_widths(x) for x in (xs[2], xs[1], xs[0])])[1:-1, 1:-1, 1:-1]
        inner = (slice(1, -1),) * 3
        ref = float(np.sqrt((vol * v_oracle[inner] ** 2).sum()))
        out["err_vs_oracle"] = {k: float(np.sqrt((vol * (a[inner] - v_oracle[inner]) ** 2).sum())) / ref
                                for k, a in kept.items()}
        out["err_vs_oracle"]["norm"] = ("relative W-norm of the difference over the interior, against the "
                                        "oracle's solve to the same tolerance (first right-hand side)")
        log("bench: error against the oracle's solution: %s" % {k: "%.2e" % e for k, e in out["err_vs_oracle"].items()
                                                                  if k != "norm"})
        if nb > 1:
            out["cpu_baseline"]["value"] = round(out["cpu_baseline"]["value"] * nb, 1)
            out["cpu_baseline"]["sample"] += "; times %d right-hand sides" % nb
    g.close()
    print(json.dumps(out), flush=True)


def copy_ceiling(lasto, gib=2.0, reps=10):
    """The streaming ceiling, event-timed over arrays of `gib` GiB (far beyond
    the 256 MB Infinity Cache): torch's device copy, and the library's stream
    probe as a copy (one read, one write) and as a + b (two reads, one write:
    the half-sweep's mix, the ceiling the smoother is held to). Bytes moved per
    second, medians of `reps`."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    d = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, nbytes):
        for _ in range(2):
            fn()
        ts = []
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = statistics.median(ts)
        return round(nbytes / (ms * 1e-3) / 1e9, 1)

    out = {"torch_copy_gbs": timed(lambda: d.copy_(a), 2 * n * 8),
           "probe_copy_gbs": timed(lambda: lasto.stream_probe(a, d), 2 * n * 8),
           "probe_two_reads_one_write_gbs": timed(lambda: lasto.stream_probe(a, d, b=b), 3 * n * 8),
           "gib_per_array": gib}
    assert torch.equal(d, a + b)
    out["gbs"] = max(out["probe_two_reads_one_write_gbs"], out["probe_copy_gbs"], out["torch_copy_gbs"])
    out["frac_of_peak"] = round(out["gbs"] / HBM_PEAK_GBS, 4)
    del a, b, d
    torch.cuda.empty_cache()
    return out


def bench_clean_roofline(args, lasto, I, form):
    """The dominant kernel where the Infinity Cache cannot hold its arrays:
    one right-hand side of the 309-atom cluster on its graded 513^3 mesh
    (FP32 u and f ~1.1 GB, FP64 ~2.2 GB), one mixed and one FP64 solve with
    every finest-level half-sweep event-timed (12 or 8 B per updated node and
    colour pass, as at 257^3), against 8 TB/s and against the measured copy
    ceiling."""
    import torch
    cc = copy_ceiling(lasto)
    log("bench: streaming ceiling %s" % cc)
    w = I.config(5)
    xs = lasto.mesh_for(w.axes)
    g = lasto.Grid(*xs)
    rho = g.pseudo_density(w.batch_atoms[0])
    v = g.empty()
    res = {"workload": "309-atom Mackay icosahedron, graded 513^3, L=80, one right-hand side", "copy_ceiling": cc}
    for name, prec in (("fp32_in_mixed", 1), ("fp64", 0)):
        for rep in range(2):   # the first also warms up
            v.zero_()
            opts = dict(form, precision=prec)
            if prec == 0:
                opts.update(inner_first=0)
            info = g.poisson_solve(rho, v, rtol=1e-10, profile=1, **opts)
        launches, ms, by = info["smooth_launches"], info["smooth_ms"], info["smooth_bytes"]
        gbs = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        res[name] = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "frac_of_copy_ceiling": round(gbs / cc["gbs"], 4),
                     "launches": launches, "avg_launch_us": round(ms * 1e3 / max(launches, 1), 2),
                     "algorithmic_bytes_per_launch": round(by / max(launches, 1)),
                     "solve_ms": round(info["ms_total"], 3), "iters": info["iters"], "vcycles": info["vcycles"],
                     "rel_resid": info["rel_resid"],
                     "iteration_alg_gbs": round(info["alg_bytes"] / (info["ms_cycles"] * 1e-3) / 1e9, 1)
                     if info["ms_cycles"] > 0 else None}
        log("bench: 513^3 %s: smoother %.1f GB/s (%.3f of 8 TB/s, %.3f of the copy ceiling), avg %.1f us; solve "
            "%.2f ms, %d iters" % (name, gbs, gbs / HBM_PEAK_GBS, gbs / cc["gbs"], ms * 1e3 / max(launches, 1),
                                   info["ms_total"], info["iters"]))
    g.close()
    del rho, v
    torch.cuda.empty_cache()
    return res


def bench_spheres(args, lasto, I, g, w, xs, v, rho, centers, radii):
    """Inside the spheres, on the solved field: projection onto y_LM
    (eq. (3.6), 8 x 9 rule), the radial solve of eq. (3.4) on 429-point log
    meshes, and the energy integral (grid part over every node, sphere parts),
    each call timed with events on the grid's stream; the median of the
    timed repetitions. With the CPU leg on, the oracle's same three steps
    once each."""
    import numpy as np
    import torch
    nb = g.n_batch
    atoms_b = w.batch_atoms if nb > 1 else [w.atoms]
    radii = I.muffin_tin_radii(w.atoms)
    rho_lm = np.stack([I.sphere_density(a, radii=radii) for a in atoms_b])
    if nb == 1:
        rho_lm = rho_lm[0]
    Z = np.full(len(radii), I.PD_Z)
    S = lasto.Spheres(g, centers, radii, Z=Z, n_theta=8, n_phi=9, n_rad=I.N_RAD, r_min=I.R_MIN)
    rl = torch.from_numpy(rho_lm).to("cuda")
    vR = S.project(v)
    v_lm = S.radial(vR, rl)
    S.energy(v, rho, v_lm, rl)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t_proj, t_rad, t_en, t_all = [], [], [], []
    for _ in range(max(args.steps, 5)):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev[0].record()
        S.project(v, vR)
        ev[1].record()
        S.radial(vR, rl, v_lm)
        ev[2].record()
        e = S.energy(v, rho, v_lm, rl)
        ev[3].record()
        torch.cuda.synchronize()
        t_all.append((time.perf_counter() - w0) * 1e6)
        t_proj.append(ev[0].elapsed_time(ev[1]) * 1e3)
        t_rad.append(ev[1].elapsed_time(ev[2]) * 1e3)
        t_en.append(ev[2].elapsed_time(ev[3]) * 1e3)
    med = statistics.median
    nodes = int(np.prod(g.shape))
    grid_bytes = 16 * nodes
    e = np.atleast_2d(e)
    log("bench: spheres: project %.1f us, radial %.1f us, energy %.1f us (grid part reads %.1f MB), "
        "whole %.1f us; E_H/2 parts %s" % (med(t_proj), med(t_rad), med(t_en), grid_bytes / 1e6, med(t_all),
                                          (0.5 * e[0]).tolist()))
    out = {"atoms": len(radii), "rule": "8 x 9", "n_rad": I.N_RAD, "right_hand_sides": nb,
           "project_us": round(med(t_proj), 2), "radial_us": round(med(t_rad), 2),
           "energy_us": round(med(t_en), 2), "whole_us": round(med(t_all), 2),
           "energy_grid_bytes": grid_bytes,
           "energy_gbs_lower_bound": round(grid_bytes / (med(t_en) * 1e-6) / 1e9, 1),
           "integral_v_rho": [round(float(x), 9) for x in e.sum(axis=1)]}
    if not args.no_cpu:
        import oracle
        oracle.lib()
        v_h = (v[0] if nb > 1 else v).cpu().numpy()
        rho_h = (rho[0] if nb > 1 else rho).cpu().numpy()
        rl_h = rho_lm[0] if nb > 1 else rho_lm
        t0 = time.perf_counter()
        d, _ = oracle.sphere_rule(8, 9)
        vals = oracle.interp(xs, v_h, oracle.sphere_points(centers, radii, d)).reshape(len(radii), -1)
        wR = oracle.sphere_project(vals, 8, 9)
        t1 = time.perf_counter()
        wl = oracle.sphere_radial(radii, Z, I.R_MIN, wR, rl_h)
        t2 = time.perf_counter()
        oracle.energy_grid(xs, v_h, rho_h, centers, radii)
        oracle.sphere_energy(radii, I.R_MIN, wl, rl_h)
        t3 = time.perf_counter()
        out["cpu_oracle_ms"] = {"project": round((t1 - t0) * 1e3, 2), "radial": round((t2 - t1) * 1e3, 2),
                                "energy": round((t3 - t2) * 1e3, 2), "cores": 1,
                                "sample": "one right-hand side, once each"}
        log("bench: spheres on the oracle: %s" % out["cpu_oracle_ms"])
    S.close()
    return out


FP64_MFMA_PEAK_TFLOPS = 78.6


def bench_interstitial(args, lasto, I, g, w, xs, centers, radii):
    """The output density at every node outside the spheres: the Table 1
    basis (25 functions per atom), 5 doubly occupied states per atom, seeded
    coefficients. Algorithmic flops 2 * nodes * n_basis * n_states (the
    contraction) per call, over the event-timed call; the median of the
    timed repetitions. With the CPU leg on, the oracle's value at a sample of
    nodes, scaled to the whole grid."""
    import numpy as np
    import torch
    nodes = int(np.prod(g.copy_shape))
    n_basis = len(radii) * sum(2 * l + 1 for _, l, _ in I.LASTO_SHELLS)
    if 2.0 * nodes * n_basis * I.STATES_PER_ATOM * len(radii) > 40e12:
        return {"skipped": "over 40 TFLOP per call at this size"}
    coef, occ = I.basis_coefficients(len(radii), seed=7)
    cd = torch.from_numpy(coef).to("cuda")
    out_t = torch.empty(g.copy_shape, dtype=torch.float64, device="cuda")
    g.interstitial_density(centers, radii, I.LASTO_SHELLS, cd, occ, rho_out=out_t)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(max(2, min(args.steps, 3))):
        torch.cuda.synchronize()
        e0.record()
        g.interstitial_density(centers, radii, I.LASTO_SHELLS, cd, occ, rho_out=out_t)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = statistics.median(ts)
    nb, n_occ = coef.shape
    flops = 2.0 * nodes * nb * n_occ
    tf = flops / (ms * 1e-3) / 1e12
    log("bench: interstitial density %.2f ms, %d functions x %d states over %d nodes: %.1f TFLOP/s (%.3f of the "
        "FP64 matrix peak)" % (ms, nb, n_occ, nodes, tf, tf / FP64_MFMA_PEAK_TFLOPS))
    res = {"ms": round(ms, 3), "basis": nb, "states": n_occ, "nodes": nodes, "algorithmic_tflop": round(flops / 1e12, 3),
           "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tf / FP64_MFMA_PEAK_TFLOPS, 4),
                        "kernel": "k_interstitial<10> and <8> (FP64 16x16x4 matrix cores)"}}
    if not args.no_cpu:
        import oracle
        oracle.lib()
        rng = np.random.default_rng(8)
        m = 400
        idx = rng.integers(0, len(xs[0]), size=(m, 3))
        pts = np.stack([xs[0][idx[:, 0]], xs[1][idx[:, 1]], xs[2][idx[:, 2]]], axis=1)
        t0 = time.perf_counter()
        oracle.density_points(centers, I.LASTO_SHELLS, coef, occ, pts)
        dt = time.perf_counter() - t0
        res["cpu_oracle_ms"] = {"value": round(dt / m * nodes * 1e3, 1), "cores": 1,
                                "sample": "%d nodes in %.2f s, scaled to %d nodes" % (m, dt, nodes)}
        log("bench: interstitial density on the oracle: %s" % res["cpu_oracle_ms"])
    return res


def bench_matrix_elements(args, lasto, I):
    """The interstitial S and H of the 13-atom icosahedron at 129^3 (2.1 M
    nodes; the 55-atom 257^3 case is 100 TFLOP) with the Table 1 basis (325
    functions) and a smooth potential: event-timed calls, the median.
    Algorithmic flops: 3 products x 2 flops per node per entry of the upper
    triangle (diagonal included), as the kernel forms them."""
    import numpy as np
    import torch
    w = I.config(2)
    xs = lasto.mesh_for(w.axes)
    g = lasto.Grid(*xs)
    c = np.array([a.center for a in w.atoms])
    r = np.array([a.radius for a in w.atoms])
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    v = torch.from_numpy(-3.0 / np.sqrt(1.0 + X * X + Y * Y + Z * Z)).to("cuda")
    g.matrix_elements(v, c, r, I.LASTO_SHELLS)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        e0.record()
        g.matrix_elements(v, c, r, I.LASTO_SHELLS)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = statistics.median(ts)
    nodes = int(np.prod(g.copy_shape))
    nb = len(c) * sum(2 * l + 1 for _, l, _ in I.LASTO_SHELLS)
    flops = 3 * 2.0 * nodes * nb * (nb + 1) / 2
    tf = flops / (ms * 1e-3) / 1e12
    log("bench: interstitial S and H, %s, %d functions: %.2f ms, %.1f TFLOP/s (%.3f of the FP64 matrix peak)"
        % (w.name, nb, ms, tf, tf / FP64_MFMA_PEAK_TFLOPS))
    g.close()
    return {"workload": w.name, "basis": nb, "nodes": nodes, "ms": round(ms, 3),
            "algorithmic_tflop": round(flops / 1e12, 3),
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / FP64_MFMA_PEAK_TFLOPS, 4),
                         "kernel": "k_matrix_elements (FP64 16x16x4 matrix cores), with its weights and reduce"}}


def cpu_baseline(w, xs, rho, min_seconds):
    """The oracle (plain C FP64 V(2,2) cycles, OpenMP) on the same 257^3
    solve: whole solves to the same tolerance from the same faces, repeated
    until about `min_seconds` of CPU time have passed; the median solve."""
    import numpy as np
    import oracle
    oracle.lib()
    # the threads the oracle's OpenMP loops actually use
    cores = oracle.max_threads()
    center = tuple(0.5 * (x[0] + x[-1]) for x in xs)
    Q = oracle.moments(xs, rho, 4, center)
    v0 = np.zeros_like(rho)
    oracle.boundary_values(xs, Q, v0, 1, 4, center)
    times, cyc, rel = [], 0, 0.0
    t_start = time.perf_counter()
    while not times or (time.perf_counter() - t_start < min_seconds and len(times) < 50):
        v = v0.copy()
        t0 = time.perf_counter()
        cyc, rel, _ = oracle.solve(xs, rho, v, rtol=w.rtol, max_cycles=60)
        times.append(time.perf_counter() - t0)
    total = time.perf_counter() - t_start
    ms = statistics.median(times) * 1e3
    log("bench: oracle %d solves in %.1f s (%d threads), %d cycles each, rel %.2e, median %.1f ms"
        % (len(times), total, cores, cyc, rel, ms))
    # one host thread: two V-cycles of the same solve, scaled to the cycles a
    # whole solve takes (a bounded sample of a ~20 s single-thread solve)
    oracle.set_threads(1)
    vs = v0.copy()
    t0 = time.perf_counter()
    oracle.solve(xs, rho, vs, rtol=1e-300, max_cycles=2)
    t1 = (time.perf_counter() - t0) / 2.0
    oracle.set_threads(cores)
    one = {"ms_per_solve": round(t1 * cyc * 1e3, 1), "ms_per_cycle": round(t1 * 1e3, 1), "cores": 1,
           "sample": "2 V(2,2) cycles timed, times %d cycles" % cyc}
    log("bench: oracle on one thread: %.1f ms per cycle, %.0f ms per solve" % (t1 * 1e3, t1 * cyc * 1e3))
    return {"value": round(ms, 1), "unit": "ms", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(), "one_thread": one,
            "sample": "%d whole FP64 solves of the %d^3 problem to %.0e (%d V(2,2) cycles each, %.1f s in "
                      "all); median per solve" % (len(times), len(xs[0]), w.rtol, cyc, total)}, v


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def dual_widths(x):
    """Dual-cell widths of one axis (half cells at the ends)."""
    import numpy as np
    m = np.empty_like(x)
    m[1:-1] = 0.5 * (x[2:] - x[:-2])
    m[0] = 0.5 * (x[1] - x[0])
    m[-1] = 0.5 * (x[-1] - x[-2])
    return m


def conv_flops(shape, ch):
    """Multiply-add flops (2 per MAC) of the learned net's forward pass."""
    n = list(shape)
    dims = []
    for _ in range(4):
        dims.append(n[0] * n[1] * n[2])
        n = [(a + 1) // 2 for a in n]
    c0, c1, c2, c3 = ch
    layers = [(8, c0, 0), (c0, c1, 1), (c1, c2, 2), (c2, c3, 3), (c3, c3, 3), (c3, c2, 3), (c2, c1, 2), (c1, c0, 1)]
    return sum(2 * 27 * ci * co * dims[l] for ci, co, l in layers) + 2 * c0 * dims[0]


def bench_learned(args):
    """Config 4: the learned initial guess (net on a coarse level of each
    graded mesh, its output interpolated to the finest) and the learned
    coarse correction inside the cycle, against plain multigrid on held-out
    random clusters at 129^3. The nets are trained first, on the GPU, by the
    library's own kernels, on `--train` seeded problems whose labels are the
    method's own FP64 solves; a sample of labels is validated by the oracle
    (its own pseudo-density and its own operator's residual of the label)."""
    import numpy as np
    import torch

    from paper_0806_1723_amd import lasto, learned
    lasto.load()
    n = args.n or 129
    ntrain, ntest, nval = args.train, 8, min(args.validate, args.train)
    glev, clev = 2, 1   # the guess net's level; the coarse correction's level (exact solve one below: coarse = 2)
    ch = (16, 32, 32, 32)
    cap = 112   # level 1 of these meshes reaches 101 nodes per axis
    net = lasto.Net((cap, cap, cap), ch=ch, seed=7, **learned.NET_SCALES)
    net_c = lasto.Net((cap, cap, cap), ch=ch, seed=9, **learned.COARSE_SCALES)
    t0 = time.perf_counter()
    pairs, cpairs, val = [], [], []
    for sidx in range(ntrain):
        p = learned.make_problem(4, sidx, n)
        pairs.append(learned.training_pair(net, p, level=glev))
        cpairs += learned.coarse_pairs(net_c, p, clev, cycles=(0, 2))
        if sidx < nval:
            val.append((sidx, p.grid.coords, p.rho.cpu().numpy(), p.v_star.cpu().numpy(), p.atoms))
        p.grid.close()
        del p
    t_data = time.perf_counter() - t0
    log("bench: %d training problems at %d^3 (pairs on levels %d and %d) in %.1f s" % (ntrain, n, glev, clev, t_data))
    # the labels against the oracle: its own pseudo-density of the same atoms
    # and its own operator's relative residual of the label
    import oracle
    from paper_0806_1723_amd import inputs as I
    oracle.lib()
    t0 = time.perf_counter()
    worst_rho, worst_res = 0.0, 0.0
    for sidx, xs, rho, vstar, atoms in val:
        rho_o = oracle.pseudo_density(xs, I.atom_arrays(atoms))
        worst_rho = max(worst_rho, float(np.abs(rho - rho_o).max() / np.abs(rho_o).max()))
        worst_res = max(worst_res, oracle.rel_residual(xs, rho_o, vstar))
    log("bench: %d labels validated by the oracle in %.1f s: source max rel diff %.2e, label residual by the "
        "oracle's operator <= %.2e" % (len(val), time.perf_counter() - t0, worst_rho, worst_res))
    t0 = time.perf_counter()
    hist = learned.train(net, [], steps=args.train_steps, lr=2e-3, pairs=pairs)
    torch.cuda.synchronize()
    t_guess = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist_c = learned.train_coarse(net_c, cpairs, steps=args.train_steps, lr=2e-3)
    torch.cuda.synchronize()
    t_corr = time.perf_counter() - t0
    k = len(pairs)
    log("bench: trained guess net %.1f s (loss %.3e -> %.3e), coarse net %.1f s (loss %.3e -> %.3e)" % (
        t_guess, np.mean(hist[:k]), np.mean(hist[-k:]), t_corr, np.mean(hist_c[:len(cpairs)]),
        np.mean(hist_c[-len(cpairs):])))
    test_p = [learned.make_problem(4, 1000 + s, n) for s in range(ntest)]
    # forward-pass time of the guess net on its level of the first test problem
    learned.use_level(net, test_p[0].grid, glev)
    x = net.features(test_p[0].grid, test_p[0].rho, test_p[0].v_guess)
    y = torch.zeros(net.shape, dtype=torch.float32, device="cuda")
    for _ in range(3):
        net.forward(x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        net.forward(x, y)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 10
    flops = conv_flops(net.shape, ch)
    rows, mixed, coarse = [], [], []
    for p in test_p:
        for _ in range(2):   # second pass timed warm
            r = learned.compare(net, p, rtol=1e-10, level=glev)
            rm = learned.compare(net, p, rtol=1e-10, level=glev, precision=1, nu1=3, nu2=3, inner_iters=8,
                                 inner_first=4, inner_rate=0.05)
        rc = learned.compare_coarse(net_c, p, clev)
        rows.append(r)
        mixed.append(rm)
        coarse.append(rc)
        log("bench: %s FP64 zero %d/%.2f ms analytic %d/%.2f ms learned %d/%.2f ms (kept %s); mixed %d/%.2f %d/%.2f "
            "%d/%.2f; coarse net %d/%.2f vs %d/%.2f ms (kept %d of %d)" % (
                p.name[:26], r["zero"]["iters"], r["zero"]["ms"], r["analytic"]["iters"], r["analytic"]["ms"],
                r["learned"]["iters"], r["learned"]["ms"], r["learned"]["accepted"], rm["zero"]["vcycles"],
                rm["zero"]["ms"], rm["analytic"]["vcycles"], rm["analytic"]["ms"], rm["learned"]["vcycles"],
                rm["learned"]["ms"], rc["learned"]["iters"], rc["learned"]["ms"], rc["plain"]["iters"],
                rc["plain"]["ms"], rc["learned"]["accepted"], rc["learned"]["applied"]))
    med = lambda v: round(float(statistics.median(v)), 3)
    out = {
        "metric": "time-to-1e-10-residual per Poisson solve: learned guess vs plain multigrid (V-cycles saved)",
        "value": med([r["learned"]["ms"] for r in mixed]),
        "unit": "ms",
        "n_gpus": 1, "steps": ntest, "warmup": 1,
        "ms_per_step": med([r["learned"]["ms"] for r in mixed]),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 net + f32/f64 solve", "data": "synthetic",
        "config": {"workload": "random 13-55-atom clusters (seeds 40000+s), graded %d^3, L=48" % n,
                   "train_problems": ntrain, "test_problems": ntest, "net_channels": list(ch),
                   "guess_net_level": glev, "coarse_net_level": clev, "parallelism": "single GPU"},
        "labels_validated_by_oracle": {"problems": len(val), "source_max_rel_diff": worst_rho,
                                       "label_residual_by_oracle_max": worst_res},
        "fp64_pcg_iters": {k: [r[k]["iters"] for r in rows] for k in ("zero", "analytic", "learned")},
        "fp64_pcg_ms": {k: med([r[k]["ms"] for r in rows]) for k in ("zero", "analytic", "learned")},
        "learned_guess_kept": [bool(r["learned"]["accepted"]) for r in rows],
        "mixed_vcycles": {k: [r[k]["vcycles"] for r in mixed] for k in ("zero", "analytic", "learned")},
        "mixed_ms": {k: med([r[k]["ms"] for r in mixed]) for k in ("zero", "analytic", "learned")},
        "mixed_err_vs_label": max(r["err_vs_label"] for r in mixed),
        "coarse_net": {"iters": {k: [r[k]["iters"] for r in coarse] for k in ("plain", "learned")},
                       "ms": {k: med([r[k]["ms"] for r in coarse]) for k in ("plain", "learned")},
                       "kept_of_proposed": [[r["learned"]["accepted"], r["learned"]["applied"]] for r in coarse],
                       "form": "FP64 MG-PCG (flexible with the net), exact coarsest solve by LDS (coarse = 2)"},
        "training_s": {"data": round(t_data, 2), "guess_net": round(t_guess, 2), "coarse_net": round(t_corr, 2)},
        "roofline": {"bound": "mfma", "achieved": round(flops / (fwd_ms * 1e-3) / 1e12, 2), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(flops / (fwd_ms * 1e-3) / 1e12 / 2500.0, 5), "traffic": None,
                     "kernel": "guess net forward pass on level %d (k_conv<*> BF16 MFMA, all layers)" % glev,
                     "gflop": round(flops / 1e9, 3), "forward_ms": round(fwd_ms, 4), "grid": list(net.shape)},
    }
    for p in test_p:
        p.grid.close()
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """Config 5: 8 SCF-like perturbations of the 309-atom Mackay cluster on
    one batched 513^3 grid, solved together by the mixed form (FP32 V-cycles
    in FP64 refinement, adaptive inner steps) from three starts: the faces
    alone (zero interior), the analytic monopole superposition, and that plus
    the learned correction (net on a coarse level of the mesh, its output
    interpolated to the finest, judged per copy). The guess net is trained
    first, on the GPU, on `--train5` other perturbations of the same cluster
    (seeds 600+s) whose labels are the method's own FP64 solves; the eight
    benchmark copies (seeds 500..507) are held out."""
    import numpy as np
    import torch

    from paper_0806_1723_amd import inputs as I
    from paper_0806_1723_amd import lasto, learned
    lasto.load()
    w = I.config(5)
    xs = lasto.mesh_for(w.axes)
    n = len(xs[0])
    glev = 2
    ch = (16, 32, 32, 32)
    # the training problems: one copy at a time on a single-copy grid of the same mesh
    g1 = lasto.Grid(*xs)
    shape = g1.levels()[glev]
    cap = max(shape)
    net = lasto.Net((cap, cap, cap), ch=ch, seed=11, **learned.NET_SCALES)
    base = w.atoms
    t0 = time.perf_counter()
    pairs = []
    rho = g1.empty()
    for sidx in range(args.train5):
        atoms = I.perturb_atoms(base, 600 + sidx)
        g1.pseudo_density(atoms, rho_out=rho)
        vg = g1.empty()
        g1.boundary_values(rho, vg, bc=1)
        g1.analytic_guess(atoms, vg)
        vs = vg.clone()
        g1.poisson_solve(rho, vs, rtol=1e-10, bc=2, nu1=3, nu2=3)
        p = learned.Problem("perturbation %d" % sidx, atoms, g1, rho, vg, vs, {})
        pairs.append(learned.training_pair(net, p, level=glev))
        del vg, vs, p
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log("bench: %d training perturbations at %d^3 in %.1f s (net on level %d, %s)" % (
        args.train5, n, t_data, glev, list(shape)))
    t0 = time.perf_counter()
    hist = learned.train(net, [], steps=args.train_steps, lr=2e-3, pairs=pairs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    k = len(pairs)
    log("bench: trained guess net in %.1f s (loss %.3e -> %.3e)" % (t_train, np.mean(hist[:k]), np.mean(hist[-k:])))
    g1.close()
    del g1, rho
    torch.cuda.empty_cache()

    nb = w.n_batch
    g = lasto.Grid(*xs, n_batch=nb)
    learned.use_level(net, g, glev)
    rho = g.empty()
    v = g.empty()
    g.pseudo_density(w.batch_atoms, rho_out=rho)
    # at 513^3 the finest level dominates a cycle: V(3,3) with 4 sweeps each
    # way on the levels below takes 5 cycles where plain V(3,3) takes 6
    form = dict(precision=1, method=0, nu1=3, nu2=3, nu_coarse=4, inner_first=4, inner_iters=8, inner_rate=0.05)
    if args.fused_sweeps is not None:
        form["fused_sweeps"] = args.fused_sweeps
    starts = {"zero": dict(guess=1), "analytic": dict(guess=2, atoms=w.batch_atoms),
              "learned": dict(guess=3, atoms=w.batch_atoms, guess_net=net)}
    res = {}
    steps = max(args.steps, 1)
    for name, st in starts.items():
        infos = []
        for si in range(args.warmup + steps):
            v.zero_()
            infos.append(g.poisson_solve(rho, v, rtol=w.rtol, profile=1 if si == args.warmup else 0, **form, **st))
        timed = infos[args.warmup:]
        ms = statistics.median(i["ms_total"] for i in (timed[1:] if len(timed) > 1 else timed))
        last = timed[-1]
        res[name] = dict(ms=round(ms, 3), ms_per_rhs=round(ms / nb, 3), vcycles=last["vcycles"],
                         refinements=last["refinements"], ms_guess=round(last["ms_guess"], 3),
                         ms_cycles=round(last["ms_cycles"], 3), rel_resid=last["rel_resid"],
                         per_rhs_rel_resid=last["batch_rel_resid"], guess_accepted=last["guess_accepted"],
                         rel_start=last["rel_start"], resid_hist=last["resid_hist"],
                         smoother=(timed[0]["smooth_bytes"], timed[0]["smooth_ms"], timed[0]["smooth_launches"]))
        log("bench: 8 x %d^3 mixed from the %s start: %.2f ms (%.2f per right-hand side), %d V-cycles, %d "
            "refinements, guess %.2f ms, start rel %.2e, after each refinement %s%s" % (
                n, name, ms, ms / nb, last["vcycles"], last["refinements"], last["ms_guess"], last["rel_start"],
                ["%.1e" % x for x in last["resid_hist"]],
                (", learned start kept on %d of %d" % (last["guess_accepted"], nb)) if name == "learned" else ""))
    # plain FP64 MG-PCG on the same batch, zero and analytic starts
    fp64 = {}
    for name in ("zero", "analytic"):
        infos = []
        for si in range(1 + min(steps, 2)):
            v.zero_()
            infos.append(g.poisson_solve(rho, v, rtol=w.rtol, precision=0, nu1=3, nu2=3, **starts[name]))
        ms = statistics.median(i["ms_total"] for i in infos[1:])
        fp64[name] = dict(ms=round(ms, 3), iters=infos[-1]["iters"])
        log("bench: 8 x %d^3 FP64 from the %s start: %.2f ms, %d iterations" % (n, name, ms, infos[-1]["iters"]))
    sb, sm, sl = res["learned"]["smoother"]
    achieved = sb / (sm * 1e-3) / 1e9 if sm > 0 else 0.0
    for r in res.values():
        r.pop("smoother")
    out = {
        "metric": "time-to-1e-10-residual per Poisson solve at 257^3; smoother HBM GB/s vs peak",
        "value": res["learned"]["ms"],
        "unit": "ms",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": res["learned"]["ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64 (bf16 net)", "data": "synthetic",
        "config": {"workload": "%s, 8 perturbations (seeds 500-507) in one batched grid" % w.name, "n": n,
                   "atoms": len(w.atoms), "rtol": w.rtol, "right_hand_sides": nb,
                   "form": "fp32 V-cycles in fp64 refinement, adaptive inner steps, learned start",
                   "parallelism": "single GPU"},
        "starts": res,
        "fp64": fp64,
        "guess_net": {"level": glev, "grid": list(shape), "channels": list(ch), "train_perturbations": args.train5,
                      "train_steps": args.train_steps, "data_s": round(t_data, 2), "train_s": round(t_train, 2),
                      "loss_first": float(np.mean(hist[:k])), "loss_last": float(np.mean(hist[-k:]))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": smoother_label("float", form) + ", 8 copies",
                     "launches": sl, "avg_launch_us": round(sm * 1e3 / max(sl, 1), 2),
                     "algorithmic_bytes_per_launch": round(sb / max(sl, 1))},
    }
    g.close()
    print(json.dumps(out), flush=True)


def copy_calibration(mib):
    """A plain device copy of known size (torch's copy kernel), for scaling
    hardware byte counters: FETCH_SIZE and WRITE_SIZE of one dispatch should
    each read `mib` MiB."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "bytes_read": n * 4, "bytes_written": n * 4,
                      "dispatches": 5}), flush=True)


if __name__ == "__main__":
    main()
