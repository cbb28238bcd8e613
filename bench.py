"""Benchmark of the multiresolution hot path on one MI355X.

A step is one SSP-RK3 step of the whole grid (three stages, each a ghost
reconstruction -- substitution, c->f and f->c patches -- plus the fused FD
advection + RK combine) followed by one detail pass (wide ghost
reconstruction, FP64 forward transform, per-block norms).  The timed region
starts with the field resident in HBM.  Adaptation is timed in a second loop
(every `adapt_every` steps) and reported separately.

Prints one JSON line.  Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2112_07537_amd import mr  # noqa: E402
from paper_2112_07537_amd import workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0
DEVICE_SRC = os.path.join(ROOT, "paper_2112_07537_amd", "csrc", "mr_device.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "c5_hbm_traffic.md")
METRIC = "RK3-step grid points/s (ghost+details+RHS) & % HBM peak, FP32-batched vs FP64-plain"


def log(*a):
    print("[bench %.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


T0 = time.time()


def make_grid(cfg, prec=None, exec_mode=0, max_blocks=150000):
    g = mr.Grid(cfg["nb"], cfg["N"], cfg["Nt"], fd_order=cfg["fd"], level_min=cfg["level_min"],
                level_max=cfg["level_max"], prec=prec or cfg["prec"],
                eps_refine=cfg["eps_refine"], eps_coarsen=cfg["eps_coarsen"],
                exec_mode=exec_mode, max_blocks=max_blocks)
    if cfg.get("tree"):
        g.set_tree(wl.geometric_tree())
        g.sample_ic(*cfg["ic"])
    else:
        st = g.init_ic(*cfg["ic"])
        log("init: %d leaves, %d refine / %d coarsen in %d adapt iterations" %
            (g.n_blocks(), st.refined, st.coarsened, st.iters))
    return g


def timed_steps(g, cfg, steps, warmup, adapt_every=0):
    kind, p = wl.velocity_spec(cfg["vel"])
    vel = mr.velocity(kind, *p)
    dt = g.cfl_dt(vel, cfg["cfl"])
    for _ in range(warmup):
        g.rk3_step(dt, vel)
        g.details_async()
    g.sync()
    t_adapt = 0.0
    n_adapt = 0
    points = 0
    t0 = time.perf_counter()
    for s in range(steps):
        points += g.n_blocks() * cfg["nb"] ** 3
        g.rk3_step(dt, vel)
        g.details_async()
        if adapt_every and (s + 1) % adapt_every == 0:
            ta = time.perf_counter()
            g.adapt()
            t_adapt += time.perf_counter() - ta
            n_adapt += 1
            dt = g.cfl_dt(vel, cfg["cfl"])
    g.sync()
    t = time.perf_counter() - t0
    return t, points, t_adapt, n_adapt


def timed_fused(g, cfg, steps, warmup):
    """The same work through the fused entry point: per step the detail pass
    of the current state, then the RK3 step whose first stage reuses the
    detail pass's ghosts (three ghost reconstructions per step, not four)."""
    kind, p = wl.velocity_spec(cfg["vel"])
    vel = mr.velocity(kind, *p)
    dt = g.cfl_dt(vel, cfg["cfl"])
    for _ in range(warmup):
        g.details_rk3_step_async(dt, vel)
    g.sync()
    points = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        points += g.n_blocks() * cfg["nb"] ** 3
        g.details_rk3_step_async(dt, vel)
    g.sync()
    return time.perf_counter() - t0, points


def cpu_baseline(g, cfg, n_sample=400, seed=1234, budget_s=15.0):
    """The FP64 oracle timed on a seeded sample of the same grid: per sampled
    block, three stages of (substitution + ghost reconstruction + RHS) and one
    detail transform, computed from the GPU's current state.  Blocks are taken
    in the seeded order until about `budget_s` seconds of CPU work."""
    from oracle import grid as og
    meta = [tuple(int(v) for v in m) for m in g.block_meta()]
    data = g.field_get()
    o = og.Grid(cfg["nb"], cfg["N"], cfg["Nt"], fd_order=cfg["fd"], level_min=cfg["level_min"],
                level_max=cfg["level_max"], eps_refine=cfg["eps_refine"],
                eps_coarsen=cfg["eps_coarsen"])
    data = data.astype(np.float64)
    o.blocks = {k: data[b] for b, k in enumerate(meta)}
    o._index()
    rng = np.random.default_rng(seed)
    sample = [meta[i] for i in rng.choice(len(meta), size=min(n_sample, len(meta)), replace=False)]
    kind, p = wl.velocity_spec(cfg["vel"])
    vel = (kind, p)
    from threadpoolctl import threadpool_limits
    limiter = threadpool_limits(limits=1)   # the oracle on exactly one core
    t0 = time.perf_counter()
    done = 0
    for k in sample:
        mask = o.substitution_mask(k)
        for _ in range(3):
            if mask.any():
                for deg in (1, 2, 3):
                    z, y, x, v = o.substitution_values(k, deg, mask)
                    o.blocks[k][z, y, x] = v
            o.rhs_block(k, vel)
        o.block_details(k)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    t = time.perf_counter() - t0
    limiter.unregister()
    sample = sample[:done]
    pts = done * cfg["nb"] ** 3
    return {"value": pts / t, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": "%d seeded blocks of the %s grid (%d^3 points each): 3 x (substitution + "
                      "ghost + RHS) + 1 detail transform per block, FP64 numpy, %.1f s" %
                      (len(sample), cfg["name"], cfg["nb"], t)}


def counter_traffic(workload):
    """HBM bytes per k_rhs launch from the committed hardware-counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None when
    the summary is for another workload or the kernels changed since."""
    import hashlib
    if not workload.startswith("c5_") or not os.path.exists(TRAFFIC_SUMMARY):
        return None
    kv = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "device_source_sha256"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(DEVICE_SRC, "rb").read()).hexdigest()
    if kv.get("device_source_sha256") != sha or "c5_adaptive_l3-9_nb24_w62_fd6_f32_eps3e-06" != workload:
        return None
    return float(kv["traffic_bytes_per_launch"])


def calibrate_copy(mib=2048, reps=3):
    """A plain device copy of known size (torch's elementwise copy kernel),
    run under the same hardware counters as the path so that the counters'
    bytes can be scaled to true HBM bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps,
                      "copy_ms": ms, "copy_gbs": 8 * n / (ms * 1e-3) / 1e9}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--eps-refine", type=float, default=None)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 2 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the whole octree on a single "
              "MI355X and has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    cfg = getattr(wl, args.config)(**({"eps_refine": args.eps_refine} if args.eps_refine else {}))
    log("config", cfg["name"])
    g = make_grid(cfg)
    n_blocks = g.n_blocks()
    ts = g.tree_stats()
    log("grid: %d leaves, levels %d..%d, %.3g points" %
        (n_blocks, ts[4], ts[3], n_blocks * cfg["nb"] ** 3))
    log("ghost work per stage fill: %d values, %d c->f / substitution items (%d substitution), "
        "%d f->c items, patch storage %d values" % (ts[1], ts[5], ts[2], ts[6], ts[9]))

    # -- headline: batched path, per-kernel HIP events around the launches
    g.prof_enable(True)
    t, points, _, _ = timed_steps(g, cfg, args.steps, args.warmup)
    value = points / t
    ms = 1e3 * t / args.steps
    log("batched %s: %.3f ms/step, %.4g points/s" % (cfg["prec"], ms, value))
    rhs_ms, rhs_n, rhs_pts = g.prof_read("rhs")
    det_ms, det_n, det_pts = g.prof_read("details")
    gr_ms, gr_n, _ = g.prof_read("ghost_refine")
    gx_ms, gx_n, _ = g.prof_read("ghost_restrict")
    g.prof_enable(False)
    esz = 4 if cfg["prec"] == "f32" else 8
    # algorithmic words per point of the three RK stages: (2 + 3 + 3)
    rhs_bytes = (2 + 3 + 3) / 3.0 * esz * rhs_pts * rhs_n
    achieved = rhs_bytes / (rhs_ms * 1e-3) / 1e9 if rhs_ms > 0 else 0.0
    det_gbs = esz * det_pts * det_n / (det_ms * 1e-3) / 1e9 if det_ms > 0 else 0.0
    step_bytes = 9 * esz * n_blocks * cfg["nb"] ** 3
    step_frac = step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    breakdown = {k: round(v / args.steps, 4) for k, v in
                 (("rhs_ms", rhs_ms), ("details_ms", det_ms), ("ghost_refine_ms", gr_ms),
                  ("ghost_restrict_ms", gx_ms))}

    # -- the fused entry point (detail pass + RK3 step sharing one ghost
    # reconstruction), same grid; reported beside the headline
    extra = {}
    tf, pf = timed_fused(g, cfg, args.steps, args.warmup)
    extra["fused_points_per_s"] = pf / tf
    extra["fused_ms_per_step"] = 1e3 * tf / args.steps
    log("fused details + rk3 step: %.3f ms/step, %.4g points/s" %
        (extra["fused_ms_per_step"], extra["fused_points_per_s"]))

    # -- adaptation amortised (second loop, same grid)
    if cfg.get("adapt_every"):
        g.prof_enable(False)   # clears the host phase timers
        ta_t, ta_pts, t_adapt, n_adapt = timed_steps(g, cfg, max(args.steps, cfg["adapt_every"]),
                                                     0, adapt_every=cfg["adapt_every"])
        extra["with_adapt_points_per_s"] = ta_pts / ta_t
        extra["adapt_ms_each"] = 1e3 * t_adapt / max(1, n_adapt)
        extra["adapt_every"] = cfg["adapt_every"]
        extra["adapt_phase_ms"] = {k: round(g.prof_read(k)[0] / max(1, n_adapt), 2) for k in
                                   ("adapt_criterion", "adapt_plan", "adapt_apply", "tree_commit")}
        log("with adapt every %d: %.4g points/s, %.1f ms per adaptation, %d leaves; phases %s" %
            (cfg["adapt_every"], extra["with_adapt_points_per_s"], extra["adapt_ms_each"],
             g.n_blocks(), extra["adapt_phase_ms"]))

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle sample)")
        cpu = cpu_baseline(g, cfg)
        log("cpu: %.4g points/s" % cpu["value"])
    g.close()

    # -- the same steps with each RK3 step replayed as one captured hipGraph
    if not args.no_plain:
        log("fp32 hipGraph path")
        gg = make_grid(cfg, exec_mode=2)
        tg, pg, _, _ = timed_steps(gg, cfg, args.steps, args.warmup)
        extra["graph_points_per_s"] = pg / tg
        extra["graph_ms_per_step"] = 1e3 * tg / args.steps
        log("hipGraph: %.3f ms/step" % extra["graph_ms_per_step"])
        gg.close()

    # -- FP64 batched path (same kernels in FP64)
    if not args.no_plain:
        log("fp64 batched path")
        gb = make_grid(cfg, prec="f64", exec_mode=0)
        tb, pb, _, _ = timed_steps(gb, cfg, max(2, args.steps // 4), 1)
        extra["fp64_batched_points_per_s"] = pb / tb
        log("fp64 batched: %.4g points/s" % extra["fp64_batched_points_per_s"])
        gb.close()

    # -- FP64 plain path (one launch per block per operation, no graph)
    if not args.no_plain:
        log("fp64 plain path")
        gp = make_grid(cfg, prec="f64", exec_mode=1)
        tp, pp, _, _ = timed_steps(gp, cfg, args.plain_steps, 1)
        extra["fp64_plain_points_per_s"] = pp / tp
        extra["speedup_vs_fp64_plain"] = value / extra["fp64_plain_points_per_s"]
        extra["fp64_plain_leaves"] = gp.n_blocks()
        log("fp64 plain: %.4g points/s" % extra["fp64_plain_points_per_s"])
        gp.close()

    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": cfg["prec"], "data": "synthetic",
        "config": {"workload": cfg["name"], "leaves": n_blocks, "points": n_blocks * cfg["nb"] ** 3,
                   "levels": [int(ts[4]), int(ts[3])], "nb": cfg["nb"],
                   "wavelet": "%d.%d" % (cfg["N"], cfg["Nt"]), "fd_order": cfg["fd"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(cfg["name"]),
                     "kernel": "k_rhs (FD advection + SSP-RK3 stage)",
                     "bytes_per_launch": rhs_bytes / max(1, rhs_n),
                     "avg_launch_ms": rhs_ms / max(1, rhs_n)},
        "step_hbm_frac_algorithmic": step_frac,
        "details_kernel_gbs": det_gbs,
        "per_step_kernel_ms": breakdown,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
