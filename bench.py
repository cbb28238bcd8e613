"""Benchmark of the multiresolution hot path on one MI355X.

A step is one SSP-RK3 step of the whole grid (three stages, each a ghost
reconstruction -- c->f patches, substitution, f->c patches -- plus the fused
FD advection + RK combine) followed by one detail pass (wide ghost
reconstruction, FP64 forward transform, per-block norms).  The timed region
starts with the field resident in HBM and runs with no per-launch
instrumentation; a second, shorter loop with HIP events around every launch
gives the per-kernel breakdown.  Adaptation is timed in a third loop (every
`adapt_every` steps) and reported separately.

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

from paper_2112_07537_amd import autotune as at  # noqa: E402
from paper_2112_07537_amd import mr  # noqa: E402
from paper_2112_07537_amd import workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0
DEVICE_SRC = os.path.join(ROOT, "paper_2112_07537_amd", "csrc", "mr_device.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "c5_hbm_traffic.md")
METRIC = "RK3-step grid points/s (ghost+details+RHS) & % HBM peak, FP32-batched vs FP64-plain"
# kernel families of the library's timers -> kernel symbol prefixes
FAMILIES = {"rhs": "mr::k_rhs", "details": "mr::k_details", "ghost_refine": "mr::k_gview",
            "ghost_subst": "mr::k_subst", "ghost_restrict": "mr::k_restrict"}


def log(*a):
    print("[bench %.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


T0 = time.time()


def make_grid(cfg, prec=None, exec_mode=0, max_blocks=150000, tree=None, n_fields=1):
    g = mr.Grid(cfg["nb"], cfg["N"], cfg["Nt"], fd_order=cfg["fd"], level_min=cfg["level_min"],
                level_max=cfg["level_max"], prec=prec or cfg["prec"],
                eps_refine=cfg["eps_refine"], eps_coarsen=cfg["eps_coarsen"],
                exec_mode=exec_mode, max_blocks=max_blocks, n_fields=n_fields)
    if tree is not None or cfg.get("tree"):
        g.set_tree(tree if tree is not None else wl.tree_of(cfg))
        g.sample_ic(*cfg["ic"])
    else:
        st = g.init_ic(*cfg["ic"])
        log("init: %d leaves, %d refine / %d coarsen in %d adapt iterations" %
            (g.n_blocks(), st.refined, st.coarsened, st.iters))
    return g


def step_loop(g, cfg, steps, adapt_every=0):
    kind, p = wl.velocity_spec(cfg["vel"])
    vel = mr.velocity(kind, *p)
    dt = g.cfl_dt(vel, cfg["cfl"])
    t_adapt = 0.0
    n_adapt = 0
    points = 0
    g.sync()
    t0 = time.perf_counter()
    for s in range(steps):
        points += g.n_blocks() * cfg["nb"] ** 3
        g.rk3_step(dt, vel)
        g.details_async()
        if adapt_every and (s + 1) % adapt_every == 0:
            g.sync()   # the queued steps are not adaptation time
            ta = time.perf_counter()
            g.adapt()
            t_adapt += time.perf_counter() - ta
            n_adapt += 1
            dt = g.cfl_dt(vel, cfg["cfl"])
    g.sync()
    return time.perf_counter() - t0, points, t_adapt, n_adapt


def fused_loop(g, cfg, steps):
    """The same work through the fused entry point: per step the detail pass
    of the current state, then the RK3 step whose first stage reuses the
    detail pass's ghosts (three ghost reconstructions per step, not four)."""
    kind, p = wl.velocity_spec(cfg["vel"])
    vel = mr.velocity(kind, *p)
    dt = g.cfl_dt(vel, cfg["cfl"])
    points = 0
    g.sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        points += g.n_blocks() * cfg["nb"] ** 3
        g.details_rk3_step_async(dt, vel)
    g.sync()
    return time.perf_counter() - t0, points


def plain_step(g, cfg):
    """One RK3 step plus a detail pass on a plain-mode grid (one launch per
    block per operation), as three mr_stage calls (fields u, A, B: the
    SSP-RK3 stages of mr_rk3_step) and mr_details, each synchronised and
    logged: at 60k leaves in FP64 a stage takes tens of seconds."""
    kind, p = wl.velocity_spec(cfg["vel"])
    vel = mr.velocity(kind, *p)
    dt = g.cfl_dt(vel, cfg["cfl"])
    g.sync()
    t0 = time.perf_counter()
    for i, (y, out, a, b) in enumerate(((0, 1, 0.0, 1.0), (1, 2, 0.75, 0.25),
                                        (2, 0, 1.0 / 3.0, 2.0 / 3.0))):
        g.stage(y, 0, out, a, b, 1.0, dt, vel)
        g.sync()
        log("  plain stage %d done at %.1f s" % (i + 1, time.perf_counter() - t0))
    g.details()
    t = time.perf_counter() - t0
    log("  plain detail pass done at %.1f s" % t)
    return t, g.n_blocks() * cfg["nb"] ** 3


def host_info():
    model, ram_kb = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram_kb = int(line.split()[1])
                break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "cpus_available": cores,
            "ram_gib": round(ram_kb / 2 ** 20, 1) if ram_kb else None}


class LazyBlocks(dict):
    """Block dict of the oracle whose values are the initial condition
    sampled in FP64 on first use (every key is present from the start)."""

    def __init__(self, keys, ic, nb):
        super().__init__((k, None) for k in keys)
        self.ic, self.nb = ic, nb

    def __getitem__(self, key):
        v = dict.__getitem__(self, key)
        if v is None:
            L, i, j, k = key
            den = float(self.nb << L)
            ax = [(o * self.nb + np.arange(self.nb)) / den for o in (i, j, k)]
            Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
            v = self.ic(X, Y, Z)
            dict.__setitem__(self, key, v)
        return v


def oracle_worker(config, tree_file, offset, stride, budget, seed=1234):
    """One process of the CPU baseline (no GPU): the FP64 oracle's per-block
    work on the seeded block order [offset::stride] of the workload, from the
    sampled initial condition, until `budget` seconds; prints one JSON line."""
    from threadpoolctl import threadpool_limits
    from oracle import grid as og
    cfg = getattr(wl, config)()
    keys = [tuple(int(v) for v in r) for r in np.load(tree_file)]
    o = og.Grid(cfg["nb"], cfg["N"], cfg["Nt"], fd_order=cfg["fd"], level_min=cfg["level_min"],
                level_max=cfg["level_max"], eps_refine=cfg["eps_refine"],
                eps_coarsen=cfg["eps_coarsen"])
    o.blocks = LazyBlocks(keys, wl.ic_function(cfg["ic"]), cfg["nb"])
    o._index()
    order = [keys[i] for i in np.random.default_rng(seed).permutation(len(keys))]
    kind, p = wl.velocity_spec(cfg["vel"])
    vel = (kind, p)
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for k in order[offset::stride]:
            mask = o.substitution_mask(k)
            for _ in range(3):
                if mask.any():
                    for deg in (1, 2, 3):
                        z, y, x, v = o.substitution_values(k, deg, mask)
                        o.blocks[k][z, y, x] = v
                o.rhs_block(k, vel)
            o.block_details(k)
            done += 1
            if time.perf_counter() - t0 > budget:
                break
        t = time.perf_counter() - t0
    print(json.dumps({"blocks": done, "seconds": t}), flush=True)


def cpu_baseline(cfg, config, tree, budget_s=12.0, max_procs=16):
    """The FP64 oracle timed on a seeded sample of blocks of the same tree:
    per sampled block, three stages of (substitution + ghost reconstruction +
    RHS) and one detail transform, on the sampled initial condition.  Child
    processes that never touch the GPU run it: one for the one-core leg, then
    one per available core (at most 16, the GPU machine's share of the host) for
    the all-core leg, each with one numpy thread and about `budget_s` seconds
    of timed work."""
    import subprocess
    import tempfile
    info = host_info()
    nproc = max(1, min(max_procs, info["cpus_available"] or 1))
    with tempfile.TemporaryDirectory() as td:
        tf = os.path.join(td, "tree.npy")
        np.save(tf, np.array(tree, dtype=np.int64))

        def leg(n, first):
            procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                                       config, tf, str(first + i), str(n), str(budget_s)],
                                      stdout=subprocess.PIPE, text=True)
                     for i in range(n)]
            res = []
            for pr in procs:
                out, _ = pr.communicate()
                if pr.returncode != 0:
                    raise RuntimeError("oracle worker failed")
                res.append(json.loads(out.strip().splitlines()[-1]))
            return res
        r1 = leg(1, 0)[0]
        pts_blk = cfg["nb"] ** 3
        one = {"value": r1["blocks"] * pts_blk / r1["seconds"], "unit": "points/s", "cores": 1,
               "kind": "oracle",
               "sample": "%d seeded blocks of the %s tree (%d^3 points each, initial condition "
                         "sampled in FP64): 3 x (substitution + ghost + RHS) + 1 detail transform "
                         "per block, numpy on one thread, %.1f s" %
                         (r1["blocks"], cfg["name"], cfg["nb"], r1["seconds"])}
        allc = None
        if nproc > 1:
            rs = leg(nproc, 0)
            blocks = sum(r["blocks"] for r in rs)
            wall = max(r["seconds"] for r in rs)
            allc = {"value": blocks * pts_blk / wall, "unit": "points/s", "cores": nproc,
                    "kind": "oracle",
                    "sample": "%d seeded blocks over %d processes (one numpy thread each), "
                              "%.1f s" % (blocks, nproc, wall)}
    one.update({"all_cores": allc, "host": info})
    return one


def counter_traffic(workload):
    """HBM bytes per launch of each kernel, and per step, from the committed
    hardware-counter summary (FETCH_SIZE and WRITE_SIZE scaled by the copy
    calibration), or None when the summary is for another workload or the
    kernels changed since it was taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    kv = {}
    per_kernel = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line and not line.startswith("|"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
        if line.startswith("traffic_family"):
            fam, b = line.split(":", 1)[1].split()
            per_kernel[fam] = float(b)
    sha = hashlib.sha256(open(DEVICE_SRC, "rb").read()).hexdigest()
    if kv.get("device_source_sha256") != sha or kv.get("workload") != workload:
        return None
    return {"step_bytes": float(kv["traffic_bytes_per_step"]), "per_launch": per_kernel}


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


def kernel_table(g, cfg, steps, esz):
    """Per-family HIP-event timings over `steps` timed steps (events on the
    grid's stream, recording started after a warm-up step) and each family's
    algorithmic traffic per step: the 8 words per point of the three RK
    stages, the field read of the detail pass, and the values the ghost work
    lists write and read (three stencil-depth reconstructions and one wide
    one per step)."""
    ts = g.tree_stats()
    nblk = g.n_blocks()
    n_pts = nblk * cfg["nb"] ** 3
    per_step = {"rhs": 8.0 * esz * n_pts,
                "details": 1.0 * esz * n_pts + 27 * 8 * nblk,
                "ghost_refine": esz * (3.0 * (ts[10] + ts[11]) + ts[16] + ts[17]),
                "ghost_subst": esz * (3.0 * (ts[12] + ts[13]) + ts[18] + ts[19]),
                "ghost_restrict": esz * (3.0 * (ts[14] + ts[15]) + ts[20] + ts[21])}
    out = {}
    for fam in FAMILIES:
        ms, n, _ = g.prof_read(fam)
        if n == 0:
            continue
        mps = ms / steps
        gbs = per_step[fam] / (mps * 1e-3) / 1e9
        out[fam] = {"ms_per_step": round(mps, 4), "launches_per_step": n / steps,
                    "avg_launch_ms": round(ms / n, 4), "bytes_per_step": per_step[fam],
                    "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-adapt", action="store_true",
                    help="skip the adaptation leg (every other leg runs on the benchmark tree)")
    ap.add_argument("--breakdown-steps", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 2 GiB device copy (counter calibration)")
    ap.add_argument("--oracle-worker", nargs=5, metavar=("CONFIG", "TREE", "OFFSET", "STRIDE",
                                                         "BUDGET"),
                    help="internal: one process of the CPU baseline")
    args = ap.parse_args()
    if args.oracle_worker:
        c, tf, off, st, bud = args.oracle_worker
        oracle_worker(c, tf, int(off), int(st), float(bud))
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the whole octree on a single "
              "MI355X and has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    cfg = getattr(wl, args.config)()
    log("config", cfg["name"])
    g = make_grid(cfg)
    # launch-shape knobs from the autotuner's cache, if it has this
    # configuration: time the defaults first, for the gain
    arch = at.gpu_arch()
    entry = at.load().get(at.cache_key(arch, cfg))
    tuning = {"arch": arch, "knobs": g.get_tuning(), "source": "defaults"}
    if entry:
        step_loop(g, cfg, args.warmup)
        td, pd, _, _ = step_loop(g, cfg, args.steps)
        tuning["ms_per_step_defaults"] = 1e3 * td / args.steps
        g.set_tuning(**entry["knobs"])
        tuning.update(knobs=g.get_tuning(), source="paper_2112_07537_amd/tuning.json")
        log("defaults: %.3f ms/step; tuned knobs %s" % (tuning["ms_per_step_defaults"],
                                                        tuning["knobs"]))
    n_blocks = g.n_blocks()
    n_pts = n_blocks * cfg["nb"] ** 3
    ts = g.tree_stats()
    tree = [tuple(int(v) for v in m) for m in g.block_meta()]
    log("grid: %d leaves, levels %d..%d, %.4g points" % (n_blocks, ts[4], ts[3], n_pts))
    log("ghost work per stage reconstruction: %d c->f items, %d substitution items, "
        "%d f->c items, %d ghost values, patch storage %d values" %
        (ts[5], ts[2], ts[6], ts[1], ts[9]))
    esz = 4 if cfg["prec"] == "f32" else 8

    # -- headline: batched path, no per-launch instrumentation
    step_loop(g, cfg, args.warmup)
    t, points, _, _ = step_loop(g, cfg, args.steps)
    value = points / t
    ms = 1e3 * t / args.steps
    log("batched %s: %.3f ms/step, %.4g points/s" % (cfg["prec"], ms, value))
    if "ms_per_step_defaults" in tuning:
        tuning["gain_vs_defaults"] = tuning["ms_per_step_defaults"] / ms

    # -- per-kernel breakdown: HIP events around every launch, recording
    # started after a warm-up step
    step_loop(g, cfg, 1)
    g.prof_enable(True)
    tb, _, _, _ = step_loop(g, cfg, args.breakdown_steps)
    kernels = kernel_table(g, cfg, args.breakdown_steps, esz)
    g.prof_enable(False)
    ms_instr = 1e3 * tb / args.breakdown_steps
    log("instrumented: %.3f ms/step; %s" %
        (ms_instr, {k: v["ms_per_step"] for k, v in kernels.items()}))

    # -- the fused entry point (detail pass + RK3 step sharing one ghost
    # reconstruction), same grid; reported beside the headline
    extra = {}
    fused_loop(g, cfg, args.warmup)
    tf, pf = fused_loop(g, cfg, args.steps)
    extra["fused_points_per_s"] = pf / tf
    extra["fused_ms_per_step"] = 1e3 * tf / args.steps
    log("fused details + rk3 step: %.3f ms/step, %.4g points/s" %
        (extra["fused_ms_per_step"], extra["fused_points_per_s"]))

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle sample)")
        cpu = cpu_baseline(cfg, args.config, tree)
        log("cpu: %.4g points/s one core; all cores %s" %
            (cpu["value"], cpu["all_cores"] and "%.4g" % cpu["all_cores"]["value"]))

    # -- adaptation amortised (third loop, same grid, changes the tree)
    if cfg.get("adapt_every") and not args.no_adapt:
        g.prof_enable(False)   # clears the host phase timers
        ta_t, ta_pts, t_adapt, n_adapt = step_loop(g, cfg, max(args.steps, cfg["adapt_every"]),
                                                   adapt_every=cfg["adapt_every"])
        extra["with_adapt_points_per_s"] = ta_pts / ta_t
        extra["adapt_ms_each"] = 1e3 * t_adapt / max(1, n_adapt)
        extra["adapt_every"] = cfg["adapt_every"]
        extra["adapt_leaves_after"] = g.n_blocks()
        extra["adapt_phase_ms"] = {k: round(g.prof_read(k)[0] / max(1, n_adapt), 2) for k in
                                   ("adapt_criterion", "adapt_plan", "adapt_apply", "tree_commit")}
        log("with adapt every %d: %.4g points/s, %.1f ms per adaptation, %d -> %d leaves; "
            "phases %s" % (cfg["adapt_every"], extra["with_adapt_points_per_s"],
                           extra["adapt_ms_each"], n_blocks, g.n_blocks(),
                           extra["adapt_phase_ms"]))
    g.close()

    if not args.no_plain:
        # -- the same steps with each RK3 step replayed as one captured hipGraph
        log("fp32 hipGraph path")
        gg = make_grid(cfg, exec_mode=2, tree=tree)
        gg.set_tuning(**tuning["knobs"])
        step_loop(gg, cfg, args.warmup)
        tg, pg, _, _ = step_loop(gg, cfg, args.steps)
        extra["graph_points_per_s"] = pg / tg
        extra["graph_ms_per_step"] = 1e3 * tg / args.steps
        log("hipGraph: %.3f ms/step" % extra["graph_ms_per_step"])
        gg.close()
        # -- FP64 batched path (same kernels in FP64, same tree)
        log("fp64 batched path")
        gb = make_grid(cfg, prec="f64", exec_mode=0, tree=tree)
        e64 = at.load().get(at.cache_key(arch, cfg, "f64"))
        if e64:
            gb.set_tuning(**e64["knobs"])
        step_loop(gb, cfg, 1)
        tb64, pb, _, _ = step_loop(gb, cfg, max(2, args.steps // 4))
        extra["fp64_batched_points_per_s"] = pb / tb64
        log("fp64 batched: %.4g points/s" % extra["fp64_batched_points_per_s"])
        gb.close()
        # -- FP64 plain path (one launch per block per operation, no graph)
        log("fp64 plain path")
        gp = make_grid(cfg, prec="f64", exec_mode=1, tree=tree, n_fields=3)
        tp, pp = plain_step(gp, cfg)
        extra["fp64_plain_points_per_s"] = pp / tp
        extra["speedup_vs_fp64_plain"] = value / extra["fp64_plain_points_per_s"]
        log("fp64 plain: %.4g points/s" % extra["fp64_plain_points_per_s"])
        gp.close()

    # roofline of the step (section 8(d) of the plan this build follows:
    # 9 words per point per step move through HBM at the least)
    step_bytes = 9 * esz * n_pts
    achieved = step_bytes / (ms * 1e-3) / 1e9
    traffic = counter_traffic(cfg["name"])
    dom = max(kernels.items(), key=lambda kv: kv[1]["ms_per_step"]) if kernels else (None, None)
    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": cfg["prec"], "data": "synthetic",
        "config": {"workload": cfg["name"], "leaves": n_blocks, "points": n_pts,
                   "levels": [int(ts[4]), int(ts[3])], "nb": cfg["nb"],
                   "wavelet": "%d.%d" % (cfg["N"], cfg["Nt"]), "fd_order": cfg["fd"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["step_bytes"] if traffic else None,
                     "kernel": "whole step: 3 x (c->f, substitution, f->c, FD + RK3 stage) + "
                               "detail pass; 9 words per point",
                     "bytes_per_step": step_bytes,
                     "dominant_kernel": dom[0],
                     "dominant_kernel_ms_per_step": dom[1]["ms_per_step"] if dom[1] else None,
                     # the same roofline for the dominant kernel alone: its
                     # algorithmic bytes per launch over its average launch
                     # duration (HIP events on the grid's stream); traffic
                     # from the counter summary when it matches the source
                     "dominant": None if not dom[1] else {
                         "kernel": dom[0], "bound": "hbm",
                         "avg_launch_ms": dom[1]["avg_launch_ms"],
                         "bytes_per_launch": dom[1]["bytes_per_step"] / dom[1]["launches_per_step"],
                         "achieved": dom[1]["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": dom[1]["frac"],
                         "traffic": (traffic["per_launch"].get(dom[0]) if traffic else None)}},
        "kernels": kernels,
        "tuning": tuning,
        "instrumented_ms_per_step": ms_instr,
        "cpu_baseline": cpu,
    }
    if traffic:
        for fam, b in traffic["per_launch"].items():
            if fam in kernels:
                kernels[fam]["counter_bytes_per_launch"] = b
                kernels[fam]["counter_frac"] = round(
                    b / (kernels[fam]["avg_launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
