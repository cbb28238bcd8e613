"""Autotuner of the ghost kernels' launch shapes (mr_tuning).

The knobs are the LDS budgets that c->f, f->c and substitution work items
are tiled to, and the substitution workgroup size.  The tuner times whole
steps of a workload (one SSP-RK3 step and one detail pass each, as the
benchmark does) on a GPU grid for candidate values of one knob at a time,
keeps the fastest, and sweeps the knobs twice (coordinate descent).  The
result is cached in a JSON file keyed by (GPU architecture, block size,
wavelet N.Nt, right-hand side, precision); `apply` sets a cached entry on a
grid.  Results do not depend on the knobs beyond the rounding order of f->c
sums.

Command line::

    python -m paper_2112_07537_amd.autotune --config c5 [--config c4 ...]
"""
import argparse
import json
import os
import sys
import time

from . import mr
from . import workloads as wl

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

CANDIDATES = {
    # substitution budgets at the workgroup counts per CU that 160 KiB of LDS
    # allows (6, 5, 4, 3 and 2 with the kernel's static tables), plus 61440
    "lds_subst": [24320, 29696, 37888, 51200, 61440, 65536],
    "lds_refine": [12288, 16384, 20480, 24576, 32768],
    "lds_restrict": [16384, 20480, 24576, 32768, 40960],
    "subst_threads": [256, 512],
}
DEFAULTS = {"lds_refine": 20480, "lds_restrict": 24576, "lds_subst": 37888, "subst_threads": 512}


def gpu_arch():
    """Architecture name of the current device (mr_device_arch)."""
    return mr.device_arch()


def cache_key(arch, cfg, prec=None):
    return "%s/nb%d/w%d.%d/fd%d/%s" % (arch, cfg["nb"], cfg["N"], cfg["Nt"], cfg["fd"],
                                       prec or cfg["prec"])


def load(path=CACHE):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(entries, path=CACHE):
    with open(path + ".tmp", "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(path + ".tmp", path)


def apply(g, cfg, path=CACHE, arch=None):
    """Set the cached knobs of this configuration on grid g; returns the cache
    entry, or None (defaults kept) when there is none."""
    entry = load(path).get(cache_key(arch or gpu_arch(), cfg))
    if entry:
        g.set_tuning(**entry["knobs"])
    return entry


def step_time(g, vel, dt, steps=4, repeats=3):
    """Fastest of `repeats` timings of `steps` steps (RK3 step + detail pass),
    after one warm-up step; ms per step."""
    g.rk3_step(dt, vel)
    g.details_async()
    g.sync()
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        for _ in range(steps):
            g.rk3_step(dt, vel)
            g.details_async()
        g.sync()
        best = min(best, (time.perf_counter() - t0) / steps)
    return 1e3 * best


def tune(g, cfg, sweeps=2, log=None):
    """Coordinate descent over CANDIDATES on grid g (its tree and field are
    advanced by the timed steps).  Returns (knobs, ms_default, ms_best,
    trials)."""
    kind, p = wl.velocity_spec(cfg["vel"])
    vel = mr.velocity(kind, *p)
    dt = g.cfl_dt(vel, cfg["cfl"])
    cur = dict(DEFAULTS)
    g.set_tuning(**cur)
    ms_default = step_time(g, vel, dt)
    best_ms = ms_default
    trials = [dict(cur, ms=ms_default)]
    if log:
        log("defaults %s: %.3f ms/step" % (cur, ms_default))
    for sweep in range(sweeps):
        changed = False
        for k, values in CANDIDATES.items():
            for v in values:
                if v == cur[k]:
                    continue
                trial = dict(cur, **{k: v})
                g.set_tuning(**trial)
                ms = step_time(g, vel, dt)
                trials.append(dict(trial, ms=ms))
                if log:
                    log("  %s=%d: %.3f ms/step" % (k, v, ms))
                if ms < best_ms * 0.995:
                    best_ms, cur, changed = ms, trial, True
            g.set_tuning(**cur)
        # re-time the incumbent: the steps change the field, and timings drift
        best_ms = step_time(g, vel, dt)
        if log:
            log("sweep %d: %s, %.3f ms/step" % (sweep + 1, cur, best_ms))
        if not changed:
            break
    return cur, ms_default, best_ms, trials


def build(cfg):
    g = mr.Grid(cfg["nb"], cfg["N"], cfg["Nt"], fd_order=cfg["fd"], level_min=cfg["level_min"],
                level_max=cfg["level_max"], prec=cfg["prec"], eps_refine=cfg["eps_refine"],
                eps_coarsen=cfg["eps_coarsen"], max_blocks=150000)
    if cfg.get("tree"):
        g.set_tree(wl.tree_of(cfg))
        g.sample_ic(*cfg["ic"])
    else:
        g.init_ic(*cfg["ic"])
    return g


def main(argv=None):
    ap = argparse.ArgumentParser(description="autotune the ghost kernels' launch shapes")
    ap.add_argument("--config", action="append", default=None)
    ap.add_argument("--cache", default=CACHE)
    ap.add_argument("--sweeps", type=int, default=2)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)
    arch = gpu_arch()
    entries = load(args.cache)
    for name in args.config or ["c5"]:
        cfg = getattr(wl, name)()
        g = build(cfg)
        log("%s: %d leaves" % (cfg["name"], g.n_blocks()))
        knobs, ms0, ms1, trials = tune(g, cfg, sweeps=args.sweeps, log=log)
        g.close()
        key = cache_key(arch, cfg)
        entries[key] = {"knobs": knobs, "workload": cfg["name"], "ms_per_step_default": ms0,
                        "ms_per_step_tuned": ms1, "gain": ms0 / ms1, "trials": len(trials)}
        print(json.dumps({"key": key, **entries[key]}), flush=True)
        save(entries, args.cache)
    return 0


if __name__ == "__main__":
    sys.exit(main())
