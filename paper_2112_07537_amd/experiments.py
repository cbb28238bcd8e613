"""The validation experiments of section 4, run on the GPU through the C ABI.

* Epsilon test (section 4.1): a Gaussian sampled on the uniform finest
  level, coarsened with the block adaptation at threshold eps_c until no
  block changes, then refined back to the finest level by zero-detail
  refinement; E_inf is the largest distance to the samples of the finest
  level, and the block count after coarsening measures the compression.
* Moment conservation (section 4.2): the discrete moments M_0 and M_1 of
  the scaling coefficients on the finest level, of the samples and of the
  compressed field refined back (refinement keeps the moments of the
  represented field).
* Two-level convergence (section 4.3): a uniform level with one eighth of
  the domain coarsened one level (jumps across faces, edges and corners),
  ghost reconstruction, then the right-hand side (advection CONS-3 / CONS-5
  or central FD, or the DIFF-2 / DIFF-4 Laplacian) on the whole grid
  against the analytic operator applied to the Gaussian.

Geometry: the paper's domain is the cube [0, 2]^3 made of eight trees, the
Gaussian exp(-r^2 / sigma^2) with sigma = 2/15 at its centre, N_b = 24 and
L_max = 5 in every tree.  Here the domain is the periodic unit cube, whose
level l + 1 has the resolution of the paper's level l: the same grids,
scaled by 1/2 (sigma = 1/15, the finest level 6; the Gaussian is below
1e-73 at the periodic boundary).  Values are reported in the paper's
units: E_inf is scale free; moments scale by the volume (M_0 by 8) and one
more factor 2 for M_1; derivatives d/dx of the paper are half of those
here, so the advection velocity (1, 1, 1) of the paper is (1/2, 1/2, 1/2)
here, the unit Laplacian of the paper is nu = 1/4 here, and h_f is twice
the unit-cube spacing.

Command line (JSON lines on stdout, one per run)::

    python -m paper_2112_07537_amd.experiments epsilon --wavelets 4.2 --lmax 6
    python -m paper_2112_07537_amd.experiments twolevel --wavelets 4.2 --fd 3 --diff 2,4
    python -m paper_2112_07537_amd.experiments report RESULTS.jsonl FIGURES.txt
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import mr

SIGMA = 1.0 / 15.0
CENTRE = (0.5, 0.5, 0.5)
EPS_LIST = (1.0, 1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10)
WAVELETS = ("2.0", "2.2", "4.0", "4.2", "6.0", "6.2")


def gauss_ic(sigma=SIGMA, centre=CENTRE):
    return "gauss", np.array([[centre[0], centre[1], centre[2], sigma, 1.0]])


def uniform_keys(L):
    n = 1 << L
    return [(L, i, j, k) for k in range(n) for j in range(n) for i in range(n)]


def parse_wavelet(w):
    N, Nt = w.split(".")
    return int(N), int(Nt)


def epsilon_test(wavelet, eps_list=EPS_LIST, lmax=6, lmin=1, nb=24, log=None):
    """Epsilon and moment tests for one wavelet; yields one record per eps_c.
    The grid is FP64; its capacity is the uniform finest level."""
    N, Nt = parse_wavelet(wavelet)
    kind, par = gauss_ic()
    g = mr.Grid(nb, N, Nt, fd_order=4, level_min=lmin, level_max=lmax, prec="f64",
                eps_refine=1.0, eps_coarsen=1e-6, max_blocks=8 ** lmax)
    full = uniform_keys(lmax)
    try:
        for eps in eps_list:
            t0 = time.perf_counter()
            g.set_tree(full)
            g.sample_ic(kind, par)
            m_fine = g.moments()
            # coarsening only: no block reaches the refinement threshold
            g.set_thresholds(1e300, eps)
            st_c = g.adapt(max_iter=4 * (lmax - lmin) + 4)
            meta = g.block_meta()
            nblk = int(len(meta))
            hist = np.bincount(meta[:, 0], minlength=lmax + 1)[lmin:].tolist()
            m_coarse = g.moments()
            # zero-detail refinement of every block back to the finest level
            g.set_thresholds(1e-300, 0.0)
            st_r = g.adapt(max_iter=4 * (lmax - lmin) + 4)
            if g.n_blocks() != 8 ** lmax:
                raise RuntimeError("refinement back to level %d left %d blocks" % (lmax, g.n_blocks()))
            einf, el2 = g.ic_error(kind, par)
            m_back = g.moments()
            # moments of section 4.2: both fields on the uniform finest level
            dm = m_fine - m_back
            # the plain sums h^3 phi over the leaves of the compressed grid
            # (not the moments of the represented field near level jumps)
            dmix = m_fine - m_coarse
            rec = dict(experiment="epsilon", wavelet=wavelet, eps=eps, lmax=lmax, nb=nb,
                       n_blocks=nblk, levels=hist, coarsen_iters=int(st_c.iters),
                       refine_iters=int(st_r.iters), e_inf=einf, e_l2=el2,
                       m0=abs(dm[0]) * 8.0, m1=float(np.linalg.norm(dm[1:])) * 16.0,
                       m0_leaf_sum=abs(dmix[0]) * 8.0,
                       m1_leaf_sum=float(np.linalg.norm(dmix[1:])) * 16.0,
                       m0_value=m_fine[0] * 8.0, seconds=time.perf_counter() - t0)
            if log:
                log(rec)
            yield rec
    finally:
        g.close()


def two_level_tree_flags(meta, L):
    """-1 for the blocks of the octant [0, 1/2)^3 (coarsened one level)."""
    half = 1 << (L - 1)
    sel = (meta[:, 1] < half) & (meta[:, 2] < half) & (meta[:, 3] < half)
    return np.where(sel, -1, 0).astype(np.int8)


def advection_exact(meta, nb, u, sigma=SIGMA, centre=CENTRE, chunk=1024):
    """-(u . grad) f of the Gaussian at every point of the leaves, per block
    (generator of (block range, values))."""
    idx = np.arange(nb, dtype=np.float64)
    for b0 in range(0, len(meta), chunk):
        m = meta[b0:b0 + chunk]
        den = (nb * (1 << m[:, 0].astype(np.int64))).astype(np.float64)
        x = (m[:, 1:2] * nb + idx[None, :]) / den[:, None]
        y = (m[:, 2:3] * nb + idx[None, :]) / den[:, None]
        z = (m[:, 3:4] * nb + idx[None, :]) / den[:, None]
        dx, dy, dz = x - centre[0], y - centre[1], z - centre[2]
        dx -= np.round(dx)
        dy -= np.round(dy)
        dz -= np.round(dz)
        X = dx[:, None, None, :]
        Y = dy[:, None, :, None]
        Z = dz[:, :, None, None]
        f = np.exp(-(X * X + Y * Y + Z * Z) / sigma ** 2)
        # grad f = -2 (x - c) / sigma^2 f
        yield b0, (2.0 / sigma ** 2) * (u[0] * X + u[1] * Y + u[2] * Z) * f


def laplacian_exact(meta, nb, nu, sigma=SIGMA, centre=CENTRE, chunk=1024):
    """nu * laplacian(f) of the Gaussian at every point of the leaves, per
    block (generator of (block range, values))."""
    idx = np.arange(nb, dtype=np.float64)
    for b0 in range(0, len(meta), chunk):
        m = meta[b0:b0 + chunk]
        den = (nb * (1 << m[:, 0].astype(np.int64))).astype(np.float64)
        d = []
        for a, c in zip((1, 2, 3), centre):
            t = (m[:, a:a + 1] * nb + idx[None, :]) / den[:, None] - c
            d.append(t - np.round(t))
        X = d[0][:, None, None, :]
        Y = d[1][:, None, :, None]
        Z = d[2][:, :, None, None]
        r2 = X * X + Y * Y + Z * Z
        f = np.exp(-r2 / sigma ** 2)
        yield b0, nu * (4.0 * r2 / sigma ** 4 - 6.0 / sigma ** 2) * f


def two_level(wavelet, fd, levels=(2, 3, 4, 5), nb=24, u=(0.5, 0.5, 0.5), log=None,
              diffusion=False):
    """Two-level convergence for one wavelet and scheme (fd_order 3 / 5:
    CONS-3 / CONS-5; 4 / 6: central FD advection; with diffusion=True,
    fd_order 2 / 4: DIFF-2 / DIFF-4, nu = 1/4, the paper's unit Laplacian).
    Yields one record per fine level."""
    N, Nt = parse_wavelet(wavelet)
    kind, par = gauss_ic()
    for L in levels:
        t0 = time.perf_counter()
        g = mr.Grid(nb, N, Nt, fd_order=fd, level_min=L - 1, level_max=L, prec="f64",
                    eps_refine=1.0, eps_coarsen=1e-6, n_fields=2, max_blocks=8 ** L)
        try:
            g.set_tree(uniform_keys(L))
            g.sample_ic(kind, par)
            st = g.adapt_flags(two_level_tree_flags(g.block_meta(), L))
            if st.coarsened != 8 ** (L - 1) // 8:
                raise RuntimeError("octant coarsening: %d sibling sets" % st.coarsened)
            nu = 0.25
            g.rhs(0, 1, mr.velocity("diffusion", nu) if diffusion else mr.velocity("const", *u))
            meta = g.block_meta()
            out = g.field_get(1)
            einf = 0.0
            exact = laplacian_exact(meta, nb, nu) if diffusion else advection_exact(meta, nb, u)
            for b0, ref in exact:
                einf = max(einf, float(np.abs(out[b0:b0 + len(ref)] - ref).max()))
            rec = dict(experiment="twolevel", wavelet=wavelet, fd=fd, level=L, nb=nb,
                       op="diff" if diffusion else "adv",
                       h_f=2.0 / (nb << L), n_blocks=int(len(meta)), e_inf=einf,
                       seconds=time.perf_counter() - t0)
        finally:
            g.close()
        if log:
            log(rec)
        yield rec


# ------------------------------------------------------------------ report
def read_figures(path):
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        s, w, x, y = line.split()
        out.setdefault((s, w), []).append((float(x), float(y)))
    return out


def report(results, figures):
    """Markdown tables of the GPU results beside the paper's figure data."""
    res = [json.loads(l) for l in open(results) if l.strip().startswith("{")]
    fig = read_figures(figures)
    lines = []
    eps_rows = [r for r in res if r["experiment"] == "epsilon"]
    if eps_rows:
        lines += ["## Epsilon test and moments (sections 4.1, 4.2)", "",
                  "| wavelet | eps_c | E_inf | paper E_inf | E_inf/eps_c | blocks | paper blocks"
                  " | M0 diff | paper M0 | M1 diff | paper M1 | s |",
                  "|---|---|---|---|---|---|---|---|---|---|---|---|"]
        for r in eps_rows:
            w, e = r["wavelet"], r["eps"]

            def pv(series):
                for x, y in fig.get((series, w), []):
                    if abs(x - e) <= 1e-9 * e:
                        return "%.3g" % y
                return "-"
            lines.append("| %s | %.0e | %.3e | %s | %.2f | %d | %s | %.2e | %s | %.2e | %s | %.1f |" % (
                w, e, r["e_inf"], pv("e1_einf"), r["e_inf"] / e, r["n_blocks"], pv("e1_nblocks"),
                r["m0"], pv("e2_m0"), r["m1"], pv("e2_m1"), r["seconds"]))
        lines.append("")
    tl = [r for r in res if r["experiment"] == "twolevel"]
    if tl:
        lines += ["## Two-level convergence (section 4.3)", "",
                  "| scheme | wavelet | h_f (paper units) | blocks | E_inf | paper E_inf | order |"
                  " paper order |", "|---|---|---|---|---|---|---|---|"]
        def name(r):
            if r.get("op") == "diff":
                return "diff%d" % r["fd"]
            return {3: "cons3", 5: "cons5", 4: "fd4", 6: "fd6"}[r["fd"]]
        for key in sorted({(name(r), r["wavelet"]) for r in tl}):
            rows = sorted([r for r in tl if (name(r), r["wavelet"]) == key], key=lambda r: r["level"])
            paper = sorted(set(fig.get(("e3_" + key[0], key[1]), [])), reverse=True)
            prev = pprev = None
            for i, r in enumerate(rows):
                pe = [y for x, y in paper if abs(x - r["h_f"]) <= 1e-6 * r["h_f"]]
                pe = pe[0] if pe else None
                order = math.log2(prev / r["e_inf"]) if prev else None
                porder = math.log2(pprev / pe) if (pprev and pe) else None
                lines.append("| %s | %s | %.6f | %d | %.3e | %s | %s | %s |" % (
                    key[0], key[1], r["h_f"], r["n_blocks"], r["e_inf"],
                    "%.3e" % pe if pe else "-", "%.2f" % order if order else "-",
                    "%.2f" % porder if porder else "-"))
                prev, pprev = r["e_inf"], pe
        lines.append("")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("epsilon")
    a.add_argument("--wavelets", default=",".join(WAVELETS))
    a.add_argument("--lmax", type=int, default=6)
    a.add_argument("--eps", default=None, help="comma-separated eps_c values")
    b = sub.add_parser("twolevel")
    b.add_argument("--wavelets", default=",".join(WAVELETS))
    b.add_argument("--fd", default="3,5")
    b.add_argument("--diff", default="", help="DIFF orders, e.g. 2,4")
    b.add_argument("--levels", default="2,3,4,5")
    c = sub.add_parser("report")
    c.add_argument("results")
    c.add_argument("figures")
    args = ap.parse_args(argv)

    def emit(rec):
        print(json.dumps(rec), flush=True)
    if args.cmd == "epsilon":
        eps = tuple(float(e) for e in args.eps.split(",")) if args.eps else EPS_LIST
        for w in args.wavelets.split(","):
            for _ in epsilon_test(w, eps, lmax=args.lmax, log=emit):
                pass
    elif args.cmd == "twolevel":
        lv = tuple(int(v) for v in args.levels.split(","))
        for fd in (int(v) for v in args.fd.split(",") if v):
            for w in args.wavelets.split(","):
                for _ in two_level(w, fd, lv, log=emit):
                    pass
        for fd in (int(v) for v in args.diff.split(",") if v):
            for w in args.wavelets.split(","):
                for _ in two_level(w, fd, lv, log=emit, diffusion=True):
                    pass
    else:
        print(report(args.results, args.figures))
    return 0


if __name__ == "__main__":
    sys.exit(main())
