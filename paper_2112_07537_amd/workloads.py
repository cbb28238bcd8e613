"""Seeded synthetic workloads (inputs only; no wavelet or stencil arithmetic).

Both the HIP path and the CPU oracle read their inputs from here: initial
condition parameters drawn from a SplitMix64 stream, velocity fields, block
sizes, thresholds, and the prescribed geometric tree of the batching workload.
The paper's own test problems are analytic fields (compact Gaussians, tanh
interfaces), so every workload is synthetic by construction.
"""
import math

import numpy as np

MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood 2014)."""

    def __init__(self, seed):
        self.s = seed & MASK

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & MASK
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    def uniform(self, lo=0.0, hi=1.0):
        return lo + (hi - lo) * ((self.next() >> 11) * (1.0 / (1 << 53)))


def gauss_params(centres, sigmas, amps):
    """Rows (cx, cy, cz, sigma, a) of a Gaussian-sum initial condition."""
    return np.array([[c[0], c[1], c[2], s, a] for c, s, a in zip(centres, sigmas, amps)],
                    dtype=np.float64)


# ------------------------------------------------------------------ configs
def c1():
    """Uniform level 1 (8 blocks of 16^3), 4.0, FD4, FP64, one Gaussian."""
    return dict(name="c1_uniform_l1_nb16_w40_fd4_f64", nb=16, N=4, Nt=0, fd=4,
                level_min=1, level_max=1, prec="f64", eps_refine=1e-2, eps_coarsen=1e-4,
                ic=("gauss", gauss_params([(0.5, 0.5, 0.5)], [0.1], [1.0])),
                vel=("const", (1.0, 0.5, 0.25)), cfl=0.5, steps=1, adapt_every=0)


def c2(seed=2):
    """Adaptive levels 2..5, 16^3 blocks, 4.2, FD4, FP64, Gaussian sigma 0.05
    at a seeded centre, constant velocity, adapt every step."""
    r = SplitMix64(seed)
    c = tuple(r.uniform(0.3, 0.7) for _ in range(3))
    return dict(name="c2_adaptive_l2-5_nb16_w42_fd4_f64", nb=16, N=4, Nt=2, fd=4,
                level_min=2, level_max=5, prec="f64", eps_refine=1e-2, eps_coarsen=1e-4,
                ic=("gauss", gauss_params([c], [0.05], [1.0])),
                vel=("const", (1.0, 0.5, 0.25)), cfl=0.5, steps=20, adapt_every=1)


def c3(seed=3):
    """Levels 3..7, 24^3 blocks, 6.2, FD6, sum of 8 Gaussians, rotating
    velocity; thresholds 1e-4 / 1e-6."""
    r = SplitMix64(seed)
    cs, ss, aa = [], [], []
    for _ in range(8):
        cs.append(tuple(r.uniform(0.25, 0.75) for _ in range(3)))
        ss.append(r.uniform(0.02, 0.08))
        aa.append(r.uniform(0.5, 1.0))
    return dict(name="c3_adaptive_l3-7_nb24_w62_fd6", nb=24, N=6, Nt=2, fd=6,
                level_min=3, level_max=7, prec="f32", eps_refine=1e-4, eps_coarsen=1e-6,
                ic=("gauss", gauss_params(cs, ss, aa)),
                vel=("rotating", (0.5, 0.5, 0.2)), cfl=0.5, steps=50, adapt_every=10)


def shell_rho(x, y, z, a=(0.20, 0.15, 0.10)):
    return np.sqrt(((x - 0.5) / a[0]) ** 2 + ((y - 0.5) / a[1]) ** 2 + ((z - 0.5) / a[2]) ** 2)


def geometric_tree(lmin=2, lmax=8, band=0.5, a=(0.20, 0.15, 0.10), focus=(0.7, 0.5, 0.5),
                   r0=0.5, q=1.4):
    """Leaves refined toward the ellipsoid rho = 1 inside a window that
    shrinks with level: a block at level L < lmax is split when the band
    |(rho - 1) min(a)| < band * 2^-L and the ball of radius r0 / q^(L-lmin)
    around the focus point (on the ellipsoid) both reach it (tested at the
    block's 27 corner / edge / centre points).  Then the tree is 2:1-balanced
    over the 26-neighbourhood with the periodic wrap.  Defaults give 21,652
    leaves on levels 2..8 with face, edge and corner jumps."""
    leaves = {(lmin, i, j, k) for i in range(1 << lmin) for j in range(1 << lmin)
              for k in range(1 << lmin)}
    amin = min(a)
    off = np.array([0.0, 0.5, 1.0])
    for L in range(lmin, lmax):
        h = 2.0 ** -L
        rad = r0 / q ** (L - lmin)
        split = []
        for (l, i, j, k) in leaves:
            if l != L:
                continue
            X, Y, Z = np.meshgrid((i + off) * h, (j + off) * h, (k + off) * h, indexing="ij")
            d = (shell_rho(X, Y, Z, a) - 1.0) * amin
            dist = np.sqrt((X - focus[0]) ** 2 + (Y - focus[1]) ** 2 + (Z - focus[2]) ** 2).min()
            if d.min() < band * h and d.max() > -band * h and dist < rad:
                split.append((l, i, j, k))
        for b in split:
            leaves.remove(b)
            l, i, j, k = b
            for c in range(8):
                leaves.add((l + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1)))
    return balance(leaves)


def _holder(leaves, L, i, j, k):
    n = 1 << L
    i, j, k = i % n, j % n, k % n
    for l in range(L, -1, -1):
        s = L - l
        key = (l, i >> s, j >> s, k >> s)
        if key in leaves:
            return key
    return None


def balance(leaves):
    """Split leaves until every pair of touching leaves differs by at most one
    level (26-neighbourhood, periodic)."""
    leaves = set(leaves)
    changed = True
    while changed:
        changed = False
        for b in sorted(leaves, key=lambda t: -t[0]):
            if b not in leaves:
                continue
            L, i, j, k = b
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        if dx == dy == dz == 0:
                            continue
                        h = _holder(leaves, L, i + dx, j + dy, k + dz)
                        if h is not None and h[0] < L - 1:
                            leaves.remove(h)
                            l, a, bb, c = h
                            for q in range(8):
                                leaves.add((l + 1, 2 * a + (q & 1), 2 * bb + ((q >> 1) & 1),
                                            2 * c + ((q >> 2) & 1)))
                            changed = True
    return sorted(leaves)


def c4():
    """Prescribed geometric tree, levels 2..8, 16^3 blocks, 4.2, FD4, FP32,
    tanh shell of width 0.01, periodic shear velocity."""
    return dict(name="c4_geometric_l2-8_nb16_w42_fd4_f32", nb=16, N=4, Nt=2, fd=4,
                level_min=2, level_max=8, prec="f32", eps_refine=1e-2, eps_coarsen=1e-4,
                ic=("shell", np.array([0.20, 0.15, 0.10, 0.01])),
                vel=("shear", ()), cfl=0.5, steps=100, adapt_every=0,
                tree=("geometric",))


def _c5_gaussians(seed):
    r = SplitMix64(seed)
    cs, ss, aa = [], [], []
    for _ in range(64):
        cs.append(tuple(r.uniform(0.0, 1.0) for _ in range(3)))
        ss.append(math.exp(r.uniform(math.log(0.005), math.log(0.1))))
        aa.append(r.uniform(0.5, 1.0))
    return gauss_params(cs, ss, aa)


def gaussian_tree(params, lmin=3, lmax=9, nb=24, m=40.0, k=1.45):
    """Leaves refined around the terms of a Gaussian-sum input: term g
    (centre c, width sigma) asks for blocks of spacing at most sigma / m,
    i.e. level L_g = ceil(log2(m / (nb sigma))) clipped to [lmin, lmax], and
    a block at level L < L_g is split when its periodic distance to c is
    below k sigma.  Then the tree is 2:1-balanced over the 26-neighbourhood
    with the periodic wrap.  The defaults give 61,461 leaves on levels 3..9
    for the 64 terms of the seed-5 draw of c5."""
    rows = np.asarray(params, dtype=np.float64).reshape(-1, 5)
    tgt = np.clip(np.ceil(np.log2(m / (nb * rows[:, 3]))), lmin, lmax).astype(int)
    leaves = {(lmin, i, j, kk) for i in range(1 << lmin) for j in range(1 << lmin)
              for kk in range(1 << lmin)}
    for L in range(lmin, lmax):
        h = 2.0 ** -L
        cur = np.array(sorted(b[1:] for b in leaves if b[0] == L), dtype=np.int64)
        if len(cur) == 0:
            continue
        lo = cur * h
        split = np.zeros(len(cur), bool)
        for (cx, cy, cz, sg, _), Lg in zip(rows, tgt):
            if Lg <= L:
                continue
            d2 = np.zeros(len(cur))
            for ax, c in enumerate((cx, cy, cz)):
                t = (c - lo[:, ax]) % 1.0      # centre relative to the block start
                d2 += np.where(t <= h, 0.0, np.minimum(t - h, 1.0 - t)) ** 2
            split |= d2 < (k * sg) ** 2
        for i, j, kk in cur[split].tolist():
            leaves.remove((L, i, j, kk))
            for c in range(8):
                leaves.add((L + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * kk + ((c >> 2) & 1)))
    return balance(leaves)


_TREES = {}


def tree_of(cfg):
    """Leaf keys of a prescribed-tree workload (cached per process)."""
    kind = cfg["tree"][0]
    if kind not in _TREES:
        if kind == "geometric":
            _TREES[kind] = geometric_tree()
        else:
            _TREES[kind] = gaussian_tree(cfg["ic"][1])
    return _TREES[kind]


def c5(seed=5):
    """The large workload: 24^3 blocks, 6.2, FD6, FP32, sum of 64 Gaussians
    with centres uniform in the periodic cube, log-uniform widths in
    [0.005, 0.1] and amplitudes in [0.5, 1], shear velocity.  The tree is
    prescribed by the Gaussians (gaussian_tree: 61,461 leaves on levels 3..9,
    0.850G points).  Flags use eps_refine 1e-4 / eps_coarsen 1e-6, ratio 100
    above 2^6, with the coarsening threshold about ten times the FP32
    rounding of unit data; the adaptation timed every 5 steps starts from
    the prescribed tree."""
    p = _c5_gaussians(seed)
    return dict(name="c5_gausstree_l3-9_nb24_w62_fd6_f32", nb=24, N=6, Nt=2, fd=6,
                level_min=3, level_max=9, prec="f32", eps_refine=1e-4, eps_coarsen=1e-6,
                ic=("gauss", p), vel=("shear", ()), cfl=0.5, steps=100, adapt_every=5,
                tree=("gaussian", seed))


def c5_adaptive(seed=5, eps_refine=3e-6):
    """The same input on a threshold-driven tree (initial refinement and
    adaptation every 5 steps).  At eps_refine 3e-6 (eps_coarsen 3e-8) the
    FP32 grid keeps its size under time stepping (17,116 leaves, levels
    3..7); below it FP32 rounding of the samples (about 6e-8 of the local
    value) produces details above the thresholds and the grid keeps
    refining, which FP64 runs of the same thresholds do not do."""
    p = _c5_gaussians(seed)
    return dict(name="c5a_adaptive_l3-7_nb24_w62_fd6_f32_eps%g" % eps_refine, nb=24, N=6, Nt=2,
                fd=6, level_min=3, level_max=9, prec="f32", eps_refine=eps_refine,
                eps_coarsen=eps_refine / 100.0, ic=("gauss", p), vel=("shear", ()), cfl=0.5,
                steps=100, adapt_every=5)


def ic_function(ic):
    """Pointwise definition of an initial condition (numpy, FP64), used to
    sample the input on a CPU tree."""
    kind, p = ic
    p = np.asarray(p, dtype=np.float64)
    if kind == "gauss":
        rows = p.reshape(-1, 5)

        def f(X, Y, Z):
            out = np.zeros(np.shape(X))
            for cx, cy, cz, s, a in rows:
                dx = X - cx
                dy = Y - cy
                dz = Z - cz
                dx = dx - np.round(dx)
                dy = dy - np.round(dy)
                dz = dz - np.round(dz)
                out = out + a * np.exp(-(dx * dx + dy * dy + dz * dz) / (s * s))
            return out
        return f

    ax, ay, az, w = p

    def g(X, Y, Z):
        rho = np.sqrt(((X - 0.5) / ax) ** 2 + ((Y - 0.5) / ay) ** 2 + ((Z - 0.5) / az) ** 2)
        return 0.5 * (1.0 - np.tanh((rho - 1.0) * min(ax, ay, az) / w))
    return g


def velocity_spec(vel):
    """(kind, params) with the constants the C ABI expects."""
    kind, p = vel
    if kind == "shear":
        return "shear", ()
    return kind, tuple(p)
