"""Pins of the block-octree oracle against what the paper and mathematics fix.

* Brute force on tiny two-level trees (independent global formulation in
  tests/brute.py): c->f ghosts equal the global Deslauriers-Dubuc
  refinement; f->c ghosts equal the global restriction.  The substitution
  has its own pins in test_oracle_substitution.py.
* Polynomial exactness of ghosts, substitution and details (sections 2.1.3,
  2.2.2 and 2.2.4): per-axis degree < N is reproduced exactly.
* One RK3 step on a uniform periodic grid equals the Fourier closed form
  R(z) = 1 + z + z^2/2 + z^3/6 with the central-FD symbol.
* Spatial orders of the FD stencils, uniform and across a resolution jump
  (validation section: p = min(k, N - 1) for a first derivative).
* Moment conservation of lifted coarsening (validation section, moments).
* Adaptation invariants (2:1, level bounds, criterion at exit) and the
  epsilon-test bound E_inf <= C1 * eps_c with C1 = O(1) (section 2.1.5).
"""
import numpy as np
import pytest

from oracle import grid as og
from oracle import wavelets as wv
from tests import brute

ALL_WAVELETS = wv.WAVELETS


def two_level_tree(nb, Lc, pattern):
    """Level-Lc tree with the blocks selected by ``pattern(i,j,k)`` refined."""
    keys = []
    n = 1 << Lc
    for k in range(n):
        for j in range(n):
            for i in range(n):
                if pattern(i, j, k):
                    for c in range(8):
                        keys.append((Lc + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1),
                                     2 * k + ((c >> 2) & 1)))
                else:
                    keys.append((Lc, i, j, k))
    return keys


def smooth_periodic(X, Y, Z):
    tp = 2 * np.pi
    return (np.sin(tp * X + 0.3) * np.cos(tp * Y - 0.2) * np.sin(tp * Z + 1.1)
            + 0.25 * np.cos(2 * tp * X + 2 * tp * Y))


def rough_field(seed):
    rng = np.random.default_rng(seed)
    return lambda key: rng.standard_normal((16, 16, 16))


# --------------------------------------------------------------- brute force
@pytest.mark.parametrize("N,Nt", ALL_WAVELETS)
def test_brute_force_two_level(N, Nt):
    nb = 16
    g = og.Grid(nb, N, Nt)
    keys = two_level_tree(nb, 1, lambda i, j, k: (i, j, k) in ((0, 0, 0), (1, 1, 0), (0, 1, 1)))
    g.set_tree(keys, init=rough_field(11 + N + Nt))
    orig = {k: v.copy() for k, v in g.blocks.items()}
    g.substitute()
    # the substitution changes no all-even point, so the global refinement of
    # the samples is the same before and after it
    bf = brute.TwoLevel(nb, 2, {k: v.copy() for k, v in g.blocks.items()})
    G = bf.refined(N)
    W = nb << 2
    changed = 0
    for key in g.keys():
        if key[0] != 2:
            continue
        o = g.origin(key)
        changed += int((g.blocks[key] != orig[key]).sum())
        # c->f ghosts (points in coarser leaves) equal G
        D = 4
        X = g.ghost_block(key, D)
        idx = [(np.arange(-D, nb + D) + o[a]) % W for a in range(3)]
        Gb = G[np.ix_(idx[2], idx[1], idx[0])]
        zz, yy, xx = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
        lev = g.owner_level(2, xx, yy, zz)
        m = lev < 2
        np.testing.assert_allclose(X[m], Gb[m], rtol=0, atol=1e-13)
        # same-level ghosts equal the fine values
        m = lev == 2
        same = np.array([g.blocks[(2, xv // nb, yv // nb, zv // nb)][zv % nb, yv % nb, xv % nb]
                         for xv, yv, zv in zip(xx[m], yy[m], zz[m])])
        np.testing.assert_array_equal(X[m], same)
    assert changed > 0
    # f->c ghosts of coarse blocks inside fine leaves: restriction of G'
    bf2 = brute.TwoLevel(nb, 2, g.blocks)
    C = bf2.coarse_view(N, Nt)
    Wc = nb << 1
    for key in g.keys():
        if key[0] != 1:
            continue
        o = g.origin(key)
        D = 3
        X = g.ghost_block(key, D)
        idx = [(np.arange(-D, nb + D) + o[a]) % Wc for a in range(3)]
        zz, yy, xx = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
        lev = g.owner_level(1, xx, yy, zz)
        m = lev == 2
        np.testing.assert_allclose(X[m], C[zz[m], yy[m], xx[m]], rtol=0, atol=1e-12)


# ------------------------------------------------------ polynomial exactness
def poly(deg):
    def f(X, Y, Z):
        # per-axis degree <= deg, centred away from the periodic wrap
        p = lambda t: sum(((t - 0.7) ** e) * (1.0 + 0.1 * e) for e in range(deg + 1))
        return p(X) * (1 + 0.5 * p(Y)) * (2 - p(Z))
    return f


@pytest.mark.parametrize("N,Nt", ALL_WAVELETS)
def test_polynomial_exactness(N, Nt):
    nb = 16
    g = og.Grid(nb, N, Nt)
    # refine the blocks around the domain centre so a fine block sees coarse
    # neighbours on several sides without touching the wrap
    keys = []
    n = 4
    for k in range(n):
        for j in range(n):
            for i in range(n):
                if (i, j, k) in ((2, 2, 2), (2, 1, 2)):
                    for c in range(8):
                        keys.append((3, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1),
                                     2 * k + ((c >> 2) & 1)))
                else:
                    keys.append((2, i, j, k))
    g.set_tree(keys)
    f = poly(N - 1)
    g.sample(f)
    before = {k: v.copy() for k, v in g.blocks.items()}
    g.substitute()
    for k in g.keys():
        np.testing.assert_allclose(g.blocks[k], before[k], rtol=0, atol=1e-12)
    for key in [(3, 5, 5, 5), (3, 4, 3, 4), (2, 1, 2, 2), (2, 2, 2, 1)]:
        L = key[0]
        D = 6
        X = g.ghost_block(key, D)
        o = g.origin(key)
        c = [(o[a] - D + np.arange(nb + 2 * D)) / (nb << L) for a in range(3)]
        Zc, Yc, Xc = np.meshgrid(c[2], c[1], c[0], indexing="ij")
        np.testing.assert_allclose(X, f(Xc, Yc, Zc), rtol=0, atol=1e-11)
        det = g.block_details(key)
        assert np.abs(det).max() < 1e-11
    # degree N is not annihilated
    g.sample(poly(N))
    assert np.abs(g.block_details((3, 5, 5, 5))).max() > 1e-11    # ~h^N, far above roundoff


# ---------------------------------------------------- RK3 Fourier closed form
@pytest.mark.parametrize("fd", [4, 6])
def test_rk3_fourier_closed_form(fd):
    nb, L = 16, 1
    g = og.Grid(nb, 4, 0, fd_order=fd)
    g.uniform(L)
    ic = lambda X, Y, Z: np.exp(-((X - .5) ** 2 + (Y - .5) ** 2 + (Z - .5) ** 2) / 0.1 ** 2)
    g.sample(ic)
    W = nb << L
    glob = np.zeros((W, W, W))
    for (l, i, j, k), a in g.blocks.items():
        glob[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb] = a
    u = (1.0, 0.5, 0.25)
    h = 1.0 / W
    dt = 0.5 * h / sum(abs(v) for v in u)
    g.rk3_step(dt, ("const", u))
    out = np.zeros_like(glob)
    for (l, i, j, k), a in g.blocks.items():
        out[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb] = a
    th = 2 * np.pi * np.fft.fftfreq(W)
    if fd == 4:
        s = (8 * np.sin(th) - np.sin(2 * th)) / 6
    else:
        s = (45 * np.sin(th) - 9 * np.sin(2 * th) + np.sin(3 * th)) / 30
    sz, sy, sx = np.meshgrid(s, s, s, indexing="ij")
    z = -1j * dt * (u[0] * sx + u[1] * sy + u[2] * sz) / h
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6
    ref = np.real(np.fft.ifftn(R * np.fft.fftn(glob)))
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


# ------------------------------------------------------------ FD convergence
def rhs_error(g, vel, exact):
    err = 0.0
    for key in g.keys():
        r = g.rhs_block(key, vel)
        x, y, z = g.positions(key)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        err = max(err, float(np.abs(r - exact(X, Y, Z)).max()))
    return err


def advect_exact(X, Y, Z, u=(1.0, 0.5, 0.25)):
    tp = 2 * np.pi
    f = np.sin(tp * X) * np.sin(tp * Y) * np.sin(tp * Z)
    fx = tp * np.cos(tp * X) * np.sin(tp * Y) * np.sin(tp * Z)
    fy = tp * np.sin(tp * X) * np.cos(tp * Y) * np.sin(tp * Z)
    fz = tp * np.sin(tp * X) * np.sin(tp * Y) * np.cos(tp * Z)
    return f, -(u[0] * fx + u[1] * fy + u[2] * fz)


@pytest.mark.parametrize("fd", [4, 6])
def test_uniform_fd_order(fd):
    errs = []
    for L in (0, 1):
        g = og.Grid(8, 4, 0, fd_order=fd)
        g.uniform(L)
        g.sample(lambda X, Y, Z: advect_exact(X, Y, Z)[0])
        errs.append(rhs_error(g, ("const", (1.0, 0.5, 0.25)),
                              lambda X, Y, Z: advect_exact(X, Y, Z)[1]))
    order = np.log2(errs[0] / errs[1])
    assert order > fd - 0.3


@pytest.mark.slow
@pytest.mark.parametrize("N,Nt,p", [(2, 2, 1), (4, 0, 3), (4, 2, 3), (6, 2, 4)])
def test_two_level_fd_order(N, Nt, p):
    """Validation section, two-level grids: one eighth of the grid one level
    coarser; FD4 first derivative converges as h^min(4, N-1)."""
    errs = []
    for Lc in (1, 2):
        g = og.Grid(8, N, Nt, fd_order=4)
        n = 1 << Lc
        keys = two_level_tree(8, Lc, lambda i, j, k: not (i < n // 2 and j < n // 2 and k < n // 2))
        g.set_tree(keys)
        g.sample(lambda X, Y, Z: advect_exact(X, Y, Z)[0])
        g.substitute()
        errs.append(rhs_error(g, ("const", (1.0, 0.5, 0.25)),
                              lambda X, Y, Z: advect_exact(X, Y, Z)[1]))
    order = np.log2(errs[0] / errs[1])
    assert order > p - 0.5, (errs, order)
    assert order < p + 1.5, (errs, order)


# ------------------------------------------------------------------ moments
@pytest.mark.parametrize("N,Nt", ALL_WAVELETS)
def test_uniform_coarsening_moments(N, Nt):
    nb = 8
    g = og.Grid(nb, N, Nt, level_min=0, level_max=3, eps_refine=1e9, eps_coarsen=1e9)
    g.uniform(2)
    # compact support (value at the periodic wrap ~1e-17): the moment identity
    # holds on the infinite line, so x must not wrap inside the field's support
    ic = lambda X, Y, Z: np.exp(-((X - .5) ** 2 + (Y - .5) ** 2 + (Z - .5) ** 2) / 0.05 ** 2)
    g.sample(ic)
    m0 = g.moments()
    g.substitute()
    g.apply(set(), {(1, i, j, k) for i in range(2) for j in range(2) for k in range(2)})
    m1 = g.moments()
    rel = np.abs(m1 - m0).max() / np.abs(m0).max()
    if Nt == 2:
        assert rel < 1e-13
    else:
        assert rel > 1e-8


@pytest.mark.parametrize("N,Nt,nb", [(2, 2, 16), (4, 2, 16), (6, 2, 24), (4, 0, 16)])
def test_partial_coarsening_moments_on_the_finest_level(N, Nt, nb):
    """Moment test of the validation section on a grid with resolution jumps:
    one sibling set coarsened next to fine blocks (the Gaussian's centre on
    its corner, so the discarded details are large at the jumps), then
    refined back.  The moments of the finest-level field (the scaling-
    coefficient moments of section 2.1.4) are those of the samples to
    round-off for the lifted wavelets, whose primal wavelets have two
    vanishing moments, and not for N.0."""
    g = og.Grid(nb, N, Nt, level_min=0, level_max=3, eps_refine=1e9, eps_coarsen=1e9)
    g.uniform(2)
    g.sample(lambda X, Y, Z: np.exp(-((X - .5) ** 2 + (Y - .5) ** 2 + (Z - .5) ** 2) / 0.08 ** 2))
    m0 = g.moments()
    g.substitute()
    g.apply(set(), {(1, 0, 0, 0)})
    assert len(g.blocks) == 57
    g.substitute()
    g.apply({(1, 0, 0, 0)}, set())
    assert len(g.blocks) == 64
    rel = np.abs(g.moments() - m0).max() / m0[0]
    if Nt == 2:
        assert rel < 1e-14
    else:
        assert rel > 1e-7


@pytest.mark.parametrize("N,Nt", ALL_WAVELETS)
def test_coarsen_and_update_match_global_transform(N, Nt):
    """Coarsening a sibling set keeps its scaling coefficients (section 2.2.1)
    and the update step turns every kept fine block into the inverse transform
    of all coefficients except the discarded details: checked against an
    independent periodic global transform with those details set to zero.
    The discarded details are those inside the coarsened sets and, in each
    kept neighbour, those of its coarse-extension slab toward them (section
    2.2.1: for 2.2 in 1D, gamma_2^0 is discarded as well when the region in
    front coarsens; the slab extent is pinned to Table 3 separately)."""
    nb, L = 8, 2
    g = og.Grid(nb, N, Nt, level_min=0, level_max=3)
    g.uniform(L)
    rng = np.random.default_rng(17 + N + Nt)
    W = nb << L
    f = rng.standard_normal((W, W, W))
    for (l, i, j, k) in g.keys():
        g.blocks[(l, i, j, k)] = f[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb,
                                   i * nb:(i + 1) * nb].copy()
    groups = {(1, 0, 0, 0), (1, 1, 1, 0)}
    g.apply(set(), groups)
    u = brute.analysis_global(f, N, Nt)
    par = (np.arange(W) % 2)
    odd = (par[:, None, None] + par[None, :, None] + par[None, None, :]) > 0
    inside = np.zeros((W, W, W), bool)
    for (_, i, j, k) in groups:
        s = 2 * nb
        inside[k * s:(k + 1) * s, j * s:(j + 1) * s, i * s:(i + 1) * s] = True
    ext = np.zeros((W, W, W), bool)
    children = {(L, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))
                for (_, i, j, k) in groups for c in range(8)}
    n = 1 << L
    for (l, i, j, k) in g.keys():
        if l != L:
            continue
        dirs = [d for d in og.DIRS
                if (L, (i + d[0]) % n, (j + d[1]) % n, (k + d[2]) % n) in children]
        ext[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb] = g.extension_mask(dirs)
    u2 = np.where((odd & inside) | ext, 0.0, u)
    f2 = brute.synthesis_global(u2, N, Nt)
    for key, a in g.blocks.items():
        l, i, j, k = key
        if l == L:
            ref = f2[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb]
        else:
            s = 2 * nb
            ref = u[k * s:(k + 1) * s:2, j * s:(j + 1) * s:2, i * s:(i + 1) * s:2]
        np.testing.assert_allclose(a, ref, rtol=0, atol=1e-12)


# -------------------------------------------------------------------- adapt
def gauss(c, s):
    def f(X, Y, Z):
        d = [X - c[0], Y - c[1], Z - c[2]]
        d = [v - np.round(v) for v in d]
        return np.exp(-(d[0] ** 2 + d[1] ** 2 + d[2] ** 2) / s ** 2)
    return f


@pytest.mark.slow
@pytest.mark.parametrize("N,Nt", [(4, 2), (4, 0)])
def test_adapt_invariants(N, Nt):
    g = og.Grid(8, N, Nt, fd_order=4, level_min=1, level_max=3,
                eps_refine=1e-3, eps_coarsen=1e-5)
    st = g.init_ic(gauss((0.42, 0.5, 0.55), 0.12))
    assert g.is_balanced()
    levels = {k[0] for k in g.keys()}
    assert min(levels) >= 1 and max(levels) <= 3
    assert max(levels) > min(levels)
    g.substitute()
    nrm = g.norms()
    for k, v in nrm.items():
        if k[0] < g.level_max:
            assert v < g.eps_r
    # one step then adapt keeps the invariants
    g.rk3_step(0.2 / (8 << 3) / 1.75, ("const", (1.0, 0.5, 0.25)))
    g.adapt()
    assert g.is_balanced()


@pytest.mark.slow
@pytest.mark.parametrize("N,Nt", [(4, 2), (6, 2), (4, 0)])
def test_epsilon_bound(N, Nt):
    """Epsilon test of the validation section at small scale: coarsen a
    uniform field with eps_c, refine back to L_max, compare."""
    nb, Lmax = 8, 3
    f = gauss((0.5, 0.5, 0.5), 0.15)
    for eps in (1e-3, 1e-4):
        g = og.Grid(nb, N, Nt, level_min=0, level_max=Lmax,
                    eps_refine=1e9, eps_coarsen=eps)
        g.uniform(Lmax)
        g.sample(f)
        g.adapt()
        assert len(g.blocks) < 8 ** Lmax
        # refine everything back to Lmax
        while min(k[0] for k in g.keys()) < Lmax:
            g.substitute()
            g.apply({k for k in g.keys() if k[0] < Lmax}, set())
        err = 0.0
        for key in g.keys():
            x, y, z = g.positions(key)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            err = max(err, float(np.abs(g.blocks[key] - f(X, Y, Z)).max()))
        assert err <= 3.0 * eps, (eps, err)


def test_translation_by_one_block_is_exact():
    nb = 8
    keys = two_level_tree(nb, 1, lambda i, j, k: (i, j, k) == (0, 1, 0))
    rng = np.random.default_rng(1)
    data = {k: rng.standard_normal((nb, nb, nb)) for k in keys}
    g1 = og.Grid(nb, 4, 2)
    g1.set_tree(keys, init=lambda k: data[k].copy())
    g2 = og.Grid(nb, 4, 2)

    def shift(k):
        L = k[0]
        s = 1 << (L - 1)           # one level-1 block = 2^(L-1) blocks at L
        return (L, (k[1] + s) % (1 << L), k[2], k[3])
    g2.set_tree([shift(k) for k in keys], init=None)
    for k in keys:
        g2.blocks[shift(k)] = data[k].copy()
    vel = ("const", (1.0, 0.5, 0.25))
    g1.rk3_step(1e-3, vel)
    g2.rk3_step(1e-3, vel)
    for k in keys:
        assert np.array_equal(g1.blocks[k], g2.blocks[shift(k)])


def test_detail_ratio_per_level():
    """Section 2.2.5: ||gamma|| scales as h^N, so one uniform refinement
    divides the block norm of a smooth field by about 2^N."""
    f = smooth_periodic
    for N, Nt in [(2, 2), (4, 0)]:
        ns = []
        for L in (2, 3):
            g = og.Grid(8, N, Nt, detail_ext=0)
            g.uniform(L)
            g.sample(f)
            ns.append(max(g.norms().values()))
        ratio = ns[0] / ns[1]
        assert 2 ** N / 1.6 < ratio < 2 ** N * 1.6, (N, ratio)


def test_refined_data_has_no_details():
    nb = 8
    g = og.Grid(nb, 4, 2, detail_ext=0)
    g.uniform(1)
    g.sample(gauss((0.4, 0.5, 0.6), 0.2))
    g.apply({k for k in g.keys()}, set())
    assert max(g.norms().values()) < 1e-14
