"""GPU edge cases against the FP64 oracle, through the C ABI.

* A single block at level 0: every neighbour is the block itself across the
  periodic wrap (ghosts, RK3 step, details).
* The smallest block size (nb = 8) with resolution jumps, for the wavelets
  whose refinement windows fit its owner map (2.0, 2.2); the wider ones are
  rejected with a clear error at creation.
* Three levels at once (2, 3, 4; 2:1 balanced over the periodic wrap).
* Capacity and non-finite error paths leave the grid usable.
"""
import numpy as np
import pytest

from oracle import grid as og
from paper_2112_07537_amd import mr
from paper_2112_07537_amd import workloads as wl

pytestmark = pytest.mark.gpu


def oracle_of(g, N, Nt, fd, **kw):
    meta = [tuple(int(v) for v in m) for m in g.block_meta()]
    data = g.field_get().astype(np.float64)
    o = og.Grid(g.nb, N, Nt, fd_order=fd, **kw)
    o.set_tree(meta)
    for b, k in enumerate(meta):
        o.blocks[k] = data[b].copy()
    return o, meta


def check_step_and_details(g, N, Nt, fd, vel=("shear", ()), tol=1e-12):
    o, meta = oracle_of(g, N, Nt, fd)
    v = mr.velocity(vel[0], *vel[1])
    dt = g.cfl_dt(v, 0.5)
    # details of the initial state (the ghost reconstruction before the
    # transform substitutes the slabs next to coarser leaves, on both sides)
    nrm = g.details()
    o.substitute()
    ref = o.norms()
    scale = max(np.abs(o.blocks[k]).max() for k in meta)
    for b, k in enumerate(meta):
        assert abs(nrm[b] - ref[k]) <= tol * scale, (k, nrm[b], ref[k])
    # one RK3 step
    g.rk3_step(dt, v)
    o.rk3_step(dt, vel)
    got = g.field_get()
    err = max(np.abs(got[b] - o.blocks[k]).max() for b, k in enumerate(meta))
    assert err <= tol * scale, err


def ic_field(g, ic):
    f = wl.ic_function(ic)
    out = []
    for (L, i, j, k) in [tuple(int(v) for v in m) for m in g.block_meta()]:
        den = float(g.nb << L)
        x = (i * g.nb + np.arange(g.nb)) / den
        y = (j * g.nb + np.arange(g.nb)) / den
        z = (k * g.nb + np.arange(g.nb)) / den
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        out.append(f(X, Y, Z))
    return np.array(out)


IC = ("gauss", wl.gauss_params([(0.3, 0.6, 0.45)], [0.15], [1.0]))


@pytest.mark.parametrize("N,Nt", [(4, 2), (6, 2), (2, 0)])
def test_single_block_level0(N, Nt):
    nb, fd = 24, 6 if N == 6 else 4
    g = mr.Grid(nb, N, Nt, fd_order=fd, level_min=0, level_max=0, max_blocks=8)
    g.set_tree([(0, 0, 0, 0)])
    g.field_set(ic_field(g, IC))
    check_step_and_details(g, N, Nt, fd)
    g.close()


def jump_tree():
    keys = []
    for k in range(2):
        for j in range(2):
            for i in range(2):
                if (i, j, k) in ((0, 0, 0), (1, 1, 1)):
                    keys += [(2, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))
                             for c in range(8)]
                else:
                    keys.append((1, i, j, k))
    return keys


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("N,Nt", [(2, 2), (2, 0)])
def test_smallest_blocks(N, Nt, prec):
    nb, fd = 8, 4
    g = mr.Grid(nb, N, Nt, fd_order=fd, level_min=0, level_max=4, prec=prec, max_blocks=256)
    g.set_tree(jump_tree())
    g.field_set(ic_field(g, IC).astype(g.dtype))
    check_step_and_details(g, N, Nt, fd, tol=1e-12 if prec == "f64" else 1e-5)
    g.close()


@pytest.mark.parametrize("N,Nt,fd", [(4, 2, 4), (6, 2, 6), (6, 0, 6)])
def test_smallest_blocks_reject_wide_wavelets(N, Nt, fd):
    """With nb = 8 the owner map (half a block around it) cannot hold the
    samples of N >= 4 ghost reconstructions: creation fails with EINVAL."""
    with pytest.raises(mr.MRError) as e:
        mr.Grid(8, N, Nt, fd_order=fd, level_min=0, level_max=4, max_blocks=256)
    assert e.value.code == mr.MR_EINVAL
    assert "nb too small" in str(e.value)


def three_level_tree():
    """Levels 2, 3 and 4 at once: level-2 blocks with indices in {0,1,2}^3
    are split into level 3, and the level-3 block (2,2,2), whose 26
    neighbours are all level 3, is split into level 4 (2:1 holds across the
    periodic wrap)."""
    keys = []
    for k in range(4):
        for j in range(4):
            for i in range(4):
                if max(i, j, k) <= 2:
                    for c in range(8):
                        keys.append((3, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1),
                                     2 * k + ((c >> 2) & 1)))
                else:
                    keys.append((2, i, j, k))
    keys.remove((3, 2, 2, 2))
    keys += [(4, 4 + (c & 1), 4 + ((c >> 1) & 1), 4 + ((c >> 2) & 1)) for c in range(8)]
    return keys


@pytest.mark.parametrize("N,Nt", [(2, 2), (2, 0)])
def test_three_levels(N, Nt):
    nb, fd = 8, 4
    g = mr.Grid(nb, N, Nt, fd_order=fd, level_min=0, level_max=6, max_blocks=512)
    g.set_tree(three_level_tree())
    g.field_set(ic_field(g, IC))
    ts = g.tree_stats()
    assert (ts[4], ts[3]) == (2, 4)
    check_step_and_details(g, N, Nt, fd)
    g.close()


def test_capacity_error_keeps_grid_usable():
    nb, N, Nt, fd = 16, 4, 2, 4
    g = mr.Grid(nb, N, Nt, fd_order=fd, level_min=1, level_max=4, eps_refine=1e-4,
                eps_coarsen=1e-6, max_blocks=16)
    g.set_tree([(1, i, j, k) for k in range(2) for j in range(2) for i in range(2)])
    g.sample_ic(*IC)
    before = g.field_get().copy()
    with pytest.raises(mr.MRError) as e:
        g.adapt()
    assert e.value.code == mr.MR_ECAPACITY
    assert g.n_blocks() == 8
    assert np.array_equal(g.field_get(), before)
    v = mr.velocity("const", 1.0, 0.5, 0.25)
    g.rk3_step(g.cfl_dt(v, 0.5), v)
    assert np.isfinite(g.field_get()).all()
    g.close()


def test_nonfinite_field_reported():
    g = mr.Grid(16, 4, 2, fd_order=4, level_min=1, level_max=2, max_blocks=64)
    g.set_tree([(1, i, j, k) for k in range(2) for j in range(2) for i in range(2)])
    f = np.zeros((8, 16, 16, 16))
    f[3, 5, 6, 7] = np.nan
    g.field_set(f)
    for call in (g.details, g.adapt):
        with pytest.raises(mr.MRError) as e:
            call()
        assert e.value.code == mr.MR_ENONFINITE
    g.field_set(np.zeros((8, 16, 16, 16)))
    assert np.isfinite(g.details()).all()
    g.close()
