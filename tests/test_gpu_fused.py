"""The fused entry point mr_details_rk3_step against the two calls it fuses
(mr_details, then mr_rk3_step) and against the FP64 oracle, through the C ABI.

The fused step's first stage uses the ghosts of the criterion's wide
reconstruction; the f->c ghost values of the two reconstructions can differ
in rounding order only, so the comparison takes the parity tolerances
(FP64 1e-12, FP32 1e-5 of max|phi|), not bit equality.
"""
import numpy as np
import pytest

from oracle import grid as og
from paper_2112_07537_amd import mr
from paper_2112_07537_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def two_level(Lc, pattern):
    keys = []
    n = 1 << Lc
    for k in range(n):
        for j in range(n):
            for i in range(n):
                if pattern(i, j, k):
                    keys += [(Lc + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))
                             for c in range(8)]
                else:
                    keys.append((Lc, i, j, k))
    return keys


TREE = two_level(1, lambda i, j, k: (i, j, k) in ((0, 0, 0), (1, 1, 0), (0, 1, 1)))
IC = ("gauss", wl.gauss_params([(0.3, 0.6, 0.45), (0.7, 0.35, 0.6)], [0.12, 0.08], [1.0, 0.7]))


def field_of(nb, keys):
    f = wl.ic_function(IC)
    out = []
    for (L, i, j, k) in keys:
        den = float(nb << L)
        x = (i * nb + np.arange(nb)) / den
        y = (j * nb + np.arange(nb)) / den
        z = (k * nb + np.arange(nb)) / den
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        out.append(f(X, Y, Z))
    return np.array(out)


def grid(nb, N, Nt, fd, prec, exec_mode=0):
    g = mr.Grid(nb, N, Nt, fd_order=fd, level_min=0, level_max=6, prec=prec, max_blocks=512,
                exec_mode=exec_mode)
    g.set_tree(TREE)
    g.field_set(field_of(nb, TREE).astype(g.dtype))
    return g


CASES = [(16, 4, 2, 4, "f64"), (16, 2, 0, 4, "f64"), (24, 6, 2, 6, "f32"), (24, 6, 0, 6, "f64")]


@pytest.mark.parametrize("nb,N,Nt,fd,prec", CASES)
@pytest.mark.parametrize("exec_mode", [0, 1, 2])
def test_fused_equals_details_then_step(nb, N, Nt, fd, prec, exec_mode):
    vel = mr.velocity("shear")
    a = grid(nb, N, Nt, fd, prec, exec_mode)
    b = grid(nb, N, Nt, fd, prec, exec_mode)
    dt = a.cfl_dt(vel, 0.5)
    scale = np.abs(a.field_get()).max()
    tol = TOL[prec] * scale
    for step in range(3):
        na = a.details_rk3_step(dt, vel)
        nb_ = b.details()
        b.rk3_step(dt, vel)
        assert np.abs(na - nb_).max() <= tol, (step, np.abs(na - nb_).max())
        fa, fb = a.field_get(), b.field_get()
        err = np.abs(fa.astype(np.float64) - fb).max()
        assert err <= tol, (step, err)
    a.close()
    b.close()


@pytest.mark.parametrize("nb,N,Nt,fd,prec", [(16, 4, 2, 4, "f64"), (24, 6, 2, 6, "f64")])
def test_fused_against_oracle(nb, N, Nt, fd, prec):
    vel = ("shear", ())
    g = grid(nb, N, Nt, fd, prec)
    meta = [tuple(int(v) for v in m) for m in g.block_meta()]
    o = og.Grid(nb, N, Nt, fd_order=fd)
    o.set_tree(meta)
    data = g.field_get().astype(np.float64)
    for i, k in enumerate(meta):
        o.blocks[k] = data[i].copy()
    v = mr.velocity(vel[0], *vel[1])
    dt = g.cfl_dt(v, 0.5)
    norms = g.details_rk3_step(dt, v)
    o.substitute()
    ref = o.norms()
    o.rk3_step(dt, vel)
    scale = max(np.abs(o.blocks[k]).max() for k in meta)
    for i, k in enumerate(meta):
        assert abs(norms[i] - ref[k]) <= TOL[prec] * scale, (k, norms[i], ref[k])
    got = g.field_get()
    err = max(np.abs(got[i] - o.blocks[k]).max() for i, k in enumerate(meta))
    assert err <= TOL[prec] * scale, err
    g.close()


def test_fused_graph_recaptured_after_adapt():
    """Graph mode: the fused graph is re-captured when the tree changes."""
    nb, N, Nt, fd = 16, 4, 2, 4
    vel = mr.velocity("const", 1.0, 0.5, 0.25)
    kw = dict(fd_order=fd, level_min=1, level_max=4, eps_refine=1e-3, eps_coarsen=1e-5,
              max_blocks=8192)
    a = mr.Grid(nb, N, Nt, exec_mode=2, **kw)
    b = mr.Grid(nb, N, Nt, exec_mode=0, **kw)
    for g in (a, b):
        g.init_ic(*IC)
    assert a.n_blocks() == b.n_blocks()
    dt = a.cfl_dt(vel, 0.5)
    for step in range(4):
        na = a.details_rk3_step(dt, vel)
        nb_ = b.details_rk3_step(dt, vel)
        assert np.array_equal(na, nb_), step
        assert np.array_equal(a.field_get(), b.field_get()), step
        if step == 1:
            a.adapt()
            b.adapt()
            assert [tuple(m) for m in a.block_meta()] == [tuple(m) for m in b.block_meta()]
            dt = a.cfl_dt(vel, 0.5)
    a.close()
    b.close()


def test_fused_rejects_bad_arguments():
    g = grid(16, 4, 2, 4, "f64")
    with pytest.raises(mr.MRError) as e:
        g.details_rk3_step(-1.0, mr.velocity("shear"))
    assert e.value.code == mr.MR_EINVAL
    g.close()


def test_fused_async_matches_sync():
    """The asynchronous form (norms left on the device, no synchronisation)
    does the same work as the synchronous one."""
    vel = mr.velocity("shear")
    a = grid(24, 6, 2, 6, "f32")
    b = grid(24, 6, 2, 6, "f32")
    dt = a.cfl_dt(vel, 0.5)
    scale = np.abs(a.field_get()).max()
    for _ in range(2):
        a.details_rk3_step_async(dt, vel)
        b.details_rk3_step(dt, vel)
    a.sync()
    tol = TOL["f32"] * scale
    assert np.abs(a.field_get().astype(np.float64) - b.field_get()).max() <= tol
    assert np.abs(a.details() - b.details()).max() <= tol
    a.close()
    b.close()


@pytest.mark.parametrize("nb,N,Nt,fd,prec", [(24, 6, 2, 6, "f32"), (16, 4, 2, 4, "f64"),
                                             (16, 4, 0, 4, "f32"), (24, 6, 0, 6, "f64")])
def test_batched_fills_repeat_bit_for_bit(nb, N, Nt, fd, prec):
    """Every field point a ghost reconstruction writes is written by one work
    item (disjoint substitution boxes, lifted or not), every substituted
    value is computed from values no item of the launch writes, and the
    launches are ordered (c->f, substitution, f->c), so batched
    reconstructions and steps repeat bit for bit from the same state."""
    vel = mr.velocity("shear")
    out = []
    for _ in range(3):
        g = grid(nb, N, Nt, fd, prec)
        dt = g.cfl_dt(vel, 0.5)
        g.ghost(depth=0)                 # the stencil depth
        ghosts = g.ghost_get(fd // 2)
        norms = g.details_rk3_step(dt, vel)
        g.rk3_step(dt, vel)
        out.append((ghosts, norms, g.field_get()))
        g.close()
    for rep in out[1:]:
        for a, b in zip(out[0], rep):
            assert np.array_equal(a, b)
