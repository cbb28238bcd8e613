"""Input validation through the C ABI on a live grid: invalid trees, sizes and
arguments return the documented codes, and the grid keeps its tree and field
(the next step still runs and matches a grid that never saw the bad calls)."""
import numpy as np
import pytest

from paper_2112_07537_amd import mr

pytestmark = pytest.mark.gpu

NB, N, NT, FD = 16, 4, 2, 4


def uniform(L):
    n = 1 << L
    return [(L, i, j, k) for k in range(n) for j in range(n) for i in range(n)]


def refine(keys, key):
    L, i, j, k = key
    out = [q for q in keys if q != key]
    out += [(L + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))
            for c in range(8)]
    return out


BAD_TREES = {
    "empty": ([], mr.MR_EINVAL),
    "duplicate": (uniform(1) + [(1, 0, 0, 0)], mr.MR_EINVAL),
    "overlapping": (uniform(1) + [(2, 0, 0, 0)], mr.MR_EINVAL),
    "gap": (uniform(1)[1:], mr.MR_EINVAL),
    "level_out_of_range": ([(13, 0, 0, 0)], mr.MR_EINVAL),
    "index_out_of_range": (uniform(1)[:-1] + [(1, 2, 1, 1)], mr.MR_EINVAL),
    # level 3 at the corner faces level 1 across the periodic wrap
    "not_2to1": (refine(refine(uniform(1), (1, 0, 0, 0)), (2, 0, 0, 0)), mr.MR_EINVAL),
    "over_capacity": (uniform(2), mr.MR_ECAPACITY),
}


def fresh():
    g = mr.Grid(NB, N, NT, fd_order=FD, level_min=0, level_max=6, max_blocks=32)
    g.set_tree(refine(uniform(1), (1, 1, 0, 1)))
    rng = np.random.default_rng(7)
    g.field_set(rng.standard_normal((g.n_blocks(), NB, NB, NB)))
    return g


def test_bad_calls_leave_the_grid_intact():
    g, ref = fresh(), fresh()
    meta0 = g.block_meta().copy()
    f0 = g.field_get().copy()
    for name, (keys, code) in BAD_TREES.items():
        with pytest.raises(mr.MRError) as e:
            g.set_tree(keys)
        assert e.value.code == code, name
        assert np.array_equal(g.block_meta(), meta0), name
        assert np.array_equal(g.field_get(), f0), name
    with pytest.raises(mr.MRError) as e:
        g.field_set(np.zeros((g.n_blocks() - 1, NB, NB, NB)))
    assert e.value.code == mr.MR_EINVAL
    with pytest.raises(mr.MRError) as e:
        g.ghost(depth=1)   # neither the stencil depth nor the wide depth
    assert e.value.code == mr.MR_EINVAL
    v = mr.velocity("const", 1.0, 0.5, 0.25)
    for dt in (0.0, -1e-3, float("nan"), float("inf")):
        with pytest.raises(mr.MRError) as e:
            g.rk3_step(dt, v)
        assert e.value.code == mr.MR_EINVAL, dt
    bad_vel = mr.velocity("const", 1.0, 0.5, 0.25)
    bad_vel.kind = 7
    with pytest.raises(mr.MRError) as e:
        g.rk3_step(1e-3, bad_vel)
    assert e.value.code == mr.MR_EINVAL
    with pytest.raises(mr.MRError) as e:
        g.details(field=3)
    assert e.value.code == mr.MR_EINVAL
    assert np.array_equal(g.field_get(), f0)
    # the grid still steps exactly like one that never saw the bad calls
    dt = g.cfl_dt(v, 0.5)
    g.rk3_step(dt, v)
    ref.rk3_step(dt, v)
    assert np.array_equal(g.field_get(), ref.field_get())
    assert np.array_equal(g.details(), ref.details())
    g.close()
    ref.close()
