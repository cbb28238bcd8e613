"""Launch-shape knobs (mr_set_tuning) change how the ghost work is tiled and
launched, not what it computes: after steps and a detail pass with other
LDS budgets and substitution workgroup size, fields and norms agree with the
defaults to FP64 rounding (f->c sums may round in another order).  Values
out of range are rejected and leave the knobs unchanged."""
import numpy as np
import pytest

from paper_2112_07537_amd import autotune as at
from paper_2112_07537_amd import mr
from paper_2112_07537_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,Nt,nb", [(4, 2, 16), (6, 2, 24), (4, 0, 16)])
def test_knobs_keep_results(N, Nt, nb):
    keys = [(1, i, j, k) for k in range(2) for j in range(2) for i in range(2) if (i, j, k) != (0, 0, 0)]
    keys += [(2, c & 1, (c >> 1) & 1, (c >> 2) & 1) for c in range(8)]
    ic = ("gauss", wl.gauss_params([(0.3, 0.35, 0.4)], [0.12], [1.0]))
    out = []
    for knobs in (None, dict(lds_refine=12288, lds_restrict=16384, lds_subst=24576,
                             subst_threads=256)):
        g = mr.Grid(nb, N, Nt, fd_order=4, level_min=1, level_max=3, prec="f64", max_blocks=512)
        g.set_tree(keys)
        if knobs:
            g.set_tuning(**knobs)
            assert g.get_tuning() == knobs
        g.sample_ic(*ic)
        v = mr.velocity("shear")
        dt = g.cfl_dt(v, 0.5)
        for _ in range(2):
            g.rk3_step(dt, v)
        out.append((g.field_get().copy(), g.details()))
        g.close()
    (fa, na), (fb, nb_) = out
    scale = np.abs(fa).max()
    assert np.abs(fa - fb).max() <= 1e-13 * scale
    assert np.abs(na - nb_).max() <= 1e-13 * scale


def test_bad_knobs_rejected():
    g = mr.Grid(16, 4, 2, fd_order=4, level_min=1, level_max=2, prec="f32", max_blocks=64)
    g.set_tree([(1, i, j, k) for k in range(2) for j in range(2) for i in range(2)])
    before = g.get_tuning()
    for bad in (dict(lds_subst=1024), dict(lds_refine=70000), dict(subst_threads=128)):
        with pytest.raises(mr.MRError):
            g.set_tuning(**bad)
        assert g.get_tuning() == before
    assert mr.device_arch().startswith("gfx")
    assert at.cache_key(mr.device_arch(), wl.c5()) == mr.device_arch() + "/nb24/w6.2/fd6/f32"
    g.close()
