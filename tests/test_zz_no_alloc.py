"""mr_details_noalloc (the entry point that allocates nothing) against
mr_details through the C ABI: two calls in a row, the second on a smaller
grid, norms identical bit for bit."""
import numpy as np
import pytest

from paper_2112_07537_amd import mr
from paper_2112_07537_amd import workloads as wl

pytestmark = pytest.mark.gpu

IC = ("gauss", wl.gauss_params([(0.31, 0.42, 0.36), (0.7, 0.6, 0.55)], [0.08, 0.05], [1.0, 0.6]))


def grid(keys):
    g = mr.Grid(16, 4, 2, fd_order=4, level_min=1, level_max=4, prec="f32", max_blocks=1024)
    g.set_tree(keys)
    g.sample_ic(*IC)
    return g


def two_level(pattern):
    keys = []
    for k in range(2):
        for j in range(2):
            for i in range(2):
                if pattern(i, j, k):
                    keys += [(2, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))
                             for c in range(8)]
                else:
                    keys.append((1, i, j, k))
    return keys


def test_noalloc_details_match_details():
    import torch
    big = two_level(lambda i, j, k: (i, j, k) in ((0, 0, 0), (1, 1, 0), (0, 1, 1)))
    small = two_level(lambda i, j, k: (i, j, k) == (1, 0, 1))
    out = torch.full((len(big),), -1.0, dtype=torch.float64, device="cuda")
    for keys in (big, small):
        a, b = grid(keys), grid(keys)
        n = a.n_blocks()
        assert n == len(keys)
        ref = b.details()
        torch.cuda.synchronize()
        a.details_noalloc(out.data_ptr())
        a.sync()
        got = out[:n].cpu().numpy()
        assert np.array_equal(got, ref)
        assert np.array_equal(a.field_get(), b.field_get())   # same substitution
        a.close()
        b.close()
    # a grid beyond the static capacity is refused before any work
    with pytest.raises(mr.MRError) as e:
        g = mr.Grid(8, 2, 2, fd_order=4, level_min=6, level_max=6, max_blocks=1 << 18)
        g.details_noalloc(out.data_ptr())
    assert e.value.code == mr.MR_ECAPACITY
