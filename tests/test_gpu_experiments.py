"""The validation experiments of section 4 at reduced size, and the
caller-flag adaptation they use, on the GPU.

* mr_adapt_flags against the oracle's policy and interpolation on the same
  block statuses (FP64, 1e-12 of max|phi|): a coarsened octant plus
  refinements that propagate to coarser neighbours.
* Epsilon test (section 4.1) with the finest level 4: E_inf <= C1 eps_c with
  C1 of order one (the paper observes C1 = O(1); its own ratios reach 2.9),
  compression monotone in eps_c, and the lifted wavelets conserve M_0 and
  M_1 (section 4.2: moments on the finest level of the samples and of the
  compressed field refined back) to round-off.
* Two-level convergence (section 4.3) on fine levels 2..4: the observed
  order approaches p = min(k, N - 1) for the advection schemes (k = 3 for
  CONS-3, 5 for CONS-5) and p = min(k, N - 2) for the DIFF-2 / DIFF-4
  Laplacian.
"""
import math

import numpy as np
import pytest

from oracle import grid as og
from paper_2112_07537_amd import experiments as ex
from paper_2112_07537_amd import mr
from paper_2112_07537_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,Nt", [(4, 2), (4, 0), (6, 2)])
def test_adapt_flags_matches_oracle(N, Nt):
    """Level 3 (8^3 blocks of 16^3, 24^3 for N = 6): the octant [0, 1/2)^3 is coarsened and
    two blocks away from it are refined (a refinement next to the octant
    would block its coarsening: no neighbour of a coarsened set may refine)."""
    nb = 16 if N < 6 else 24
    kw = dict(level_min=1, level_max=4, eps_refine=1e-2, eps_coarsen=1e-4)
    keys = ex.uniform_keys(3)
    ic = ("gauss", wl.gauss_params([(0.45, 0.55, 0.5)], [0.12], [1.0]))
    g = mr.Grid(nb, N, Nt, fd_order=4, prec="f64", max_blocks=4096, **kw)
    g.set_tree(keys)
    g.sample_ic(*ic)
    meta = g.block_meta()
    flags = ex.two_level_tree_flags(meta, 3)
    index = [tuple(int(v) for v in m) for m in meta]
    for key in ((3, 6, 6, 6), (3, 5, 2, 6)):
        flags[index.index(key)] = 1
    st = g.adapt_flags(flags)
    o = og.Grid(nb, N, Nt, fd_order=4, **kw)
    o.set_tree(keys)
    o.sample(wl.ic_function(ic))
    o.substitute()
    fl = {tuple(int(v) for v in m): {1: og.FINER, -1: og.COARSER, 0: og.SAME}[int(f)]
          for m, f in zip(meta, flags)}
    refine, coarsen = o.policy(fl, set())
    o.apply(refine, coarsen)
    assert (st.refined, st.coarsened) == (len(refine), len(coarsen))
    assert st.coarsened == 8 and st.refined == 2
    got = [tuple(int(v) for v in m) for m in g.block_meta()]
    assert sorted(got) == o.keys()
    f = g.field_get()
    scale = max(float(np.abs(a).max()) for a in o.blocks.values())
    err = max(float(np.abs(f[b] - o.blocks[k]).max()) for b, k in enumerate(got))
    assert err <= 1e-12 * scale, err
    with pytest.raises(mr.MRError):
        g.adapt_flags(np.full(g.n_blocks(), 2, np.int8))
    g.close()


@pytest.mark.parametrize("w", ex.WAVELETS)
def test_epsilon_and_moments_small(w):
    recs = list(ex.epsilon_test(w, eps_list=(1e-2, 1e-4, 1e-6, 1e-8), lmax=4))
    for r in recs:
        print("%s eps %.0e: %d blocks, E_inf %.3e (%.2f eps), M0 %.2e, M1 %.2e "
              "(leaf sums %.2e, %.2e), %.1fs"
              % (w, r["eps"], r["n_blocks"], r["e_inf"], r["e_inf"] / r["eps"], r["m0"],
                 r["m1"], r["m0_leaf_sum"], r["m1_leaf_sum"], r["seconds"]))
    nblk = [r["n_blocks"] for r in recs]
    assert nblk == sorted(nblk) and nblk[-1] > nblk[0]
    for r in recs:
        assert r["e_inf"] <= 4.0 * r["eps"], r
        if w.endswith(".2"):
            assert r["m0"] <= 1e-13 * r["m0_value"], r
            assert r["m1"] <= 1e-13 * r["m0_value"], r


@pytest.mark.parametrize("w,fd,diff", [("2.2", 3, False), ("4.2", 3, False), ("4.0", 5, False),
                                       ("6.2", 5, False), ("4.2", 2, True), ("6.2", 4, True),
                                       ("4.0", 4, True)])
def test_two_level_convergence_small(w, fd, diff):
    """Advection: p = min(k, N - 1); the DIFF-2 / DIFF-4 Laplacian: p =
    min(k, N - 2) (section 4.3)."""
    N = int(w[0])
    p = min(fd, N - (2 if diff else 1))
    recs = list(ex.two_level(w, fd, levels=(2, 3, 4), diffusion=diff))
    e = [r["e_inf"] for r in recs]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
    print(w, fd, e, orders)
    assert orders[-1] >= p - 0.6, (e, orders)
    assert orders[-1] <= p + 1.0, (e, orders)
