"""Pins of the oracle against numbers the paper prints (fixtures under
tests/golden/, each file names the table it holds).

* Dual-lifting coefficients (section 2.1.4 table): the oracle's dual-lifting
  rows and its Deslauriers-Dubuc prediction weights.
* Ghost-point requirements (section 2.2.5 table), derived here from the
  supports of the oracle's filter rows:
  - coarsening: H^a applied at every even position of a block,
  - refinement: zero-detail synthesis of every fine position of a block,
  - 1D coarse-region extension: the farthest detail coefficient outside the
    block that the synthesis rows of the block's points read,
  - the oracle's detail-band extension equals the printed 3D column.
"""
import os
from fractions import Fraction as Fr

import pytest

from oracle import grid as og
from oracle import wavelets as wv

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
WAVELETS = [(2, 0), (2, 2), (4, 0), (4, 2), (6, 0), (6, 2)]
NB = 16


def _rows(name):
    with open(os.path.join(HERE, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _requirements():
    out = {}
    for r in _rows("ghost_point_requirements.txt"):
        v = [int(x) for x in r]
        out[(v[0], v[1])] = dict(zip(
            ["cf", "cb", "ef1", "ef3", "eb1", "eb3", "uf1", "uf3", "ub1", "ub3", "rf", "rb"], v[2:]))
    return out


REQ = _requirements()


def test_fixture_covers_all_wavelets():
    assert sorted(REQ) == WAVELETS


def test_dual_lifting_rows():
    printed = {}
    for n, i, s in _rows("dual_lifting_coefficients.txt"):
        printed.setdefault(int(n), {})[int(i)] = Fr(s)
    for N in (2, 4, 6):
        assert wv.DUAL_LIFT[N] == printed[N]
        # the prediction of the odd point 2k+1 from lambda_{k+j} uses -S~_j
        assert wv.dd_weights(N, exact=True) == {j: -s for j, s in printed[N].items()}
        assert sum(printed[N].values()) == -1


@pytest.mark.parametrize("N,Nt", WAVELETS)
def test_coarsening_ghost_points(N, Nt):
    """Coarse samples sit at the even positions 0, 2, .., NB-2 of the block and
    read H^a; the positions read outside [0, NB) are the ghost points."""
    ha = wv.table(N, Nt, exact=True)["Ha"]
    read = {p + o for p in range(0, NB, 2) for o in ha}
    front = max(0, -min(read))
    back = max(0, max(read) - (NB - 1))
    assert (front, back) == (REQ[(N, Nt)]["cf"], REQ[(N, Nt)]["cb"])


@pytest.mark.parametrize("N,Nt", WAVELETS)
def test_refinement_ghost_points(N, Nt):
    """A block of NB/2 coarse samples refines to NB fine points: fine position p
    reads the interleaved coefficients p+o of J^s (p even) or K^s (p odd); with
    zero details only the even ones (coarse samples q/2) are needed."""
    t = wv.table(N, Nt, exact=True)
    coarse = set()
    for p in range(NB):
        row = t["Js"] if p % 2 == 0 else t["Ks"]
        coarse |= {(p + o) // 2 for o, c in row.items() if (p + o) % 2 == 0 and c != 0}
    front = max(0, -min(coarse))
    back = max(0, max(coarse) - (NB // 2 - 1))
    assert (front, back) == (REQ[(N, Nt)]["rf"], REQ[(N, Nt)]["rb"])


@pytest.mark.parametrize("N,Nt", WAVELETS)
def test_coarse_region_extension_1d(N, Nt):
    """In 1D the fine points [0, NB) of a block next to a coarsened region are
    affected by the discarded details (odd interleaved positions) that their
    synthesis rows read; the farthest such position outside the block is the
    printed extension."""
    t = wv.table(N, Nt, exact=True)
    det = set()
    for p in range(NB):
        row = t["Js"] if p % 2 == 0 else t["Ks"]
        det |= {p + o for o, c in row.items() if (p + o) % 2 == 1 and c != 0}
    outside_front = [-q for q in det if q < 0]
    outside_back = [q - (NB - 1) for q in det if q >= NB]
    front = max(outside_front, default=0)
    back = max(outside_back, default=0)
    assert (front, back) == (REQ[(N, Nt)]["ef1"], REQ[(N, Nt)]["eb1"])


@pytest.mark.parametrize("N,Nt", WAVELETS)
def test_detail_band_is_3d_extension(N, Nt):
    r = REQ[(N, Nt)]
    assert og.DETAIL_EXT[(N, Nt)] == (r["ef3"], r["eb3"])
    # the update step needs the extension's coefficients at level L, i.e. 2e
    # fine points in front and 2e-1 behind (the back face ends on an odd point)
    for e, u in ((r["ef3"], r["uf3"]), (r["ef1"], r["uf1"])):
        assert u == 2 * e
    for e, u in ((r["eb3"], r["ub3"]), (r["eb1"], r["ub1"])):
        assert u == max(0, 2 * e - 1)
