"""Pins of the oracle's filter banks against what the paper fixes independently.

* The lifting scheme of section 2.1.4 (split, dual lift with the printed S~ of
  the dual-lifting table, primal lift S = -1/2 S~ of the two-point rule) must
  reproduce every printed H^a, G^a, J^s, K^s row exactly (exact rationals).
* Perfect reconstruction, polynomial annihilation of order N, conservation of
  the first N~ moments (moment-conservation identity of section 2.1.4).
* The 2.2 worked ghost example of section 2.2.2.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import wavelets as wv

NP = 64  # periodic length used for impulse responses


def lifting_analysis(f, N, Nt):
    """Forward transform by the three lifting steps (section 2.1.4)."""
    n = len(f) // 2
    lam = [f[2 * k] for k in range(n)]
    gam = [f[2 * k + 1] for k in range(n)]
    St = wv.DUAL_LIFT[N]
    gam = [gam[m] + sum(St[i] * lam[(m + i) % n] for i in sorted(St))
           for m in range(n)]
    if Nt == 2:
        S = -Fr(1, 2) * wv.DUAL_LIFT[2][0]   # S = -1/2 S~ (two-point rule) = 1/4
        lam = [lam[k] + S * (gam[(k - 1) % n] + gam[k]) for k in range(n)]
    out = [None] * (2 * n)
    out[0::2] = lam
    out[1::2] = gam
    return out


def lifting_synthesis(u, N, Nt):
    n = len(u) // 2
    lam = list(u[0::2])
    gam = list(u[1::2])
    if Nt == 2:
        S = -Fr(1, 2) * wv.DUAL_LIFT[2][0]
        lam = [lam[k] - S * (gam[(k - 1) % n] + gam[k]) for k in range(n)]
    St = wv.DUAL_LIFT[N]
    gam = [gam[m] - sum(St[i] * lam[(m + i) % n] for i in sorted(St))
           for m in range(n)]
    out = [None] * (2 * n)
    out[0::2] = lam
    out[1::2] = gam
    return out


def impulse_rows(transform, N, Nt):
    """Read filter rows centred at position 2*c (even) and 2*c+1 (odd)."""
    c = NP // 4
    even, odd = {}, {}
    for j in range(NP):
        e = [Fr(0)] * NP
        e[j] = Fr(1)
        out = transform(e, N, Nt)
        if out[2 * c] != 0:
            even[j - 2 * c] = out[2 * c]
        if out[2 * c + 1] != 0:
            odd[j - 2 * c - 1] = out[2 * c + 1]
    return even, odd


def synthesis_rows(N, Nt):
    """J^s / K^s rows: f[p] = sum_o row[o] u[p+o]; read from the synthesis of
    coefficient impulses."""
    c = NP // 4
    even, odd = {}, {}
    for j in range(NP):
        e = [Fr(0)] * NP
        e[j] = Fr(1)
        out = lifting_synthesis(e, N, Nt)
        if out[2 * c] != 0:
            even[j - 2 * c] = out[2 * c]
        if out[2 * c + 1] != 0:
            odd[j - 2 * c - 1] = out[2 * c + 1]
    return even, odd


@pytest.mark.parametrize("N,Nt", wv.WAVELETS)
def test_tables_match_lifting_scheme(N, Nt):
    t = wv.table(N, Nt, exact=True)
    Ha, Ga = impulse_rows(lifting_analysis, N, Nt)
    Js, Ks = synthesis_rows(N, Nt)
    assert t["Ha"] == Ha
    assert t["Ga"] == Ga
    assert t["Js"] == Js
    assert t["Ks"] == Ks


@pytest.mark.parametrize("N", [2, 4, 6])
def test_dd_weights_are_negated_dual_lifting(N):
    w = wv.dd_weights(N, exact=True)
    St = wv.DUAL_LIFT[N]
    assert w == {j: -c for j, c in St.items()}
    assert sum(w.values()) == 1


@pytest.mark.parametrize("N,Nt", wv.WAVELETS)
def test_perfect_reconstruction_exact(N, Nt):
    rng = np.random.default_rng(7)
    f = [Fr(int(v), 97) for v in rng.integers(-1000, 1000, size=48)]
    u = wv.analysis_periodic(f, N, Nt, exact=True)
    assert wv.synthesis_periodic(u, N, Nt, exact=True) == f


@pytest.mark.parametrize("N,Nt", wv.WAVELETS)
def test_details_annihilate_polynomials_below_N(N, Nt):
    # on a long window (no wrap inside the support), degree < N -> gamma = 0
    t = wv.table(N, Nt, exact=True)
    for deg in range(N + 1):
        vals = {p: Fr(p) ** deg for p in range(-20, 21)}
        g = sum(c * vals[1 + o] for o, c in t["Ga"].items())
        if deg < N:
            assert g == 0
        else:
            assert g != 0


@pytest.mark.parametrize("N,Nt", wv.WAVELETS)
def test_moment_conservation(N, Nt):
    """sum_j f_j x_j^p = 2 sum_k lambda_k x_k^p for p < N~ (moment identity of
    section 2.1.4), on a compactly supported signal."""
    t = wv.table(N, Nt, exact=True)
    rng = np.random.default_rng(3)
    n = 60
    f = [Fr(0)] * 20 + [Fr(int(v), 13) for v in rng.integers(-50, 50, size=20)] + [Fr(0)] * 20
    lam = {}
    for k in range(3, n // 2 - 3):
        lam[k] = sum(c * f[2 * k + o] for o, c in t["Ha"].items())
    for p in range(3):
        fine = sum(f[j] * Fr(j, 2) ** p for j in range(n))      # x_{L+1,j} = j/2
        coarse = 2 * sum(lam[k] * Fr(k) ** p for k in lam)     # x_{L,k} = k
        if p < Nt:
            assert fine == coarse
        else:
            assert fine != coarse


def test_worked_example_2_2_ghosts():
    """Section 2.2.2, wavelet 2.2: with the details across the jump taken as
    zero, lambda^1_10 = lambda^0_5, lambda^1_11 = (lambda^0_5 + lambda^0_6)/2
    and lambda^1_3 = (lambda^0_1 + lambda^0_2)/2."""
    lam0 = np.array([0.3, -1.2, 2.5, 0.7, 1.9, -0.4, 3.3, 0.05, -2.0])
    fine = wv.refine_1d(lam0[None, :], 1, 0, 2, 16, 2, 2)[0]   # positions 2..15
    assert fine[10 - 2] == lam0[5]
    assert fine[11 - 2] == 0.5 * (lam0[5] + lam0[6])
    assert fine[3 - 2] == 0.5 * (lam0[1] + lam0[2])


@pytest.mark.parametrize("N", [2, 4, 6])
def test_refinement_identical_for_lifted_and_unlifted(N):
    lam0 = np.sin(np.arange(20) * 0.7)
    a = wv.refine_1d(lam0[None, :], 1, 0, 2 * N, 40 - 2 * N, N, 0)
    b = wv.refine_1d(lam0[None, :], 1, 0, 2 * N, 40 - 2 * N, N, 2)
    assert np.array_equal(a, b)
