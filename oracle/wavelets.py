"""Interpolating-wavelet filter banks and 1D transforms (FP64 / exact rationals).

TEST INFRASTRUCTURE ONLY.  This module belongs to the CPU oracle: it may be
imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py`` -- never by the product path.

Source: Gillis & van Rees, "MURPHY" (arXiv 2112.07537).

* Filter tables: Supplementary section "Implementation details - filters bank",
  tables of non-lifted (2.0, 4.0, 6.0) and lifted (2.2, 4.2, 6.2) coefficients.
  They act on the interleaved layout u = [.. lambda_k, gamma_k, lambda_{k+1} ..].
  H^a and J^s are centred on even (scaling) positions, G^a and K^s on odd
  (detail) positions.
* Analysis (forward transform), section 2.1.2:
  lambda_k = sum_o H^a[o] f[2k+o],  gamma_k = sum_o G^a[o] f[2k+1+o].
* Synthesis in interleaved form (supplementary filter-bank section):
  f[2k] = sum_o J^s[o] u[2k+o],     f[2k+1] = sum_o K^s[o] u[2k+1+o].
* Dual-lifting coefficients S~ (table of dual-lifting coefficients, section
  2.1.4) are kept as an independent printed source used by the pins.
"""
from fractions import Fraction as Fr

import numpy as np

# ---------------------------------------------------------------------------
# Filter tables, transcribed from the two coefficient tables of the filter-bank
# supplement.  Each row is (first offset, list of coefficients).
# ---------------------------------------------------------------------------


def _row(first, coefs):
    return {first + i: Fr(c) for i, c in enumerate(coefs) if Fr(c) != 0}


_T = {}
# 2.0 (non-lifted, N=2)
_T[(2, 0)] = dict(
    Ha=_row(0, [1]),
    Ga=_row(-1, [Fr(-1, 2), 1, Fr(-1, 2)]),
    Js=_row(0, [1]),
    Ks=_row(-1, [Fr(1, 2), 1, Fr(1, 2)]),
)
# 4.0
_T[(4, 0)] = dict(
    Ha=_row(0, [1]),
    Ga=_row(-3, [Fr(1, 16), 0, Fr(-9, 16), 1, Fr(-9, 16), 0, Fr(1, 16)]),
    Js=_row(0, [1]),
    Ks=_row(-3, [Fr(-1, 16), 0, Fr(9, 16), 1, Fr(9, 16), 0, Fr(-1, 16)]),
)
# 6.0
_T[(6, 0)] = dict(
    Ha=_row(0, [1]),
    Ga=_row(-5, [Fr(-3, 256), 0, Fr(25, 256), 0, Fr(-75, 128), 1,
                 Fr(-75, 128), 0, Fr(25, 256), 0, Fr(-3, 256)]),
    Js=_row(0, [1]),
    Ks=_row(-5, [Fr(3, 256), 0, Fr(-25, 256), 0, Fr(75, 128), 1,
                 Fr(75, 128), 0, Fr(-25, 256), 0, Fr(3, 256)]),
)
# 2.2 (lifted, N=2, N~=2)
_T[(2, 2)] = dict(
    Ha=_row(-2, [Fr(-1, 8), Fr(1, 4), Fr(3, 4), Fr(1, 4), Fr(-1, 8)]),
    Ga=_row(-1, [Fr(-1, 2), 1, Fr(-1, 2)]),
    Js=_row(-1, [Fr(-1, 4), 1, Fr(-1, 4)]),
    Ks=_row(-2, [Fr(-1, 8), Fr(1, 2), Fr(3, 4), Fr(1, 2), Fr(-1, 8)]),
)
# 4.2
_T[(4, 2)] = dict(
    Ha=_row(-4, [Fr(1, 64), 0, Fr(-1, 8), Fr(1, 4), Fr(23, 32), Fr(1, 4),
                 Fr(-1, 8), 0, Fr(1, 64)]),
    Ga=_row(-3, [Fr(1, 16), 0, Fr(-9, 16), 1, Fr(-9, 16), 0, Fr(1, 16)]),
    Js=_row(-1, [Fr(-1, 4), 1, Fr(-1, 4)]),
    Ks=_row(-4, [Fr(1, 64), Fr(-1, 16), Fr(-1, 8), Fr(9, 16), Fr(23, 32),
                 Fr(9, 16), Fr(-1, 8), Fr(-1, 16), Fr(1, 64)]),
)
# 6.2
_T[(6, 2)] = dict(
    Ha=_row(-6, [Fr(-3, 1024), 0, Fr(11, 512), 0, Fr(-125, 1024), Fr(1, 4),
                 Fr(181, 256), Fr(1, 4), Fr(-125, 1024), 0, Fr(11, 512), 0,
                 Fr(-3, 1024)]),
    Ga=_row(-5, [Fr(-3, 256), 0, Fr(25, 256), 0, Fr(-75, 128), 1,
                 Fr(-75, 128), 0, Fr(25, 256), 0, Fr(-3, 256)]),
    Js=_row(-1, [Fr(-1, 4), 1, Fr(-1, 4)]),
    Ks=_row(-6, [Fr(-3, 1024), Fr(3, 256), Fr(11, 512), Fr(-25, 256),
                 Fr(-125, 1024), Fr(75, 128), Fr(181, 256), Fr(75, 128),
                 Fr(-125, 1024), Fr(-25, 256), Fr(11, 512), Fr(3, 256),
                 Fr(-3, 1024)]),
)

# Dual-lifting coefficients S~ (table of dual-lifting coefficients), indexed so
# that gamma_m <- gamma_m + sum_i S~_i lambda_{m+i}; symmetric S~_{-i}=S~_{i}
# about the detail (offsets 0 and 1 are the two nearest scaling coefficients).
DUAL_LIFT = {
    2: {0: Fr(-1, 2), 1: Fr(-1, 2)},
    4: {-1: Fr(1, 16), 0: Fr(-9, 16), 1: Fr(-9, 16), 2: Fr(1, 16)},
    6: {-2: Fr(-3, 256), -1: Fr(25, 256), 0: Fr(-75, 128), 1: Fr(-75, 128),
        2: Fr(25, 256), 3: Fr(-3, 256)},
}

WAVELETS = sorted(_T.keys())


def table(N, Nt, exact=False):
    """Return the filter bank {'Ha','Ga','Js','Ks'} as {offset: coef} dicts."""
    t = _T[(N, Nt)]
    if exact:
        return {k: dict(v) for k, v in t.items()}
    return {k: {o: float(c) for o, c in v.items()} for k, v in t.items()}


def reach(filt):
    """(min offset, max offset) of a filter dict."""
    return min(filt), max(filt)


# ---------------------------------------------------------------------------
# 1D transforms on an index window.  An array ``a`` along ``axis`` holds the
# values at global positions first, first+1, ...  Outputs are produced for the
# global positions [out_lo, out_hi).  All sums run over taps in increasing
# offset order.
# ---------------------------------------------------------------------------


def _apply(a, axis, first, out_lo, out_hi, even_filt, odd_filt):
    a = np.moveaxis(np.asarray(a), axis, -1)
    n_out = out_hi - out_lo
    out = np.zeros(a.shape[:-1] + (n_out,), dtype=np.result_type(a, np.float64))
    for p in range(out_lo, out_hi):
        filt = even_filt if p % 2 == 0 else odd_filt
        acc = np.zeros(a.shape[:-1], dtype=out.dtype)
        for o in sorted(filt):
            idx = p + o - first
            if idx < 0 or idx >= a.shape[-1]:
                raise IndexError(f"filter reach leaves the window at {p}+{o}")
            acc = acc + filt[o] * a[..., idx]
        out[..., p - out_lo] = acc
    return np.moveaxis(out, -1, axis)


def analysis(a, axis, first, out_lo, out_hi, N, Nt):
    """Forward transform along ``axis``: H^a at even, G^a at odd positions.
    Interleaved output (lambda at even, gamma at odd positions)."""
    t = table(N, Nt)
    return _apply(a, axis, first, out_lo, out_hi, t["Ha"], t["Ga"])


def synthesis(u, axis, first, out_lo, out_hi, N, Nt):
    """Inverse transform along ``axis`` from interleaved coefficients:
    J^s at even, K^s at odd positions."""
    t = table(N, Nt)
    return _apply(u, axis, first, out_lo, out_hi, t["Js"], t["Ks"])


def analysis_periodic(f, N, Nt, exact=False):
    """Periodic 1D forward transform of a 1D list/array of even length."""
    t = table(N, Nt, exact)
    n = len(f)
    out = [None] * n
    for p in range(n):
        filt = t["Ha"] if p % 2 == 0 else t["Ga"]
        acc = Fr(0) if exact else 0.0
        for o in sorted(filt):
            acc += filt[o] * f[(p + o) % n]
        out[p] = acc
    return out


def synthesis_periodic(u, N, Nt, exact=False):
    """Periodic 1D inverse transform of interleaved coefficients."""
    t = table(N, Nt, exact)
    n = len(u)
    out = [None] * n
    for p in range(n):
        filt = t["Js"] if p % 2 == 0 else t["Ks"]
        acc = Fr(0) if exact else 0.0
        for o in sorted(filt):
            acc += filt[o] * u[(p + o) % n]
        out[p] = acc
    return out


def refine_1d(coarse, axis, cfirst, out_lo, out_hi, N, Nt):
    """Zero-detail refinement along ``axis`` (section 2.2.2: all unknown details
    taken as zero).  ``coarse`` holds scaling coefficients at coarse indices
    cfirst, cfirst+1, ...; the result holds fine values at fine positions
    [out_lo, out_hi).  Implemented literally as the interleaved synthesis of
    [lambda, 0, lambda, 0, ...]."""
    c = np.moveaxis(np.asarray(coarse, dtype=np.float64), axis, -1)
    m = c.shape[-1]
    u = np.zeros(c.shape[:-1] + (2 * m,), dtype=np.float64)
    u[..., 0::2] = c
    # u holds interleaved coefficients at fine positions 2*cfirst ...
    out = synthesis(u, -1, 2 * cfirst, out_lo, out_hi, N, Nt)
    return np.moveaxis(out, -1, axis)


def dd_weights(N, exact=False):
    """Deslauriers-Dubuc prediction weights of order N read from the K^s row at
    the scaling positions: odd fine value = sum_j w[j] lambda_{k+j}, j in
    [1-N/2, N/2], for the odd position 2k+1."""
    t = table(N, 0, exact)["Ks"]
    # K^s offset o (odd) reads position 2k+1+o = 2(k + (o+1)/2).
    return {(o + 1) // 2: c for o, c in t.items() if o % 2 != 0}
