"""Brute-force global formulation of the ghost reconstruction on tiny periodic
trees with two levels (used only by tests; independent of ``oracle/``).

On a tree whose leaves sit at levels Lf-1 and Lf only, every level-(Lf-1)
point is held by some leaf, so the whole coarse sample array exists globally.
The coarse-extension assumption of section 2.2.2 then says the fine-level view
of the coarse region is the global Deslauriers-Dubuc refinement G of that
array.  Weights are derived here from Lagrange interpolation at the midpoint
(section 2.1.3, interpolating wavelets), not read from the paper's tables; the
lifted restriction H^a is built from the lifting steps with S = 1/4.
"""
from fractions import Fraction as Fr

import numpy as np


def lagrange_midpoint_weights(N):
    """Weights w_j, j in [1-N/2, N/2], of the degree-(N-1) interpolant of the
    nodes j evaluated at 1/2 (exact rationals)."""
    nodes = list(range(1 - N // 2, N // 2 + 1))
    w = {}
    for j in nodes:
        num, den = Fr(1), Fr(1)
        for m in nodes:
            if m != j:
                num *= Fr(1, 2) - m
                den *= j - m
        w[j] = num / den
    return w


def refine_axis(S, axis, N):
    """Periodic zero-detail refinement of S along ``axis`` (length doubles)."""
    w = lagrange_midpoint_weights(N)
    S = np.moveaxis(S, axis, 0)
    out = np.empty((2 * S.shape[0],) + S.shape[1:])
    out[0::2] = S
    odd = np.zeros(S.shape)
    for j in sorted(w):
        odd = odd + float(w[j]) * np.roll(S, -j, axis=0)
    out[1::2] = odd
    return np.moveaxis(out, 0, axis)


def restriction_taps(N, Nt):
    """Impulse response of lambda_k as a function of the fine values f_{2k+o},
    from the lifting steps of section 2.1.4 with the Lagrange dual lift."""
    if Nt == 0:
        return {0: Fr(1)}
    w = lagrange_midpoint_weights(N)
    taps = {0: Fr(1)}
    # gamma_m = f_{2m+1} - sum_j w_j f_{2(m+j)};  lambda_k += 1/4 (gamma_{k-1}+gamma_k)
    for m in (-1, 0):
        taps[2 * m + 1] = taps.get(2 * m + 1, 0) + Fr(1, 4)
        for j, c in w.items():
            o = 2 * (m + j)
            taps[o] = taps.get(o, 0) - Fr(1, 4) * c
    return {o: c for o, c in taps.items() if c != 0}


def restrict_axis(F, axis, N, Nt):
    taps = restriction_taps(N, Nt)
    F = np.moveaxis(F, axis, 0)
    acc = np.zeros(F.shape)
    for o in sorted(taps):
        acc = acc + float(taps[o]) * np.roll(F, -o, axis=0)
    return np.moveaxis(acc[0::2], 0, axis)


class TwoLevel:
    """Global arrays of a two-level periodic tree (levels Lf-1 and Lf)."""

    def __init__(self, nb, Lf, blocks):
        self.nb, self.Lf = nb, Lf
        self.blocks = blocks
        W = nb << Lf
        self.fine_mask = np.zeros((W, W, W), bool)
        self.fine = np.zeros((W, W, W))
        self.coarse = np.zeros((W // 2,) * 3)
        for (L, i, j, k), a in blocks.items():
            if L == Lf:
                sl = (slice(k * nb, (k + 1) * nb), slice(j * nb, (j + 1) * nb),
                      slice(i * nb, (i + 1) * nb))
                self.fine[sl] = a
                self.fine_mask[sl] = True
                self.coarse[k * nb // 2:(k + 1) * nb // 2, j * nb // 2:(j + 1) * nb // 2,
                            i * nb // 2:(i + 1) * nb // 2] = a[0::2, 0::2, 0::2]
            elif L == Lf - 1:
                self.coarse[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb,
                            i * nb:(i + 1) * nb] = a
            else:
                raise ValueError("two levels only")

    def refined(self, N):
        G = self.coarse
        for ax in (2, 1, 0):
            G = refine_axis(G, ax, N)
        return G

    def coarse_view(self, N, Nt):
        """Level-(Lf-1) view: restriction of G' = fine values on fine leaves,
        G elsewhere."""
        G = np.where(self.fine_mask, self.fine, self.refined(N))
        for ax in (2, 1, 0):
            G = restrict_axis(G, ax, N, Nt)
        return G


def analysis_global(f, N, Nt):
    """Periodic 3D forward transform (x, then y, then z) by lifting steps:
    predict with the Lagrange weights, then (lifted) update with S = 1/4."""
    w = lagrange_midpoint_weights(N)
    out = f
    for axis in (2, 1, 0):
        a = np.moveaxis(out, axis, 0)
        lam = a[0::2].copy()
        gam = a[1::2].copy()
        for j in sorted(w):
            gam = gam - float(w[j]) * np.roll(lam, -j, axis=0)
        if Nt == 2:
            lam = lam + 0.25 * (np.roll(gam, 1, axis=0) + gam)
        r = np.empty_like(a)
        r[0::2] = lam
        r[1::2] = gam
        out = np.moveaxis(r, 0, axis)
    return out


def synthesis_global(u, N, Nt):
    """Inverse of analysis_global (z, then y, then x), undoing the steps."""
    w = lagrange_midpoint_weights(N)
    out = u
    for axis in (0, 1, 2):
        a = np.moveaxis(out, axis, 0)
        lam = a[0::2].copy()
        gam = a[1::2].copy()
        if Nt == 2:
            lam = lam - 0.25 * (np.roll(gam, 1, axis=0) + gam)
        odd = gam.copy()
        for j in sorted(w):
            odd = odd + float(w[j]) * np.roll(lam, -j, axis=0)
        r = np.empty_like(a)
        r[0::2] = lam
        r[1::2] = odd
        out = np.moveaxis(r, 0, axis)
    return out


def level_field(tl, N):
    """Global level-Lf field of a two-level tree: the fine leaves' values
    where a fine leaf holds the point, the refinement G elsewhere."""
    return np.where(tl.fine_mask, tl.fine, tl.refined(N))


def point_details(f, N):
    """Detail of every point of a periodic level field with respect to the
    interpolating prediction, over the point's odd axes only: along x, then
    y, then z, odd positions take value minus the Lagrange prediction from
    the even positions of the running array (the all-even points keep their
    value).  Degree-k points thus get the tensor product of the k 1D
    predict-and-subtract filters, the quantity the substitution zeroes."""
    w = lagrange_midpoint_weights(N)
    out = f.copy()
    for axis in (2, 1, 0):
        a = np.moveaxis(out, axis, 0)
        ev = a[0::2]
        pred = np.zeros(ev.shape)
        for j in sorted(w):
            pred = pred + float(w[j]) * np.roll(ev, -j, axis=0)
        r = a.copy()
        r[1::2] = a[1::2] - pred
        out = np.moveaxis(r, 0, axis)
    return out


def lifted_coarse(f, N, Nt):
    """Level-(Lf-1) scaling coefficients [H^a]^3 f of a periodic level field."""
    out = f
    for ax in (2, 1, 0):
        out = restrict_axis(out, ax, N, Nt)
    return out
