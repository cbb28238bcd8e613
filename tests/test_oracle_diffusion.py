"""Pins of the oracle's diffusion right-hand side nu * laplacian(phi)
(DIFF-2 / DIFF-4 of the finite-difference supplement, and order 6).

* The stencils equal the central second-difference weights derived here in
  exact arithmetic from the Taylor conditions.
* One RK3 step of the heat equation on a uniform periodic grid equals the
  Fourier closed form R(z) = 1 + z + z^2/2 + z^3/6 with the stencils'
  symbols.
* Observed spatial orders 2, 4 and 6 against the analytic Laplacian.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import grid as og


def central_d2(order):
    """Weights w_o, o = -k..k (k = order / 2), with sum_o w_o o^m = 2 delta_m2
    for m = 0 .. 2k (exact), i.e. f'' to order `order` at unit spacing."""
    k = order // 2
    offs = list(range(-k, k + 1))
    n = len(offs)
    M = [[Fr(o) ** m for o in offs] + [Fr(2) if m == 2 else Fr(0)] for m in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return {o: M[i][n] / M[i][i] for i, o in enumerate(offs)}


@pytest.mark.parametrize("order", [2, 4, 6])
def test_stencils_are_the_central_second_differences(order):
    exact = central_d2(order)
    w = og.d2_weights(order)
    assert set(w) == set(exact)
    for o, c in exact.items():
        assert abs(w[o] - float(c)) <= 1e-15


def global_field(g, nb, L):
    W = nb << L
    out = np.zeros((W, W, W))
    for (l, i, j, k), a in g.blocks.items():
        out[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb] = a
    return out


@pytest.mark.parametrize("order", [2, 4, 6])
def test_rk3_heat_fourier_closed_form(order):
    nb, L, nu = 16, 1, 0.3
    g = og.Grid(nb, 4, 2, fd_order=order)
    g.uniform(L)
    rng = np.random.default_rng(order)
    for key in g.keys():
        g.blocks[key] = rng.standard_normal((nb, nb, nb))
    glob = global_field(g, nb, L)
    W = nb << L
    h = 1.0 / W
    dt = 0.1 * h * h / nu
    g.rk3_step(dt, ("diffusion", (nu,)))
    out = global_field(g, nb, L)
    th = 2 * np.pi * np.fft.fftfreq(W)
    sym = sum(float(c) * np.cos(o * th) for o, c in central_d2(order).items())
    sz, sy, sx = np.meshgrid(sym, sym, sym, indexing="ij")
    z = dt * nu * (sx + sy + sz) / (h * h)
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6
    ref = np.real(np.fft.ifftn(R * np.fft.fftn(glob)))
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("order", [2, 4, 6])
def test_diffusion_spatial_order(order):
    tp = 2 * np.pi
    f = lambda X, Y, Z: np.sin(tp * X) * np.sin(tp * Y + 0.3) * np.sin(tp * Z + 0.7)
    errs = []
    for L in (1, 2):
        g = og.Grid(8, 4, 0, fd_order=order)
        g.uniform(L)
        g.sample(f)
        err = 0.0
        for key in g.keys():
            r = g.rhs_block(key, ("diffusion", (0.5,)))
            x, y, z = g.positions(key)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            err = max(err, float(np.abs(r - 0.5 * (-3 * tp * tp) * f(X, Y, Z)).max()))
        errs.append(err)
    rate = np.log2(errs[0] / errs[1])
    assert order - 0.3 < rate < order + 0.6, (errs, rate)
