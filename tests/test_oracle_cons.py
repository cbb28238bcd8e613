"""Pins of the oracle's conservative CONS-3 / CONS-5 right-hand side (finite-
difference supplement, tables of the order-3 and order-5 WENO stencils).

* The fixed-weight fluxes equal the upwind-biased conservative flux of
  Shu's finite-difference reconstruction, derived here independently: the
  coefficients c_o that reproduce the interface value x_{i+1/2} of every
  polynomial of degree < k from its cell averages over the cells i+o
  (k = 3 or 5; offsets -1..1 / -2..2 for f^+, mirrored for f^-).
* One RK3 step on a uniform periodic grid with a constant velocity of mixed
  signs equals the Fourier closed form R(z) = 1 + z + z^2/2 + z^3/6 with the
  upwind symbols of those derived fluxes.
* Observed spatial orders 3 and 5 on smooth periodic data.
* Conservation: on a uniform periodic grid the fluxes telescope, so the RHS
  sums to zero.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import grid as og


def shu_flux(k, offsets):
    """Coefficients c_o (exact) with sum_o c_o * avg_{cell i+o}(p) =
    p(x_{i+1/2}) for all polynomials p of degree < k (unit spacing, cell j =
    [j - 1/2, j + 1/2], interface x_{i+1/2} = 1/2 with i = 0)."""
    n = len(offsets)
    assert n == k
    A = [[Fr(0)] * n for _ in range(k)]
    b = [Fr(0)] * k
    for m in range(k):                       # monomial x^m
        for c, o in enumerate(offsets):
            lo, hi = Fr(2 * o - 1, 2), Fr(2 * o + 1, 2)
            A[m][c] = (hi ** (m + 1) - lo ** (m + 1)) / (m + 1)
        b[m] = Fr(1, 2) ** m
    # Gaussian elimination in exact arithmetic
    M = [row[:] + [b[r]] for r, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return {o: M[i][n] / M[i][i] for i, o in enumerate(offsets)}


UPWIND = {3: (-1, 0, 1), 5: (-2, -1, 0, 1, 2)}


@pytest.mark.parametrize("k", [3, 5])
def test_fluxes_are_the_upwind_reconstruction(k):
    plus, minus = og.cons_fluxes(k, exact=True)
    assert plus == shu_flux(k, UPWIND[k])
    # f^- at i+1/2 is biased to the right: cells i+1-o for the mirrored offsets
    assert minus == shu_flux(k, tuple(1 - o for o in reversed(UPWIND[k])))


def symbol(coef, th):
    """Symbol of D phi_i = F_{i+1/2} - F_{i-1/2}, F = sum c_o phi_{i+o}."""
    return sum(float(c) * (np.exp(1j * o * th) - np.exp(1j * (o - 1) * th)) for o, c in coef.items())


def global_field(g, nb, L):
    W = nb << L
    out = np.zeros((W, W, W))
    for (l, i, j, k), a in g.blocks.items():
        out[k * nb:(k + 1) * nb, j * nb:(j + 1) * nb, i * nb:(i + 1) * nb] = a
    return out


@pytest.mark.parametrize("k", [3, 5])
def test_rk3_fourier_closed_form(k):
    nb, L = 16, 1
    g = og.Grid(nb, 4, 0, fd_order=k)
    g.uniform(L)
    ic = lambda X, Y, Z: np.exp(-((X - .5) ** 2 + (Y - .45) ** 2 + (Z - .55) ** 2) / 0.1 ** 2)
    g.sample(ic)
    glob = global_field(g, nb, L)
    u = (1.0, -0.5, 0.25)
    W = nb << L
    h = 1.0 / W
    dt = 0.5 * h / sum(abs(v) for v in u)
    g.rk3_step(dt, ("const", u))
    out = global_field(g, nb, L)
    th = 2 * np.pi * np.fft.fftfreq(W)
    sp = symbol(shu_flux(k, UPWIND[k]), th)
    sm = symbol(shu_flux(k, tuple(1 - o for o in reversed(UPWIND[k]))), th)
    s = [sp if v > 0 else sm for v in u]
    sz, sy, sx = np.meshgrid(s[2], s[1], s[0], indexing="ij")
    z = -dt * (u[0] * sx + u[1] * sy + u[2] * sz) / h
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6
    ref = np.real(np.fft.ifftn(R * np.fft.fftn(glob)))
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()
    # the upwind scheme damps: |R| < 1 at the highest frequency
    assert np.abs(R).min() < 0.999


@pytest.mark.parametrize("k", [3, 5])
def test_spatial_order(k):
    tp = 2 * np.pi
    f = lambda X, Y, Z: np.sin(tp * X) * np.sin(tp * Y + 0.3) * np.sin(tp * Z + 0.7)
    errs = []
    for L in (1, 2):
        g = og.Grid(8, 4, 0, fd_order=k)
        g.uniform(L)
        g.sample(f)
        u = ("rotating", (0.5, 0.5, 0.2))       # both signs along x and y
        err = 0.0
        for key in g.keys():
            r = g.rhs_block(key, u)
            x, y, z = g.positions(key)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            ux, uy, uz = -(Y - 0.5), X - 0.5, 0.2
            fx = tp * np.cos(tp * X) * np.sin(tp * Y + 0.3) * np.sin(tp * Z + 0.7)
            fy = tp * np.sin(tp * X) * np.cos(tp * Y + 0.3) * np.sin(tp * Z + 0.7)
            fz = tp * np.sin(tp * X) * np.sin(tp * Y + 0.3) * np.cos(tp * Z + 0.7)
            err = max(err, float(np.abs(r + ux * fx + uy * fy + uz * fz).max()))
        errs.append(err)
    order = np.log2(errs[0] / errs[1])
    assert k - 0.4 < order < k + 1.0, (errs, order)


@pytest.mark.parametrize("k", [3, 5])
def test_conservation_on_a_uniform_grid(k):
    g = og.Grid(8, 4, 0, fd_order=k)
    g.uniform(1)
    rng = np.random.default_rng(k)
    for key in g.keys():
        g.blocks[key] = rng.standard_normal((8, 8, 8))
    tot = sum(float(g.rhs_block(key, ("shear", ())).sum()) for key in g.keys())
    scale = sum(float(np.abs(g.rhs_block(key, ("shear", ()))).sum()) for key in g.keys())
    assert abs(tot) <= 1e-12 * scale
