"""Plain FP64 oracle of the block-octree multiresolution method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP path; both sides read the same seeded inputs only.

Source: Gillis & van Rees, "MURPHY" (arXiv 2112.07537).  Each function names
the passage it follows.  Where a passage is silent or ambiguous, the reading
taken is marked READING at the place it is used.

Geometry (READING, node-based left-aligned points): periodic unit cube, one
tree, root level 0.  Leaf (L, i, j, k) holds nb^3 points; local point (x,y,z)
sits at ((i*nb+x), (j*nb+y), (k*nb+z)) / (nb*2^L).  Even local indices coincide
with level L-1 points.  Arrays are indexed [z, y, x] (x fastest in memory).

The central object is the *level view* Phi_L(P): the field as seen at level L
at a level-L grid point P, which is what the ghost reconstruction of section
2.2.2 and the supplementary ghosting algorithms (Part 1 and Part 2) produce:
  * leaf holding P at level L            -> its value (same-level copy);
  * leaf holding P is coarser            -> G_L(P), the zero-detail refinement
    (coarse-extension assumption, section 2.2.2) of the level-(L-1) samples,
    each sample being the value of the leaf holding that coarse point
    (the "Sample" of Part 1; injection when that leaf is finer).  READING
    R-ORDER: the samples are the values from before the substitution of the
    current reconstruction (Part 1 refines the coarse data before Part 2
    overwrites anything);
  * leaf holding P is finer (one level)  -> [H^a x H^a x H^a] restriction of
    Phi_{L+1} (coarsening of the fine data incl. its ghosts, Part 2);
    inside that restriction, points held by an even finer leaf are injected
    (READING: one restriction level).  For N.0 H^a is the identity, so this is
    plain injection.
"""
from fractions import Fraction as Fr

import numpy as np

from . import wavelets as wv

DIRS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
        for dx in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]

FINER, SAME, COARSER = 1, 0, -1


def fd_weights(order):
    """Central first-derivative weights {offset: w} (times 1/h)."""
    if order == 2:
        return {-1: -0.5, 1: 0.5}
    if order == 4:
        return {-2: 1.0 / 12, -1: -8.0 / 12, 1: 8.0 / 12, 2: -1.0 / 12}
    if order == 6:
        return {-3: -1.0 / 60, -2: 9.0 / 60, -1: -45.0 / 60,
                1: 45.0 / 60, 2: -9.0 / 60, 3: 1.0 / 60}
    raise ValueError(order)


def d2_weights(order):
    """Central second-derivative weights {offset: w} (times 1/h^2) of order
    2, 4 and 6: the DIFF-2 / DIFF-4 Laplacian stencils of the
    finite-difference supplement and their sixth-order sibling."""
    if order == 2:
        return {-1: 1.0, 0: -2.0, 1: 1.0}
    if order == 4:
        return {-2: -1.0 / 12, -1: 16.0 / 12, 0: -30.0 / 12, 1: 16.0 / 12, 2: -1.0 / 12}
    if order == 6:
        return {-3: 2.0 / 180, -2: -27.0 / 180, -1: 270.0 / 180, 0: -490.0 / 180,
                1: 270.0 / 180, 2: -27.0 / 180, 3: 2.0 / 180}
    raise ValueError(order)


# Stencils and ideal weights of the fixed-weight WENO fluxes (tables of the
# finite-difference supplement, WENO order 3 and order 5): for f^+ at the
# interface i+1/2 and for f^- at i-1/2, each candidate stencil S_r as
# {offset from i: coefficient} with its ideal weight gamma_r.
_WENO = {
    3: dict(plus=[({-1: Fr(-1, 2), 0: Fr(3, 2)}, Fr(1, 3)),
                  ({0: Fr(1, 2), 1: Fr(1, 2)}, Fr(2, 3))],
            minus=[({-1: Fr(1, 2), 0: Fr(1, 2)}, Fr(2, 3)),
                   ({0: Fr(3, 2), 1: Fr(-1, 2)}, Fr(1, 3))]),
    5: dict(plus=[({-2: Fr(1, 3), -1: Fr(-7, 6), 0: Fr(11, 6)}, Fr(1, 10)),
                  ({-1: Fr(-1, 6), 0: Fr(5, 6), 1: Fr(1, 3)}, Fr(3, 5)),
                  ({0: Fr(1, 3), 1: Fr(5, 6), 2: Fr(-1, 6)}, Fr(3, 10))],
            minus=[({-2: Fr(-1, 6), -1: Fr(5, 6), 0: Fr(1, 3)}, Fr(3, 10)),
                   ({-1: Fr(1, 3), 0: Fr(5, 6), 1: Fr(-1, 6)}, Fr(3, 5)),
                   ({0: Fr(11, 6), 1: Fr(-7, 6), 2: Fr(1, 3)}, Fr(1, 10))]),
}


def cons_fluxes(order, exact=False):
    """CONS-3 / CONS-5 (finite-difference supplement): the fixed-weight WENO
    interface fluxes, sum_r gamma_r S_r.  Returns (plus, minus) as
    {offset: coefficient} for the flux at the interface i+1/2 built from the
    values f_{i+offset}: plus is f^+_{i+1/2}, minus is f^-_{i+1/2} (the
    tabulated f^-_{i-1/2} shifted by one point)."""
    t = _WENO[order]
    plus, minus = {}, {}
    for st, gm in t["plus"]:
        for o, c in st.items():
            plus[o] = plus.get(o, 0) + gm * c
    for st, gm in t["minus"]:
        for o, c in st.items():
            minus[o + 1] = minus.get(o + 1, 0) + gm * c
    if not exact:
        plus = {o: float(c) for o, c in plus.items()}
        minus = {o: float(c) for o, c in minus.items()}
    return plus, minus


def stencil_depth(order):
    """Ghost points a block's RHS reads: FD2 one, FD4 and CONS-3 two, FD6
    and CONS-5 three."""
    return {2: 1, 3: 2, 4: 2, 5: 3, 6: 3}[order]


def transform_reach(N, Nt):
    """Ghost depth (front, back) needed by the block forward transform over
    local positions [0, nb): H^a at even and G^a at odd positions."""
    t = wv.table(N, Nt)
    h = max(-min(t["Ha"]), max(t["Ha"]))
    g = max(t["Ga"])
    return max(h, g - 1), max(h - 1, g)


# Table 3 of section 2.2.5, 3D values of the "coarse region extension" column,
# in interleaved (fine-level) index units (READING R-EXT; unit fixed by the 1D
# 2.2 example of section 2.2.1: one coefficient in front, two behind).
DETAIL_EXT = {(2, 0): (0, 1), (2, 2): (1, 2), (4, 0): (2, 3),
              (4, 2): (3, 4), (6, 0): (4, 5), (6, 2): (5, 6)}


class Grid:
    """Periodic octree of nb^3 blocks with one scalar field (FP64)."""

    def __init__(self, nb, N, Nt, fd_order=4, level_min=0, level_max=12,
                 eps_refine=1e-2, eps_coarsen=1e-4, detail_ext=1):
        assert nb % 2 == 0 and nb >= 8
        self.nb, self.N, self.Nt = nb, N, Nt
        self.fd_order = fd_order
        self.level_min, self.level_max = level_min, level_max
        self.eps_r, self.eps_c = eps_refine, eps_coarsen
        self.detail_ext = detail_ext
        self._pre = None          # field before the last substitution (R-ORDER)
        self.blocks = {}          # (L, i, j, k) -> float64 array [z, y, x]
        self._index()

    @property
    def blocks(self):
        return self._blocks

    @blocks.setter
    def blocks(self, value):
        # a new field: the samples of G_L are read from it again
        self._blocks = value
        self._pre = None

    # ------------------------------------------------------------------ tree
    def _index(self):
        self._keys = {}
        for (L, i, j, k) in self.blocks:
            self._keys.setdefault(L, []).append((i + (j << 21) + (k << 42)))
        self._keys = {L: np.array(sorted(v), dtype=np.int64)
                      for L, v in self._keys.items()}

    def set_tree(self, keys, init=None):
        nb = self.nb
        self.blocks = {tuple(int(v) for v in k): (
            np.zeros((nb, nb, nb)) if init is None else init(k)) for k in keys}
        self._index()

    def uniform(self, L):
        n = 1 << L
        self.set_tree([(L, i, j, k) for k in range(n) for j in range(n)
                       for i in range(n)])

    def levels(self):
        return sorted(self._keys)

    def width(self, L):
        return self.nb << L

    def origin(self, key):
        L, i, j, k = key
        return np.array([i * self.nb, j * self.nb, k * self.nb])

    def owner_level(self, L, X, Y, Z):
        """Level of the leaf holding each level-L point (arrays, any int)."""
        W = self.width(L)
        X, Y, Z = X % W, Y % W, Z % W
        lev = np.full(np.shape(X), -1, dtype=np.int64)
        for l in self.levels():
            if l <= L:
                s = L - l
                bx, by, bz = (X >> s) // self.nb, (Y >> s) // self.nb, (Z >> s) // self.nb
            else:
                s = l - L
                bx, by, bz = (X << s) // self.nb, (Y << s) // self.nb, (Z << s) // self.nb
            code = bx + (by << 21) + (bz << 42)
            ks = self._keys[l]                     # sorted codes of level l
            pos = np.minimum(np.searchsorted(ks, code), len(ks) - 1)
            lev[ks[pos] == code] = l
        assert (lev >= 0).all(), "point outside every leaf"
        return lev

    def values_at(self, l, L, X, Y, Z, src=None):
        """Values of the level-l leaves at level-L points P (l >= L, or P on
        the level-l grid).  P must lie in level-l leaves.  ``src`` is the
        block dict read (default: the current field)."""
        src = self.blocks if src is None else src
        W = self.width(L)
        X, Y, Z = X % W, Y % W, Z % W
        if l >= L:
            s = l - L
            Xl, Yl, Zl = X << s, Y << s, Z << s
        else:
            s = L - l
            assert ((X % (1 << s)) == 0).all() and ((Y % (1 << s)) == 0).all() \
                and ((Z % (1 << s)) == 0).all()
            Xl, Yl, Zl = X >> s, Y >> s, Z >> s
        nb = self.nb
        bx, by, bz = Xl // nb, Yl // nb, Zl // nb
        out = np.empty(np.shape(X))
        code = bx + (by << 21) + (bz << 42)
        for c in np.unique(code):
            m = code == c
            key = (l, int(c & ((1 << 21) - 1)), int((c >> 21) & ((1 << 21) - 1)),
                   int(c >> 42))
            a = src[key]
            out[m] = a[Zl[m] % nb, Yl[m] % nb, Xl[m] % nb]
        return out

    # ---------------------------------------------------------- level views
    @staticmethod
    def _box(lo, shape):
        z, y, x = np.meshgrid(np.arange(lo[2], lo[2] + shape[2]),
                              np.arange(lo[1], lo[1] + shape[1]),
                              np.arange(lo[0], lo[0] + shape[0]), indexing="ij")
        return x, y, z

    def sample_box(self, L, lo, shape):
        """Level-L samples used as coarse data by a refinement (Part 1
        "Sample"): the value of the leaf holding each point, by injection when
        that leaf is at level L or finer; G_L when it is coarser.  Values are
        those from before the last substitution (READING R-ORDER); the
        substitution never changes a point that a finer level samples (it
        keeps every all-even point), so only coarser leaves' values differ."""
        X, Y, Z = self._box(lo, shape)
        lev = self.owner_level(L, X, Y, Z)
        out = np.empty(X.shape)
        src = self._pre if self._pre is not None else self.blocks
        for l in np.unique(lev):
            m = lev == l
            if l >= L:
                out[m] = self.values_at(int(l), L, X[m], Y[m], Z[m], src)
        if (lev < L).any():
            G = self.refine_box(L, lo, shape)
            out[lev < L] = G[lev < L]
        return out

    def refine_box(self, L, lo, shape):
        """G_L over a box of level-L points: zero-detail refinement (inverse
        transform with all unknown details zero, section 2.2.2 / 2.2.3), applied
        along x, then y, then z, to the level-(L-1) samples."""
        N = self.N
        lo = np.asarray(lo)
        hi = lo + np.asarray(shape)
        clo = lo // 2 - N // 2
        chi = (hi - 1) // 2 + N // 2 + 1
        S = self.sample_box(L - 1, clo, chi - clo)
        # arrays are [z, y, x]: x is axis 2
        T = wv.refine_1d(S, 2, clo[0], lo[0], hi[0], N, self.Nt)
        T = wv.refine_1d(T, 1, clo[1], lo[1], hi[1], N, self.Nt)
        T = wv.refine_1d(T, 0, clo[2], lo[2], hi[2], N, self.Nt)
        return T

    def restrict_box(self, L, lo, shape):
        """[H^a]^3 restriction of Phi_{L+1} at the level-L points of a box
        (coarsening of section 2.2.1 / 2.3), with points held by leaves finer
        than L+1 injected."""
        Ha = wv.table(self.N, self.Nt)["Ha"]
        h = max(Ha)
        lo = np.asarray(lo)
        shape = np.asarray(shape)
        flo = 2 * lo - h
        fshape = 2 * (shape - 1) + 1 + 2 * h
        V = self.level_view(L + 1, flo, fshape, restrict=False)
        for ax_arr, ax in ((2, 0), (1, 1), (0, 2)):
            V = np.moveaxis(V, ax_arr, -1)
            out = np.zeros(V.shape[:-1] + (int(shape[ax]),))
            for q in range(int(shape[ax])):
                p = 2 * q + h          # window index of fine position 2*(lo+q)
                acc = np.zeros(V.shape[:-1])
                for o in sorted(Ha):
                    acc = acc + Ha[o] * V[..., p + o]
                out[..., q] = acc
            V = np.moveaxis(out, -1, ax_arr)
        return V

    def level_view(self, L, lo, shape, restrict=True):
        """Phi_L over a box of level-L points (see module docstring)."""
        lo = np.asarray(lo)
        shape = np.asarray(shape)
        X, Y, Z = self._box(lo, shape)
        lev = self.owner_level(L, X, Y, Z)
        out = np.empty(X.shape)
        m = lev == L
        if m.any():
            out[m] = self.values_at(L, L, X[m], Y[m], Z[m])
        m = lev < L
        if m.any():
            G = self.refine_box(L, lo, shape)
            out[m] = G[m]
        m = lev > L
        if m.any():
            if restrict and self.Nt > 0:
                R = self.restrict_box(L, lo, shape)
                out[m] = R[m]
            else:
                for l in np.unique(lev[m]):
                    mm = lev == l
                    out[mm] = self.values_at(int(l), L, X[mm], Y[mm], Z[mm])
        return out

    def neighbor_level(self, key, d):
        """Level of the leaf holding the region of block ``key`` in direction d."""
        L = key[0]
        o = self.origin(key)
        rep = [o[a] + (self.nb if d[a] == 1 else (-1 if d[a] == -1 else 0))
               for a in range(3)]
        return int(self.owner_level(L, np.array(rep[0]), np.array(rep[1]),
                                    np.array(rep[2])))

    def ghost_block(self, key, depth):
        """Block ``key`` with a ghost layer of ``depth`` points (Phi_L)."""
        L = key[0]
        return self.level_view(L, self.origin(key) - depth,
                               (self.nb + 2 * depth,) * 3)

    # --------------------------------------------------------- substitution
    def substitution_slab(self, d):
        """READING R-SUB: per-axis ranges [lo, hi) of the slab of a fine block
        next to a coarser leaf in direction d (sections 2.2.2, 2.2.4, 2.3).
        The slab holds the points whose details the zero-detail ghost
        refinement takes as zero: lifted, the details around every even
        sample of the fine block that the refinement of its ghost points reads
        (N-1 points in front, N-2 behind) enter those samples through the
        lifting; unlifted, the tangential details at those samples enter (the
        3D inverse transform reads them along the facing axis), and every
        detail up to that distance is discarded (see extension_mask).  Seen
        from the neighbour that would coarsen, the far end of the slab lies at
        the distance of the 3D "coarse region extension" column of Table 3."""
        N, nb = self.N, self.nb
        rng = []
        for a in range(3):
            if d[a] == 0:
                rng.append((0, nb))
            elif self.Nt == 0:
                rng.append((0, N - 1) if d[a] < 0 else (nb - N + 2, nb))
            else:
                rng.append((0, N) if d[a] < 0 else (nb - N + 1, nb))
        return rng

    def extension_mask(self, dirs):
        """Points of a fine block whose details the coarse-extension assumption
        discards toward coarser regions in the directions ``dirs``: every
        detail (point with an odd index, of any degree) in the union of the
        R-SUB slabs.  In 3D the paper discards any first, second and third
        degree detail involved in the multi-dimensional refinement, up to the
        3D coarse region extension of Table 3 (section 2.3); for N.0 this is
        wider than the 1D column (0), which applies to 1D grids (READING
        R-SUB: with it the epsilon and moment tests of sections 4.1 and 4.2
        reproduce the paper's printed values for 4.0 and 6.0)."""
        nb = self.nb
        z, y, x = np.meshgrid(np.arange(nb), np.arange(nb), np.arange(nb), indexing="ij")
        pos = (x, y, z)
        M = np.zeros((nb, nb, nb), bool)
        for d in dirs:
            rng = self.substitution_slab(d)
            inr = np.ones((nb, nb, nb), bool)
            for a in range(3):
                inr &= (pos[a] >= rng[a][0]) & (pos[a] < rng[a][1])
            M |= inr
        return M & ((x % 2 + y % 2 + z % 2) > 0)

    def substitution_mask(self, key):
        """Points of block ``key`` whose neglected details are discarded: the
        extension mask over the directions with a coarser leaf."""
        L = key[0]
        return self.extension_mask([d for d in DIRS if self.neighbor_level(key, d) < L])

    def substitution_values(self, key, deg, M):
        """Substitution of section 2.3 for the points of degree ``deg`` (number
        of odd indices) in the mask M of block ``key``: each gets the value
        that makes its detail vanish, minus the sum over the non-central taps
        of the tensor product of G^a over its odd axes (the G^a centre tap is
        1; READING: the 1D sign of section 2.2.4).  The taps read the block's
        level view at depth N-1 as it stands, so degree-1 points read only
        all-even points and degree 2 and 3 read the values of the lower
        degrees set before them.  Returns (z, y, x, values)."""
        N = self.N
        D = N - 1
        X = self.ghost_block(key, D)
        ga = wv.table(N, 0)["Ga"]
        z, y, x = np.nonzero(M)
        par = (x % 2, y % 2, z % 2)
        keep = (par[0] + par[1] + par[2]) == deg
        z, y, x = z[keep], y[keep], x[keep]
        par = (x % 2, y % 2, z % 2)
        out = np.zeros(len(x))
        for pat in {(a, b, c) for a, b, c in zip(*par)}:
            sel = (par[0] == pat[0]) & (par[1] == pat[1]) & (par[2] == pat[2])
            taps = [ga if pat[a] else {0: 1.0} for a in range(3)]
            acc = np.zeros(int(sel.sum()))
            for oz in sorted(taps[2]):
                for oy in sorted(taps[1]):
                    for ox in sorted(taps[0]):
                        if (ox, oy, oz) == (0, 0, 0):
                            continue
                        w = taps[2][oz] * taps[1][oy] * taps[0][ox]
                        acc = acc + w * X[z[sel] + D + oz, y[sel] + D + oy, x[sel] + D + ox]
            out[sel] = -acc
        return z, y, x, out

    def substitute(self, keys=None):
        """Substitution step of sections 2.2.4 and 2.3 on every fine block
        next to a coarser leaf, in degree order: all degree-1 points of every
        block, then degree 2, then degree 3 (each degree reads the values the
        lower degrees were given, in its own block and in its same-level
        neighbours; ghost values in coarser regions come from the samples
        before the substitution, READING R-ORDER).  Returns the number of
        points written.

        With ``keys``, only those blocks' substituted values are exact: the
        degrees 1 and 2 run on them and their same-level neighbours (whose
        values their stencils read), degree 3 on them alone (a sampled check
        of a large grid; other blocks are left partly substituted)."""
        if keys is None:
            inner = ring = set(self.blocks)
        else:
            inner = {tuple(k) for k in keys}
            ring = set(inner)
            for k in inner:
                ring |= {n for n in self.leaf_neighbors(k) if n[0] == k[0]}
        masks = {k: self.substitution_mask(k) for k in sorted(ring)}
        touched = {k for k, m in masks.items() if m.any()}
        self._pre = {k: (v.copy() if k in touched else v) for k, v in self.blocks.items()}
        n = 0
        for deg in (1, 2, 3):
            writes = []
            for key, M in masks.items():
                if key in touched and (deg < 3 or key in inner):
                    writes.append((key,) + self.substitution_values(key, deg, M))
            for key, z, y, x, v in writes:
                self._blocks[key][z, y, x] = v
                n += len(v)
        return n

    # ---------------------------------------------------------------- RHS
    def positions(self, key):
        L = key[0]
        o = self.origin(key)
        den = float(self.nb << L)
        idx = np.arange(self.nb)
        return ((o[0] + idx) / den, (o[1] + idx) / den, (o[2] + idx) / den)

    @staticmethod
    def velocity(vel, x, y, z):
        """Velocity components on the [z, y, x] grid of the 1D coordinates."""
        kind, p = vel
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        if kind == "const":
            return (np.full(X.shape, p[0]), np.full(X.shape, p[1]),
                    np.full(X.shape, p[2]))
        if kind == "rotating":
            return (-(Y - p[1]), X - p[0], np.full(X.shape, p[2]))
        if kind == "shear":
            tp = 2.0 * np.pi
            return np.sin(tp * Z), np.sin(tp * X), np.sin(tp * Y)
        raise ValueError(kind)

    def rhs_block(self, key, vel):
        """Right-hand side of the transport problem of section 5 on the
        ghost-filled block.  fd_order 4 / 6: -(u . grad) phi with central FD
        of that order, equal to -div(u phi) for the velocity fields used
        here, where each u_d does not depend on x_d.  fd_order 3 / 5: the
        conservative CONS-3 / CONS-5 form of the finite-difference
        supplement (see cons_rhs_block).  Velocity kind "diffusion" (nu,):
        nu * laplacian(phi) (see diffusion_rhs_block)."""
        if vel[0] == "diffusion":
            return self.diffusion_rhs_block(key, vel[1][0])
        if self.fd_order in (3, 5):
            return self.cons_rhs_block(key, vel)
        g = self.fd_order // 2
        Xg = self.ghost_block(key, g)
        nb = self.nb
        h = 1.0 / (nb << key[0])
        w = fd_weights(self.fd_order)
        core = slice(g, g + nb)
        dx = sum(w[o] * Xg[core, core, g + o:g + o + nb] for o in sorted(w)) / h
        dy = sum(w[o] * Xg[core, g + o:g + o + nb, core] for o in sorted(w)) / h
        dz = sum(w[o] * Xg[g + o:g + o + nb, core, core] for o in sorted(w)) / h
        ux, uy, uz = self.velocity(vel, *self.positions(key))
        return -(ux * dx + uy * dy + uz * dz)

    def diffusion_rhs_block(self, key, nu):
        """Diffusion right-hand side nu * laplacian(phi) with the central
        second differences of order fd_order (2: DIFF-2, 4: DIFF-4, 6) of
        the finite-difference supplement, on the ghost-filled block."""
        if self.fd_order not in (2, 4, 6):
            raise ValueError("diffusion takes fd_order 2, 4 or 6")
        g = self.fd_order // 2
        Xg = self.ghost_block(key, g)
        nb = self.nb
        h = 1.0 / (nb << key[0])
        w = d2_weights(self.fd_order)
        core = slice(g, g + nb)
        dxx = sum(w[o] * Xg[core, core, g + o:g + o + nb] for o in sorted(w))
        dyy = sum(w[o] * Xg[core, g + o:g + o + nb, core] for o in sorted(w))
        dzz = sum(w[o] * Xg[g + o:g + o + nb, core, core] for o in sorted(w))
        return nu * (dxx + dyy + dzz) / (h * h)

    def cons_rhs_block(self, key, vel):
        """Conservative RHS of the finite-difference supplement:
        d phi_i / dt = -sum_d (f_{i+1/2} - f_{i-1/2}) / h with f = u_d phi and
        the fixed-weight WENO interface flux of order 3 or 5 (cons_fluxes):
        f^+ where the interface velocity is positive, f^- where it is
        negative.  READING (the interface velocity printed as the mean of
        u_{i+1} and u_{i-1}): u_{i+1/2} = (u_i + u_{i+1}) / 2; for the
        velocity fields used here u_d does not vary along x_d, so both
        readings give u_d itself."""
        g = stencil_depth(self.fd_order)
        nb = self.nb
        L = key[0]
        h = 1.0 / (nb << L)
        Xg = self.ghost_block(key, g)
        o = self.origin(key)
        den = float(nb << L)
        ext = np.arange(-g, nb + g)
        u = self.velocity(vel, (o[0] + ext) / den, (o[1] + ext) / den, (o[2] + ext) / den)
        plus, minus = cons_fluxes(self.fd_order)
        out = np.zeros((nb, nb, nb))
        for a, ax in ((0, 2), (1, 1), (2, 0)):          # x, y, z; array axis
            f = u[a] * Xg                                 # flux u_d phi
            fa = np.moveaxis(f, ax, -1)
            ua = np.moveaxis(u[a], ax, -1)
            # interfaces i+1/2 for i = -1 .. nb-1 (window index g-1 .. g+nb-1)
            fl = []
            for i in range(g - 1, g + nb):
                up = sum(c * fa[..., i + k] for k, c in sorted(plus.items()))
                dn = sum(c * fa[..., i + k] for k, c in sorted(minus.items()))
                ui = 0.5 * (ua[..., i] + ua[..., i + 1])
                fl.append(np.where(ui > 0, up, dn))
            F = np.stack(fl, axis=-1)                    # [..., nb + 1]
            d = (F[..., 1:] - F[..., :-1]) / h
            d = np.moveaxis(d, -1, ax)
            sl = [slice(g, g + nb)] * 3
            sl[ax] = slice(None)
            out -= d[tuple(sl)]
        return out

    def rk3_step(self, dt, vel):
        """SSP-RK3 of the time-integration supplement (standard Gottlieb-Shu
        form, READING of the garbled stage formula).  Each stage starts with a
        ghost reconstruction (substitution + level view)."""
        self.substitute()
        u = {k: v.copy() for k, v in self.blocks.items()}
        f = {k: self.rhs_block(k, vel) for k in self.blocks}
        y1 = {k: u[k] + dt * f[k] for k in u}
        self.blocks = y1
        self.substitute()
        f = {k: self.rhs_block(k, vel) for k in self.blocks}
        y2 = {k: 0.75 * u[k] + 0.25 * (self.blocks[k] + dt * f[k]) for k in u}
        self.blocks = y2
        self.substitute()
        f = {k: self.rhs_block(k, vel) for k in self.blocks}
        self.blocks = {k: (1.0 / 3.0) * u[k] + (2.0 / 3.0) * (self.blocks[k] + dt * f[k])
                       for k in u}

    # ------------------------------------------------------------ details
    def block_transform(self, key):
        """One-level forward transform of the ghost-filled block: 1D analysis
        along x, then y, then z (section 2.3).  Returns the interleaved
        coefficients on the block's own positions [0, nb)^3."""
        f, b = transform_reach(self.N, self.Nt)
        D = max(f, b)
        return self.transform_of(self.ghost_block(key, D), D)

    def transform_of(self, X, D):
        """The transform of block_transform applied to a given ghost-filled
        block X of depth D (array [z, y, x] of (nb + 2D)^3 values)."""
        nb = self.nb
        T = wv.analysis(X, 2, -D, 0, nb, self.N, self.Nt)
        T = wv.analysis(T, 1, -D, 0, nb, self.N, self.Nt)
        T = wv.analysis(T, 0, -D, 0, nb, self.N, self.Nt)
        return T

    def details_of(self, T):
        """Detail coefficients (points with at least one odd index) of a
        block transform T, zero at the scaling (all-even) positions."""
        idx = np.arange(self.nb) % 2
        odd = (idx[:, None, None] + idx[None, :, None] + idx[None, None, :]) > 0
        return np.where(odd, T, 0.0)

    def block_details(self, key):
        """Detail coefficients of the block's ghost-filled transform."""
        return self.details_of(self.block_transform(key))

    def block_norm(self, key, det=None):
        """Block criterion of section 2.2.5 for one block: max |gamma^{L-1}|
        over its own detail positions and, with the extension (READING R-EXT),
        over the band of E_f / E_b points of each same-level neighbour next to
        it (Table 3, 3D coarse region extension).  ``det`` caches
        block_details results."""
        det = {} if det is None else det

        def D(k):
            if k not in det:
                det[k] = self.block_details(k)
            return det[k]
        best = float(np.max(np.abs(D(key))))
        if not self.detail_ext:
            return best
        Ef, Eb = DETAIL_EXT[(self.N, self.Nt)]
        nb = self.nb
        L, i, j, k = key
        n = 1 << L
        for d in DIRS:
            nk = (L, (i + d[0]) % n, (j + d[1]) % n, (k + d[2]) % n)
            if nk not in self.blocks:
                continue
            sl = []
            for a in (2, 1, 0):          # z, y, x array axes
                if d[a] == 0:
                    sl.append(slice(0, nb))
                elif d[a] == 1:
                    sl.append(slice(0, Eb))
                else:
                    sl.append(slice(nb - Ef, nb))
            band = D(nk)[tuple(sl)]
            if band.size:
                best = max(best, float(np.max(np.abs(band))))
        return best

    def norms(self):
        """Block criterion of section 2.2.5 for every block (see block_norm)."""
        det = {}
        return {k: self.block_norm(k, det) for k in self.blocks}

    # ------------------------------------------------------------- moments
    def moments(self):
        """Discrete moments M0 and M1 (x, y, z) of the field (equation of the
        interpolating-wavelet moments, section 2.1.4, applied per axis)."""
        m = np.zeros(4)
        for key, a in self.blocks.items():
            x, y, z = self.positions(key)
            w = (1.0 / (self.nb << key[0])) ** 3
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            m[0] += w * a.sum()
            m[1] += w * (a * X).sum()
            m[2] += w * (a * Y).sum()
            m[3] += w * (a * Z).sum()
        return m

    # --------------------------------------------------------------- adapt
    def leaf_neighbors(self, key):
        """Leaves touching block ``key`` (26-neighbourhood, periodic): the
        owners of the one-point shell around the block at level L+1."""
        L = key[0]
        nb = self.nb
        Lf = L + 1
        lo = self.origin(key) * 2 - 1
        n = 2 * nb + 2
        X, Y, Z = self._box(lo, (n, n, n))
        shell = ((X == lo[0]) | (X == lo[0] + n - 1) | (Y == lo[1]) |
                 (Y == lo[1] + n - 1) | (Z == lo[2]) | (Z == lo[2] + n - 1))
        W = self.width(Lf)
        X, Y, Z = X[shell] % W, Y[shell] % W, Z[shell] % W
        lev = self.owner_level(Lf, X, Y, Z)
        out = set()
        for l in np.unique(lev):
            m = lev == l
            if l <= Lf:
                s = Lf - l
                bx, by, bz = (X[m] >> s) // nb, (Y[m] >> s) // nb, (Z[m] >> s) // nb
            else:
                s = l - Lf
                bx, by, bz = (X[m] << s) // nb, (Y[m] << s) // nb, (Z[m] << s) // nb
            for t in set(zip(bx.tolist(), by.tolist(), bz.tolist())):
                out.add((int(l),) + tuple(int(v) for v in t))
        out.discard(key)
        return out

    def is_balanced(self):
        for key in self.blocks:
            for n in self.leaf_neighbors(key):
                if abs(n[0] - key[0]) > 1:
                    return False
        return True

    def flags(self, norms):
        """Block status of the grid-adaptation supplement (READING R-TIE:
        >= eps_r refines, <= eps_c may coarsen)."""
        fl = {}
        for key, n in norms.items():
            L = key[0]
            if n >= self.eps_r and L < self.level_max:
                fl[key] = FINER
            elif n <= self.eps_c and L > self.level_min:
                fl[key] = COARSER
            else:
                fl[key] = SAME
        return fl

    def policy(self, fl, created, allow_coarsen=True):
        """Adaptation policy of the grid-adaptation supplement: refinement has
        priority and propagates to coarser neighbours (2:1); a sibling set
        coarsens only if all eight leaves agree, none was created by
        refinement in this adaptation, and 2:1 holds afterwards."""
        refine = {k for k, f in fl.items() if f == FINER}
        nbrs = {}
        todo = list(refine)
        while todo:
            b = todo.pop()
            for n in nbrs.setdefault(b, self.leaf_neighbors(b)):
                if n[0] < b[0] and n not in refine:
                    refine.add(n)
                    todo.append(n)
        coarsen = set()
        if allow_coarsen:
            groups = {}
            for k, f in fl.items():
                if f == COARSER and k not in refine and k not in created:
                    L, i, j, kk = k
                    groups.setdefault((L - 1, i >> 1, j >> 1, kk >> 1), []).append(k)
            for p, ch in groups.items():
                if len(ch) != 8:
                    continue
                ok = True
                for c in ch:
                    for n in nbrs.setdefault(c, self.leaf_neighbors(c)):
                        if (n[0] > c[0]) or (n[0] == c[0] and n in refine):
                            ok = False
                            break
                    if not ok:
                        break
                if ok:
                    coarsen.add(p)
        return refine, coarsen

    def _refine_children(self, key):
        """Block refinement of section 2.2.3: zero-detail inverse transform of
        the ghost-filled block (Table 3 refinement ghosts)."""
        L = key[0]
        nb, N = self.nb, self.N
        D = max(N // 2, 1)       # Table 3 refinement ghosts: N/2-1 front, N/2 back
        X = self.ghost_block(key, D)
        out = {}
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    flo = np.array([cx, cy, cz]) * nb    # child origin in the parent's level-(L+1) frame
                    T = wv.refine_1d(X, 2, -D, flo[0], flo[0] + nb, N, self.Nt)
                    T = wv.refine_1d(T, 1, -D, flo[1], flo[1] + nb, N, self.Nt)
                    T = wv.refine_1d(T, 0, -D, flo[2], flo[2] + nb, N, self.Nt)
                    ck = (L + 1, 2 * key[1] + cx, 2 * key[2] + cy, 2 * key[3] + cz)
                    out[ck] = T
        return out

    def _coarsen_parent(self, pkey):
        """Block coarsening of section 2.2.1 / 2.3: [H^a]^3 of the eight
        children's level-L field with their ghosts (Table 3 coarsening)."""
        Lp = pkey[0]
        L = Lp + 1
        nb = self.nb
        Ha = wv.table(self.N, self.Nt)["Ha"]
        h = max(Ha)
        lo = self.origin(pkey) * 2 - h
        V = self.level_view(L, lo, (2 * nb + 2 * h,) * 3, restrict=True)
        for ax_arr in (2, 1, 0):
            V = np.moveaxis(V, ax_arr, -1)
            out = np.zeros(V.shape[:-1] + (nb,))
            for q in range(nb):
                p = 2 * q + h
                acc = np.zeros(V.shape[:-1])
                for o in sorted(Ha):
                    acc = acc + Ha[o] * V[..., p + o]
                out[..., q] = acc
            V = np.moveaxis(out, -1, ax_arr)
        return V

    def _update_delta(self, fkey, discarded):
        """Update step of section 2.2.1 / Table 3 for a kept block at level L
        next to a new coarse parent: the inverse transform (z, then y, then x)
        of the discarded level-(L-1) details (``discarded``: block key ->
        detail array, zero where kept), with all scaling coefficients zero,
        evaluated on the block's points."""
        t = wv.table(self.N, self.Nt)
        r = max(max(t["Js"]), max(t["Ks"]))
        L = fkey[0]
        nb = self.nb
        lo = self.origin(fkey) - r
        shape = np.array([nb + 2 * r] * 3)
        X, Y, Z = self._box(lo, shape)
        W = self.width(L)
        Dd = np.zeros(X.shape)
        bx, by, bz = (X % W) // nb, (Y % W) // nb, (Z % W) // nb
        for ck, det in discarded.items():
            if ck[0] != L:
                continue
            m = (bx == ck[1]) & (by == ck[2]) & (bz == ck[3])
            if m.any():
                Dd[m] = det[(Z[m] % W) % nb, (Y[m] % W) % nb, (X[m] % W) % nb]
        if not Dd.any():
            return None
        T = wv.synthesis(Dd, 0, -r, 0, nb, self.N, self.Nt)
        T = wv.synthesis(T, 1, -r, 0, nb, self.N, self.Nt)
        T = wv.synthesis(T, 2, -r, 0, nb, self.N, self.Nt)
        return T

    def apply(self, refine, coarsen):
        """Interpolate (refine / coarsen) and update, computed from the current
        ghost-filled field; then replace the tree."""
        new = {}
        for k in refine:
            new.update(self._refine_children(k))
        children = {}
        for p in coarsen:
            new[p] = self._coarsen_parent(p)
            L = p[0] + 1
            for cz in (0, 1):
                for cy in (0, 1):
                    for cx in (0, 1):
                        ck = (L, 2 * p[1] + cx, 2 * p[2] + cy, 2 * p[3] + cz)
                        children[ck] = None
        deltas = {}
        # The discarded details are those of the coarsened children and, in
        # each kept same-level neighbour, its coarse-extension slab toward the
        # new parent: section 2.2.1 discards, with a coarsening neighbour, the
        # fine side's details up to the coarse region extension distance of
        # Table 3 as well (for 2.2 in 1D: gamma_2^0 when the region in front
        # coarsens), and the update subtracts the synthesis of all of them
        # (READING R-UPD).  In 3D the update is needed for N.0 as well: the
        # tensor inverse transform carries discarded details of one axis into
        # the fine neighbour along another (3D values of the update column of
        # Table 3).
        if children:
            for ck in children:
                children[ck] = self.block_details(ck)
            kept_next = set()
            for ck in children:
                for n in self.leaf_neighbors(ck):
                    if n[0] == ck[0] and n not in children and n not in refine:
                        kept_next.add(n)
            discarded = dict(children)
            for fk in sorted(kept_next):
                L, i, j, k = fk
                n = 1 << L
                dirs = [d for d in DIRS if (L, (i + d[0]) % n, (j + d[1]) % n,
                                             (k + d[2]) % n) in children]
                M = self.extension_mask(dirs)
                if M.any():
                    discarded[fk] = np.where(M, self.block_details(fk), 0.0)
            for fk in sorted(kept_next):
                dlt = self._update_delta(fk, discarded)
                if dlt is not None:
                    deltas[fk] = dlt
        blocks = {}
        for k, v in self.blocks.items():
            if k in refine or k in children:
                continue
            blocks[k] = v - deltas[k] if k in deltas else v.copy()
        blocks.update(new)
        self.blocks = blocks
        self._index()

    def adapt(self, max_iter=16):
        """Iterative grid adaptation of the grid-adaptation supplement: ghost,
        criterion, policy, interpolate, update; until no block changes."""
        created = set()
        stats = dict(iters=0, refined=0, coarsened=0)
        for _ in range(max_iter):
            self.substitute()
            fl = self.flags(self.norms())
            refine, coarsen = self.policy(fl, created)
            if not refine and not coarsen:
                break
            self.apply(refine, coarsen)
            for k in refine:
                L, i, j, kk = k
                for c in range(8):
                    created.add((L + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1),
                                 2 * kk + ((c >> 2) & 1)))
            stats["iters"] += 1
            stats["refined"] += len(refine)
            stats["coarsened"] += len(coarsen)
        stats["n_blocks"] = len(self.blocks)
        return stats

    def init_ic(self, ic, max_iter=32):
        """READING R-INIT: uniform tree at level_min; refine only, re-sampling
        the initial condition on every leaf, until stable; then one normal
        adaptation."""
        self.uniform(self.level_min)
        self.sample(ic)
        for _ in range(max_iter):
            self.substitute()
            fl = self.flags(self.norms())
            fl = {k: (f if f == FINER else SAME) for k, f in fl.items()}
            refine, _ = self.policy(fl, set(), allow_coarsen=False)
            if not refine:
                break
            new_keys = [k for k in self.blocks if k not in refine]
            for k in refine:
                L, i, j, kk = k
                for c in range(8):
                    new_keys.append((L + 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1),
                                     2 * kk + ((c >> 2) & 1)))
            self.set_tree(new_keys)
            self.sample(ic)
        return self.adapt()

    def sample(self, ic):
        self._pre = None
        for key in self.blocks:
            x, y, z = self.positions(key)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            self.blocks[key] = ic(X, Y, Z)

    # ------------------------------------------------------------- export
    def keys(self):
        return sorted(self.blocks)

    def flat(self, order):
        return np.concatenate([self.blocks[tuple(k)].ravel() for k in order])
