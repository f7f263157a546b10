"""Pins of the oracle's sub-cycled step (per-level time steps, Sec. 4;
time-accurate coarse data in fine ghost cells, Sec. 3; the recursion and
flux correction of Berger and Oliger 1984 / Berger and Colella 1989):

- on a single-level forest it is the global-dt step, bit for bit;
- it conserves mass to rounding on adaptive forests, across regrids;
- constants (free stream, lake at rest) stay exact;
- every row of a forest with bands of finer patches (two and three levels)
  equals an independent one-dimensional sub-cycled mixed-resolution
  flux-form routine written here from the method: coarse columns step
  first, finer columns twice with half the step, fine ghost cells from the
  coarse state interpolated in time, coarse cells at a coarse-fine face
  corrected by the time average of the fine face fluxes;
- a smooth translation on an adaptive forest converges at second order.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I


@pytest.mark.parametrize("phys", ["advection", "shallow"])
def test_single_level_is_the_global_step(phys):
    m = 8
    if phys == "advection":
        trees, pl = I.periodic_square()
        par = O.params(m, O.ADVECTION, ax=0.7, ay=-0.4)
        fn = lambda x, y: I.gaussian(x, y, 0.4, 0.6, 0.02)
    else:
        trees, pl = I.walled_square()
        par = O.params(m, O.SHALLOW)
        fn = lambda x, y: I.dam_break(x, y)
    lv = O.sfc_sort(I.uniform_leaves(1, 3))
    mesh = O.Mesh(trees, lv, m)
    q = I.state_from(lv, m, fn, pl)
    for _ in range(3):
        a, nua = O.advance(mesh, par, q, 2e-3)
        b, nub = O.advance_subcycled(mesh, par, q, 2e-3 * 8)     # level 3
        assert np.array_equal(a, b) and nua == nub
        q = a


def _levels(lv):
    return sorted(set(int(v) for v in lv["level"]))


def test_mass_is_conserved_across_levels_and_regrids():
    m = 8
    trees, pl = I.walled_square()
    par = O.params(m, O.SHALLOW)
    lv = O.balance(trees, I.random_leaves(3, 1, 2, 5, 30))
    assert len(_levels(lv)) >= 3
    q = I.state_from(lv, m, lambda x, y: I.dam_break(x, y, 0.45, 0.55, 0.2), pl)
    mesh = O.Mesh(trees, lv, m)
    f = O.framed(q, m)
    O.ghost_fill(mesh, par, f)
    m0 = O.sums(mesh, par, f)[0]
    dt = 0.4 / m / 1.8                      # a level-0 patch's step
    rng = np.random.default_rng(1)
    for step in range(6):
        q, nu = O.advance_subcycled(mesh, par, q, dt)
        assert 0 < nu < 1
        dt *= 0.9 / nu
        if step % 2 == 1:
            f = O.framed(q, m)
            O.ghost_fill(mesh, par, f)
            tg = rng.integers(-1, 2, len(lv)).astype(np.int8)
            lv2 = O.regrid(mesh, tg, 1, 5)
            mesh2 = O.Mesh(trees, lv2, m)
            q = O.interior(O.transfer(mesh, mesh2, par, f), m)
            mesh, lv = mesh2, lv2
        f = O.framed(q, m)
        O.ghost_fill(mesh, par, f)
        assert abs(O.sums(mesh, par, f)[0] - m0) <= 1e-14 * m0


@pytest.mark.parametrize("phys", ["advection", "shallow"])
def test_constants_stay_exact(phys):
    m = 8
    if phys == "advection":
        trees, pl = I.periodic_square()
        par = O.params(m, O.ADVECTION, ax=0.9, ay=0.35)
        c = np.array([1.5])
    else:
        trees, pl = I.walled_square()
        par = O.params(m, O.SHALLOW)
        c = np.array([1.5, 0.0, 0.0])
    lv = O.balance(trees, I.random_leaves(5, 1, 2, 5, 25))
    q = np.broadcast_to(c[None, :, None, None], (len(lv), len(c), m, m)).copy()
    mesh = O.Mesh(trees, lv, m)
    out, _ = O.advance_subcycled(mesh, par, q, 0.3 / m)
    assert np.array_equal(out, q)


# ---------------------------------------------------------------------------
# the independent band routine
# ---------------------------------------------------------------------------
def _minmod(a, b):
    if a * b <= 0.0:
        return 0.0
    return a if abs(a) <= abs(b) else b


def _mc(th):
    return max(0.0, min((1.0 + th) / 2.0, 2.0, 2.0 * th))


class _SubcycledBands:
    """One-dimensional mixed-resolution flux-form scheme for a = (u, 0) on
    the periodic square, in patch columns of relative levels `levels` (base
    level 2; neighbouring columns differ by at most one level), m cells per
    patch row.  A column of relative level k has R * 2^k rows of m cells of
    size 1 / (m 2^(2 + k)) and steps 2^k times per coarse step.  Cell values
    of a column are read at a time t: its state if it is at t, else the
    linear interpolation in time of its state at the start and the end of
    its current step."""

    def __init__(self, m, coarse_rows, levels):
        self.m, self.R, self.lev = m, coarse_rows, list(levels)
        self.n = len(levels)
        self.L = max(levels)

    def rows(self, s):
        return self.R << self.lev[s]

    def h(self, s):
        return 1.0 / (self.m << (2 + self.lev[s]))

    def val(self, s, r, i, t):
        """Interior cell (r, i) of column s read at time t."""
        r %= self.rows(s)
        if self.t_new[s] == t or self.t_old[s] == self.t_new[s]:
            return self.cur[s][r, i]
        a = (t - self.t_old[s]) / (self.t_new[s] - self.t_old[s])
        return (1.0 - a) * self.old[s][r, i] + a * self.cur[s][r, i]

    def ghost(self, s, r, i, t):
        m = self.m
        side = -1 if i < 0 else 1
        s2 = (s + side) % self.n
        k = i if i < 0 else i - m
        if self.lev[s2] == self.lev[s]:
            return self.val(s2, r, k % m if side < 0 else k, t)
        if self.lev[s2] > self.lev[s]:
            cols = [m + 2 * k, m + 2 * k + 1] if side < 0 else [2 * k, 2 * k + 1]
            v = 0.0
            for rr in (2 * r, 2 * r + 1):
                for c in cols:
                    v += self.val(s2, rr, c, t)
            return v / 4.0
        c = m - 1 if side < 0 else 0
        Rr = r // 2
        dxo = (0.25 if k == -1 else -0.25) if side < 0 else (-0.25 if k == 0 else 0.25)
        dyo = -0.25 if r % 2 == 0 else 0.25
        qc = self.val(s2, Rr, c, t)
        qe = self.ext(s2, Rr, c + 1, t)
        qw = self.ext(s2, Rr, c - 1, t)
        qn = self.val(s2, Rr + 1, c, t)
        qs = self.val(s2, Rr - 1, c, t)
        return qc + dxo * _minmod(qe - qc, qc - qw) + dyo * _minmod(qn - qc, qc - qs)

    def ext(self, s, r, i, t):
        if 0 <= i < self.m:
            return self.val(s, r, i, t)
        return self.ghost(s, r, i, t)

    def fluxes(self, s, r, u, dt, t):
        m = self.m
        q = np.array([self.ext(s, r, i, t) for i in range(-2, m + 2)])
        W = q[1:] - q[:-1]
        nu = abs(u) * dt / self.h(s)
        F = np.zeros(m + 1)
        for f in range(m + 1):
            e = f + 1
            wv = W[e]
            up = W[e - 1] if u > 0 else W[e + 1]
            lim = 0.0 if wv == 0.0 else _mc(up * wv / (wv * wv))
            qup = q[e] if u > 0 else q[e + 1]
            F[f] = u * qup + 0.5 * abs(u) * (1.0 - nu) * lim * wv
        return F

    def coarse_step(self, seg, u, dt0):
        self.cur = [a.copy() for a in seg]
        self.old = [a.copy() for a in seg]
        self.t_old = [0.0] * self.n
        self.t_new = [0.0] * self.n
        # time-integrated fine face fluxes at each coarse-fine face, per
        # coarse column and side: [rows of the coarse column]
        self.acc = {}
        self._advance(0, 0.0, u, dt0)
        return self.cur

    def _advance(self, k, t, u, dt0):
        dt = dt0 / (1 << k)
        cols = [s for s in range(self.n) if self.lev[s] == k]
        flux = {}
        for s in cols:
            self.old[s] = self.cur[s].copy()
            self.t_old[s], self.t_new[s] = t, t
        new = {}
        for s in cols:
            flux[s] = [self.fluxes(s, r, u, dt, t) for r in range(self.rows(s))]
            new[s] = np.array([self.cur[s][r] - dt / self.h(s) * (F[1:] - F[:-1])
                               for r, F in enumerate(flux[s])])
        for s in cols:
            self.cur[s] = new[s]
            self.t_new[s] = t + dt
        # this level's face fluxes at faces with the next coarser level,
        # averaged over the two fine rows and weighted by dt / dt_coarse
        for s in cols:
            for side in (-1, 1):
                s2 = (s + side) % self.n
                if self.lev[s2] != k - 1:
                    continue
                key = (s2, -side)
                acc = self.acc.setdefault(key, np.zeros(self.rows(s2)))
                face = 0 if side < 0 else self.m
                for R2 in range(self.rows(s2)):
                    fine = 0.5 * (flux[s][2 * R2][face] + flux[s][2 * R2 + 1][face])
                    acc[R2] += 0.5 * fine
        if k < self.L:
            for s in range(self.n):
                for side in (-1, 1):
                    if self.lev[s] == k:
                        self.acc.pop((s, side), None)
            self._advance(k + 1, t, u, dt0)
            self._advance(k + 1, t + 0.5 * dt, u, dt0)
            for s in cols:
                for side in (-1, 1):
                    if (s, side) not in self.acc:
                        continue
                    fine = self.acc[(s, side)]
                    i = self.m - 1 if side > 0 else 0
                    for r in range(self.rows(s)):
                        Fc = flux[s][r][self.m if side > 0 else 0]
                        if side > 0:
                            self.cur[s][r, i] -= dt / self.h(s) * (fine[r] - Fc)
                        else:
                            self.cur[s][r, i] -= dt / self.h(s) * (Fc - fine[r])


def _band_forest(levels, transpose):
    """Leaves of patch columns with the given relative levels (base level 2),
    each column a full-height stack of square patches."""
    lv = []
    x = 0                                    # in units of level-6 cells
    for k in levels:
        l = 2 + k
        w = 1 << (6 - l)
        for iy in range(1 << l):
            ix = x // w
            a, b = (iy, ix) if transpose else (ix, iy)
            lv.append((0, l, a, b))
        x += w
    assert x == 1 << 6
    return O.sfc_sort(np.array(lv, dtype=O.LEAF_DTYPE))


def _segments(lv, q, m, levels, transpose):
    starts, x = [], 0
    for k in levels:
        starts.append(x)
        x += 1 << (4 - k)
    seg = [np.zeros(((4 << k) * m, m)) for k in levels]
    for p, a in enumerate(lv):
        lev, ix, iy = int(a["level"]), int(a["ix"]), int(a["iy"])
        blk = q[p, 0]
        if transpose:
            ix, iy = iy, ix
            blk = blk.T
        x0 = ix << (6 - lev)
        s = starts.index(x0)
        seg[s][iy * m:(iy + 1) * m, :] = blk
    return seg


@pytest.mark.parametrize("levels", [(0, 1, 1, 0, 0), (0, 1, 2, 2, 1, 1, 0)])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("u", [0.8, -0.65])
def test_subcycled_rows_equal_the_band_routine(levels, transpose, u):
    m = 8
    trees, pl = I.periodic_square()
    lv = _band_forest(levels, transpose)
    mesh = O.Mesh(trees, lv, m)
    assert mesh.balanced()
    ax, ay = (0.0, u) if transpose else (u, 0.0)
    par = O.params(m, O.ADVECTION, ax=ax, ay=ay)

    def fn(x, y):
        a, b = (y, x) if transpose else (x, y)
        return (np.exp(-40 * (a - 0.35) ** 2) * (1.0 + 0.5 * np.sin(2 * np.pi * b))
                + 0.3 * np.cos(2 * np.pi * a) * np.cos(4 * np.pi * b + 0.3)
                + np.where(np.abs(a - 0.6) < 0.1, 0.4 + 0.2 * b, 0.0))
    q = I.state_from(lv, m, fn, pl)
    ref = _SubcycledBands(m, 4 * m, levels)
    seg = _segments(lv, q, m, levels, transpose)
    dt0 = 0.7 / (m << 2) / abs(u)                # Courant 0.7 on every level
    for _ in range(3):
        q, nu = O.advance_subcycled(mesh, par, q, dt0 * 4)
        assert abs(nu - 0.7) < 1e-12
        seg = ref.coarse_step(seg, u, dt0)
        got = _segments(lv, q, m, levels, transpose)
        for a, b in zip(got, seg):
            assert np.max(np.abs(a - b)) <= 1e-14 * max(1.0, np.abs(b).max())


def test_smooth_translation_converges_at_second_order():
    """A smooth bump carried once across the periodic square by a = (1, 0.5)
    on a forest refined around a band (levels 2-4 and 3-5 with m = 8: the
    same geometry at twice the resolution); the error in the cell means
    of the exact translate drops by at least 2^1.7."""
    errs = []
    for base in (2, 3):
        m = 8
        trees, pl = I.periodic_square()
        raw = I.refine_near(1, base, base + 2, [(0.5, 0.5)], pl, radius=1.0)
        lv = O.balance(trees, raw)
        mesh = O.Mesh(trees, lv, m)
        par = O.params(m, O.ADVECTION, ax=1.0, ay=0.5)
        fn = lambda x, y: np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 2.0
        q = I.state_from(lv, m, fn, pl)
        T = 1.0
        dt0 = 0.5 / (m << base)
        n = int(round(T / dt0))
        for _ in range(n):
            q, _ = O.advance_subcycled(mesh, par, q, dt0 * (1 << base))
        # exact: cell means of the translate (smooth: the centre value is
        # second-order accurate, compared at the same order)
        want = I.state_from(lv, m, lambda x, y: fn(x - T, y - 0.5 * T), pl)
        h = np.ldexp(1.0, -lv["level"].astype(int)) / m
        errs.append(np.sum(np.abs(q - want)[:, 0] * (h ** 2)[:, None, None]))
    assert errs[0] / errs[1] >= 2 ** 1.7, errs
