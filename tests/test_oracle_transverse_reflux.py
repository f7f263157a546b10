"""Pins of the oracle's transverse splitting and of the placement of its
coarse-fine flux correction, against facts outside the oracle.

Transverse splitting (LeVeque 1997, and LeVeque 2002 Sec. 21.3-21.5, the
method the paper adopts in Sec. 3): a fluctuation psi from an edge of one
direction is split with the eigenstructure of the other direction's flux
Jacobian, evaluated at the normal edge's Roe state (Roe 1981): B-psi carries
the parts with negative eigenvalues, B+psi those with positive ones, so
B-psi + B+psi must be that Jacobian times psi, and for psi = q_r - q_l the
transverse flux difference itself (the Roe averages of shallow water serve
both directions).  Checked against the Jacobian written from the flux
function, against numpy's eigendecomposition of it, and against the flux
differences, for the planar directions and for the rotated split of the
cubed sphere in an edge frame.

A 2D case whose accuracy rests on the transverse terms: a smooth shallow-water
wave travelling along the diagonal of the periodic square, compared with the
exact cell averages of the same wave in one dimension (a Fourier
pseudo-spectral solution), converges at second order; without transverse
terms it does not.

Reflux placement (Berger and Colella 1989, cited in Sec. 1; Sec. 4 carries
fine-level corrections back to the coarse level): with a = (u, 0) every row
of a forest with a vertical band of finer patches evolves as a row of a
one-dimensional mixed-resolution scheme, coupled to its neighbours only by
the ghost values and by the coarse cells that take the mean of the two fine
face fluxes.  An independent routine written here in flux form (ghost cells
by the location rule, flux-limited Lax-Wendroff per patch, coarse face flux
replaced by the fine one) must reproduce every row of the oracle's step.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I


# ---------------------------------------------------------------------------
# transverse splitting
# ---------------------------------------------------------------------------
def _roe_state(ql, qr, mom):
    """Roe-averaged velocity components and mean depth of a shallow-water
    edge pair (Roe 1981; LeVeque 2002 Sec. 15.3.3): sqrt(h)-weighted
    velocities, arithmetic mean of the depths.  `mom` selects the momentum
    components."""
    sl, sr = np.sqrt(ql[0]), np.sqrt(qr[0])
    u = (ql[mom] / sl + qr[mom] / sr) / (sl + sr)
    return u, 0.5 * (ql[0] + qr[0])


def _sw_flux(q, d, g):
    """Planar shallow-water flux in direction d (0: x, 1: y) of q = (h, hu, hv)."""
    h, hu, hv = q
    if d == 0:
        return np.array([hu, hu * hu / h + 0.5 * g * h * h, hu * hv / h])
    return np.array([hv, hv * hu / h, hv * hv / h + 0.5 * g * h * h])


def _sw_jacobian(u, v, h, d, g):
    """Jacobian of _sw_flux with respect to (h, hu, hv) at velocity (u, v)
    and depth h."""
    if d == 0:
        return np.array([[0.0, 1.0, 0.0],
                         [g * h - u * u, 2 * u, 0.0],
                         [-u * v, v, u]])
    return np.array([[0.0, 0.0, 1.0],
                     [-u * v, v, u],
                     [g * h - v * v, 0.0, 2 * v]])


def _eig_split(J, psi):
    lam, R = np.linalg.eig(J)
    lam, R = lam.real, R.real
    beta = np.linalg.solve(R, psi)
    return R @ (np.minimum(lam, 0) * beta), R @ (np.maximum(lam, 0) * beta)


def _random_sw_pair(rng):
    ql = np.array([rng.uniform(0.3, 3.0), rng.normal(0, 1.5), rng.normal(0, 1.5)])
    qr = np.array([rng.uniform(0.3, 3.0), rng.normal(0, 1.5), rng.normal(0, 1.5)])
    return ql, qr


@pytest.mark.parametrize("d", [0, 1])
def test_shallow_water_split_is_the_transverse_eigensplit(d):
    """For the edge of direction d the split uses the flux Jacobian of the
    other direction e = 1 - d."""
    rng = np.random.default_rng(100 + d)
    g = 1.3
    par = O.params(8, O.SHALLOW, g=g)
    e = 1 - d
    worst = 0.0
    for _ in range(200):
        ql, qr = _random_sw_pair(rng)
        psi = rng.normal(size=3)
        bm, bp = O.tsplit(par, d, ql, qr, psi)
        vel, hbar = _roe_state(ql, qr, [1, 2])
        J = _sw_jacobian(vel[0], vel[1], hbar, e, g)
        scale = 1.0 + np.abs(J).max() * np.abs(psi).max()
        worst = max(worst, np.abs(bm + bp - J @ psi).max() / scale)
        em, ep = _eig_split(J, psi)
        np.testing.assert_allclose(bm, em, rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(bp, ep, rtol=0, atol=1e-12 * scale)
        # psi = q_r - q_l: the transverse flux difference (Roe property in
        # the other direction)
        dm, dp = O.tsplit(par, d, ql, qr, qr - ql)
        df = _sw_flux(qr, e, g) - _sw_flux(ql, e, g)
        np.testing.assert_allclose(dm + dp, df, rtol=0,
                                   atol=1e-12 * (1 + np.abs(df).max()))
    assert worst <= 1e-13


def test_shallow_water_split_keeps_signs_apart():
    """A fluctuation along one eigenvector goes entirely down or up by the
    sign of its eigenvalue (supersonic transverse flow: all parts up)."""
    par = O.params(8, O.SHALLOW, g=1.0)
    ql = np.array([1.0, 0.3, 2.5])
    qr = np.array([1.2, 0.1, 3.1])
    for d in (0, 1):
        vel, hbar = _roe_state(ql, qr, [1, 2])
        J = _sw_jacobian(vel[0], vel[1], hbar, 1 - d, 1.0)
        lam, R = np.linalg.eig(J)
        for k in range(3):
            bm, bp = O.tsplit(par, d, ql, qr, R[:, k].real)
            if lam[k].real > 0:
                assert np.abs(bm).max() <= 1e-14
                np.testing.assert_allclose(bp, lam[k].real * R[:, k].real, atol=1e-13)
            else:
                assert np.abs(bp).max() <= 1e-14
                np.testing.assert_allclose(bm, lam[k].real * R[:, k].real, atol=1e-13)


@pytest.mark.parametrize("d", [0, 1])
def test_advection_split(d):
    par = O.params(8, O.ADVECTION, ax=-0.7, ay=0.45)
    b = (0.45, -0.7)[d]
    for psi in (1.25, -3.0):
        bm, bp = O.tsplit(par, d, [0.0], [0.0], [psi])
        assert bm[0] == min(b, 0.0) * psi and bp[0] == max(b, 0.0) * psi


def _sphere_flux(q, n, g):
    """Shallow-water flux through a unit normal n of q = (h, m) with 3D
    Cartesian momentum m: (m.n, m (m.n)/h + g h^2/2 n)."""
    h, mv = q[0], q[1:]
    mn = mv @ n
    return np.concatenate([[mn], mv * mn / h + 0.5 * g * h * h * n])


def _sphere_jacobian_times(psi, u, h, n, g):
    """Jacobian of _sphere_flux at velocity u and depth h applied to psi."""
    ph, pm = psi[0], psi[1:]
    un = u @ n
    return np.concatenate([[pm @ n], pm * un + u * (pm @ n) - u * un * ph + g * h * n * ph])


def _frame(rng):
    a = rng.normal(size=3)
    n = a / np.linalg.norm(a)
    b = rng.normal(size=3)
    b -= (b @ n) * n
    t = b / np.linalg.norm(b)
    return n, t


def test_sphere_split_is_the_eigensplit_in_the_edge_frame():
    """Rotated split of the cubed sphere: with the frame (gamma, n, t) of a
    transverse edge and momenta in the plane of n and t, down + up parts are
    gamma times the Jacobian of the flux through n, and for psi = q_r - q_l
    gamma times the flux difference; each part equals the eigensplit of the
    Jacobian restricted to (h, m.n, m.t)."""
    rng = np.random.default_rng(7)
    g = 1.1
    par = O.params(8, O.SPHERE, g=g)
    for _ in range(100):
        n, t = _frame(rng)
        gamma = rng.uniform(0.5, 1.5)
        def state():
            h = rng.uniform(0.3, 3.0)
            return np.concatenate([[h], rng.normal(0, 1.5) * n + rng.normal(0, 1.5) * t])
        ql, qr = state(), state()
        psi = np.concatenate([[rng.normal()], rng.normal() * n + rng.normal() * t])
        lo = O.tsplit_sphere(par, gamma, n, t, ql, qr, psi, 0)
        hi = O.tsplit_sphere(par, gamma, n, t, ql, qr, psi, 1)
        u, hbar = _roe_state(ql, qr, [1, 2, 3])
        want = gamma * _sphere_jacobian_times(psi, u, hbar, n, g)
        scale = 1.0 + np.abs(want).max()
        np.testing.assert_allclose(lo + hi, want, rtol=0, atol=1e-12 * scale)
        # eigensplit in the (h, normal, tangential) coordinates of the frame
        un, ut = u @ n, u @ t
        J = gamma * _sw_jacobian(un, ut, hbar, 0, g)
        P = np.array([psi[0], psi[1:] @ n, psi[1:] @ t])
        em, ep = _eig_split(J, P)
        back = lambda c: np.concatenate([[c[0]], c[1] * n + c[2] * t])
        np.testing.assert_allclose(lo, back(em), rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(hi, back(ep), rtol=0, atol=1e-12 * scale)
        dl = O.tsplit_sphere(par, gamma, n, t, ql, qr, qr - ql, 0)
        dh = O.tsplit_sphere(par, gamma, n, t, ql, qr, qr - ql, 1)
        df = gamma * (_sphere_flux(qr, n, g) - _sphere_flux(ql, n, g))
        np.testing.assert_allclose(dl + dh, df, rtol=0, atol=1e-12 * (1 + np.abs(df).max()))


# ---------------------------------------------------------------------------
# a 2D case that depends on the transverse terms
# ---------------------------------------------------------------------------
def _spectral_sw_1d(h0, p0, T, speed_scale, g=1.0, nsub=4000):
    """Shallow water h_t + k p_w = 0, p_t + k (p^2/h + g h^2/2)_w = 0 on the
    periodic unit interval (k = speed_scale), Fourier pseudo-spectral in w
    with 2/3 de-aliasing, classical RK4 in time.  Returns the Fourier
    coefficients of h and p at time T."""
    N = len(h0)
    kw = 2j * np.pi * np.fft.fftfreq(N, 1.0 / N)
    keep = np.abs(np.fft.fftfreq(N, 1.0 / N)) <= N // 3

    def ddw(f):
        return np.real(np.fft.ifft(kw * keep * np.fft.fft(f)))

    def rhs(h, p):
        return (-speed_scale * ddw(p),
                -speed_scale * ddw(p * p / h + 0.5 * g * h * h))

    h, p = h0.copy(), p0.copy()
    dt = T / nsub
    for _ in range(nsub):
        a1, b1 = rhs(h, p)
        a2, b2 = rhs(h + 0.5 * dt * a1, p + 0.5 * dt * b1)
        a3, b3 = rhs(h + 0.5 * dt * a2, p + 0.5 * dt * b2)
        a4, b4 = rhs(h + dt * a3, p + dt * b3)
        h = h + dt / 6 * (a1 + 2 * a2 + 2 * a3 + a4)
        p = p + dt / 6 * (b1 + 2 * b2 + 2 * b3 + b4)
    return np.fft.fft(h) / N, np.fft.fft(p) / N


def _cell_means_of_diagonal(coef, xc, yc, dx):
    """Cell means over squares of side dx centred at (xc, yc) of
    f(x, y) = sum_k coef_k exp(2 pi i k (x + y))."""
    N = len(coef)
    k = np.fft.fftfreq(N, 1.0 / N)
    sinc = np.sinc(k * dx)
    ph = np.exp(2j * np.pi * np.multiply.outer(xc + yc, k))
    return np.real(ph @ (coef * sinc * sinc))


def _uniform_periodic(level, m):
    trees, pl = I.periodic_square()
    lv = O.sfc_sort(I.uniform_leaves(1, level))
    return trees, pl, lv, O.Mesh(trees, lv, m)


def _diagonal_wave_errors(transverse, levels=(2, 3, 4), T=0.25, eps=0.05):
    """L1 errors of h and of hu for the diagonal wave h = 1 + eps sin(2 pi
    (x + y)) at rest, against the exact cell means of the one-dimensional
    solution along the diagonal (coordinate w = x + y: speeds scale by
    sqrt 2, and hu = hv = p / sqrt 2 with p the momentum along it)."""
    N = 256
    w = np.arange(N) / N
    ch, cp = _spectral_sw_1d(1.0 + eps * np.sin(2 * np.pi * w), np.zeros(N), T,
                             np.sqrt(2.0))
    c0 = np.zeros(N, complex)
    c0[0], c0[1], c0[-1] = 1.0, eps / 2j, -eps / 2j
    out = []
    for level in levels:
        m = 8
        trees, pl, lv, mesh = _uniform_periodic(level, m)
        par = O.params(m, O.SHALLOW, transverse=transverse)
        dx = 1.0 / (m << level)
        x, y = I.cell_centres(lv, m, pl)
        h0 = _cell_means_of_diagonal(c0, x.ravel(), y.ravel(), dx).reshape(x.shape)
        q = np.stack([h0, 0 * h0, 0 * h0], axis=1)
        nsteps = int(np.ceil(T / (0.4 * dx)))
        for _ in range(nsteps):
            q, nu = O.advance(mesh, par, q, T / nsteps)
            assert nu < 1.0
        he = _cell_means_of_diagonal(ch, x.ravel(), y.ravel(), dx).reshape(x.shape)
        pe = _cell_means_of_diagonal(cp, x.ravel(), y.ravel(), dx).reshape(x.shape)
        out.append((np.abs(q[:, 0] - he).sum() * dx * dx,
                    np.abs(q[:, 1] - pe / np.sqrt(2.0)).sum() * dx * dx,
                    np.abs(q[:, 2] - pe / np.sqrt(2.0)).sum() * dx * dx))
    return np.array(out)


def test_diagonal_wave_is_second_order_with_transverse_terms():
    err = _diagonal_wave_errors(2)
    orders = np.log2(err[:-1] / err[1:])
    assert np.all(orders[-1] >= 1.6), (err, orders)
    # hu and hv agree by symmetry of the scheme, up to the sweep order
    assert np.allclose(err[:, 1], err[:, 2], rtol=1e-6)


def test_diagonal_wave_without_transverse_terms_is_first_order():
    """The same case with the transverse terms switched off: the cross
    derivative of the second-order scheme is missing and the error is far
    larger and first order, so the pin above rests on those terms."""
    err2 = _diagonal_wave_errors(2, levels=(3, 4))
    err0 = _diagonal_wave_errors(0, levels=(3, 4))
    orders0 = np.log2(err0[0] / err0[1])
    assert np.all(orders0 < 1.3), orders0
    assert np.all(err0[-1] > 5 * err2[-1])


# ---------------------------------------------------------------------------
# reflux placement
# ---------------------------------------------------------------------------
def _minmod(a, b):
    if a * b <= 0.0:
        return 0.0
    return a if abs(a) <= abs(b) else b


def _mc(th):
    return max(0.0, min((1.0 + th) / 2.0, 2.0, 2.0 * th))


class _BandReference:
    """One-dimensional mixed-resolution flux-form scheme for a = (u, 0) on
    the periodic square with patch columns [coarse, fine, fine, coarse,
    coarse] (base level 2, the second column refined once), m cells per patch
    row.  seg[s] holds the rows of patch column s, shape (rows, m)."""

    def __init__(self, m, coarse_rows):
        self.m = m
        self.level = [0, 1, 1, 0, 0]       # 0 coarse, 1 fine
        self.R = coarse_rows

    def rows(self, s):
        return self.R * (2 if self.level[s] else 1)

    def _cell(self, seg, s, r, i):
        return seg[s][r % self.rows(s), i]

    def ghost(self, seg, s, r, i):
        """Ghost value of patch column s, row r, frame position i (i < 0 or
        i >= m in 0-based cells) by the location rule."""
        m = self.m
        n = len(seg)
        side = -1 if i < 0 else 1
        s2 = (s + side) % n
        k = i if i < 0 else i - m          # -2, -1 (left) or 0, 1 (right)
        if self.level[s2] == self.level[s]:
            return self._cell(seg, s2, r, k % m if side < 0 else k)
        if self.level[s2] > self.level[s]:
            # coarse ghost over 2 x 2 finer cells: fine columns and rows
            cols = [m + 2 * k, m + 2 * k + 1] if side < 0 else [2 * k, 2 * k + 1]
            v = 0.0
            for rr in (2 * r, 2 * r + 1):
                for c in cols:
                    v += seg[s2][rr, c]
            return v / 4.0
        # fine ghost inside a coarser cell: minmod-limited linear values
        c = m - 1 if side < 0 else 0
        Rr = r // 2
        dxo = (0.25 if k == -1 else -0.25) if side < 0 else (-0.25 if k == 0 else 0.25)
        dyo = -0.25 if r % 2 == 0 else 0.25
        qc = seg[s2][Rr, c]
        qe = self.ext(seg, s2, Rr, c + 1)
        qw = self.ext(seg, s2, Rr, c - 1)
        qn = self._cell(seg, s2, Rr + 1, c)
        qs = self._cell(seg, s2, Rr - 1, c)
        return qc + dxo * _minmod(qe - qc, qc - qw) + dyo * _minmod(qn - qc, qc - qs)

    def ext(self, seg, s, r, i):
        if 0 <= i < self.m:
            return seg[s][r, i]
        return self.ghost(seg, s, r, i)

    def fluxes(self, seg, s, r, u, dt):
        """Face fluxes F_{i-1/2}, i = 0..m (m+1 faces) of one patch row."""
        m = self.m
        h = 1.0 / (m << (2 + self.level[s]))
        q = np.array([self.ext(seg, s, r, i) for i in range(-2, m + 2)])  # index i+2
        W = q[1:] - q[:-1]                 # W[e] at the face between q[e], q[e+1]
        nu = abs(u) * dt / h
        F = np.zeros(m + 1)
        for f in range(m + 1):             # face f-1/2 of cell f: W index f+1
            e = f + 1
            wv = W[e]
            up = W[e - 1] if u > 0 else W[e + 1]
            lim = 0.0 if wv == 0.0 else _mc(up * wv / (wv * wv))
            qup = q[e] if u > 0 else q[e + 1]
            F[f] = u * qup + 0.5 * abs(u) * (1.0 - nu) * lim * wv
        return F, h

    def step(self, seg, u, dt):
        n = len(seg)
        new = [a.copy() for a in seg]
        flux = [[None] * self.rows(s) for s in range(n)]
        for s in range(n):
            for r in range(self.rows(s)):
                F, h = self.fluxes(seg, s, r, u, dt)
                flux[s][r] = F
                new[s][r] = seg[s][r] - dt / h * (F[1:] - F[:-1])
        # coarse cells at a coarse-fine face take the mean of the two fine
        # face fluxes instead of their own
        m = self.m
        for s in range(n):
            if self.level[s]:
                continue
            h = 1.0 / (m << 2)
            for side in (-1, 1):
                s2 = (s + side) % n
                if not self.level[s2]:
                    continue
                for r in range(self.R):
                    if side > 0:
                        fine = 0.5 * (flux[s2][2 * r][0] + flux[s2][2 * r + 1][0])
                        new[s][r, m - 1] -= dt / h * (fine - flux[s][r][m])
                    else:
                        fine = 0.5 * (flux[s2][2 * r][m] + flux[s2][2 * r + 1][m])
                        new[s][r, 0] -= dt / h * (flux[s][r][0] - fine)
        return new


def _band_forest(transpose):
    lv = []
    for iy in range(4):
        for ix in range(4):
            a, b = (iy, ix) if transpose else (ix, iy)
            if ix == 1:
                for cy in range(2):
                    for cx in range(2):
                        lv.append((0, 3, 2 * a + (cy if transpose else cx),
                                   2 * b + (cx if transpose else cy)))
            else:
                lv.append((0, 2, a, b))
    return O.sfc_sort(np.array(lv, dtype=O.LEAF_DTYPE))


def _to_segments(lv, q, m, transpose):
    """Oracle interiors -> patch-column rows of the reference (x along the
    columns; transposed forests are read with x and y swapped)."""
    starts = {0: 0, 1: 1, 2: 3, 3: 4}
    seg = [np.zeros((4 * m, m)), np.zeros((8 * m, m)), np.zeros((8 * m, m)),
           np.zeros((4 * m, m)), np.zeros((4 * m, m))]
    for p, a in enumerate(lv):
        lev, ix, iy = int(a["level"]), int(a["ix"]), int(a["iy"])
        blk = q[p, 0]
        if transpose:
            ix, iy = iy, ix
            blk = blk.T
        if lev == 2:
            s = starts[ix]
        else:
            s = 1 + (ix - 2)
        seg[s][iy * m:(iy + 1) * m, :] = blk
    return seg


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("u", [0.8, -0.65])
def test_reflux_rows_equal_mixed_resolution_flux_form(u, transpose):
    m = 8
    trees, pl = I.periodic_square()
    lv = _band_forest(transpose)
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
    ref = _BandReference(m, 4 * m)
    seg = _to_segments(lv, q, m, transpose)
    dt = 0.7 / (m << 3) / abs(u)
    for _ in range(6):
        q, _ = O.advance(mesh, par, q, dt, reflux=True)
        seg = ref.step(seg, u, dt)
        got = _to_segments(lv, q, m, transpose)
        for a, b in zip(got, seg):
            assert np.max(np.abs(a - b)) <= 1e-14 * max(1.0, np.abs(b).max())
    # without the correction the coarse cells at the band differ
    q0 = I.state_from(lv, m, fn, pl)
    qn, _ = O.advance(mesh, par, q0, dt, reflux=False)
    s0 = ref.step(_to_segments(lv, q0, m, transpose), u, dt)
    diff = max(np.max(np.abs(a - b)) for a, b in zip(_to_segments(lv, qn, m, transpose), s0))
    assert diff > 1e-6
