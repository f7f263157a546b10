"""Pins of the oracle's wave-propagation step: Roe property, limiter
function, free stream / lake at rest, exact shifts at CFL 1, 1D reduction
against an independent flux-limited Lax-Wendroff routine, convergence for
translation and for the exact dam break, forest = uniform grid, mass
conservation with and without the coarse-fine reflux, D4 symmetry."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sw_flux(q, d, g=1.0):
    h, hu, hv = q
    u, v = hu / h, hv / h
    if d == 0:
        return np.array([hu, hu * u + 0.5 * g * h * h, hu * v])
    return np.array([hv, hv * u, hv * v + 0.5 * g * h * h])


@pytest.mark.parametrize("d", [0, 1])
def test_roe_property_and_wave_sum(d):
    rng = np.random.default_rng(5 + d)
    par = O.params(8, O.SHALLOW, g=1.3)
    for _ in range(50):
        ql = np.array([rng.uniform(0.5, 3), rng.normal(), rng.normal()])
        qr = np.array([rng.uniform(0.5, 3), rng.normal(), rng.normal()])
        W, s, am, ap = O.riemann(par, d, ql, qr)
        np.testing.assert_allclose(W.sum(axis=0), qr - ql, rtol=0, atol=1e-13)
        np.testing.assert_allclose(am + ap, sw_flux(qr, d, 1.3) - sw_flux(ql, d, 1.3),
                                   rtol=0, atol=1e-12)
        assert s[0] < s[1] < s[2]
    par = O.params(8, O.ADVECTION, ax=-0.7, ay=0.4)
    W, s, am, ap = O.riemann(par, d, np.array([2.0]), np.array([-1.0]))
    a = (-0.7, 0.4)[d]
    assert s[0] == a and np.allclose(am + ap, a * (-3.0))


def test_limiter_properties():
    """Textbook values and the symmetry phi(t)/t = phi(1/t) of the limiters
    (LeVeque 2002, Sec. 6.12); second order needs phi(1) = 1."""
    known = {1: [(0.5, 0.5), (2.0, 1.0), (-1.0, 0.0)],
             2: [(0.5, 1.0), (1.5, 1.5), (3.0, 2.0)],
             3: [(1.0, 1.0), (3.0, 1.5), (-2.0, 0.0)],
             4: [(1.0 / 3.0, 2.0 / 3.0), (3.0, 2.0), (1.0, 1.0), (-0.5, 0.0)]}
    for lim, pairs in known.items():
        for th, want in pairs:
            assert abs(O.phi(lim, th) - want) < 1e-15
        for th in (0.2, 0.7, 1.9, 4.0):
            assert abs(O.phi(lim, th) / th - O.phi(lim, 1.0 / th)) < 1e-14
            assert 0.0 <= O.phi(lim, th) <= min(2.0, 2.0 * th) + 1e-15
    assert O.phi(0, -3.0) == 1.0


@pytest.mark.parametrize("physics", [O.ADVECTION, O.SHALLOW])
def test_free_stream_and_lake_at_rest_bitwise(physics):
    if physics == O.ADVECTION:
        trees, pl = I.periodic_square()
        par = O.params(8, physics, ax=0.8, ay=-0.45)
        c = np.array([0.731])
    else:
        trees, pl = I.walled_square()
        par = O.params(8, physics)
        c = np.array([1.5, 0.0, 0.0])
    lv = O.balance(trees, I.random_leaves(21, 1, 2, 5, 30))
    mesh = O.Mesh(trees, lv, 8)
    q = np.broadcast_to(c[None, :, None, None], (len(lv), par.meqn, 8, 8)).copy()
    for _ in range(3):
        q, _ = O.advance(mesh, par, q, 0.5 / 256)
    for k in range(par.meqn):
        assert np.all(q[:, k] == c[k])


def _uniform_periodic(level, m):
    trees, pl = I.periodic_square()
    lv = O.sfc_sort(I.uniform_leaves(1, level))
    return trees, pl, lv, O.Mesh(trees, lv, m)


def _assemble(lv, q, m, level):
    n = m << level
    big = np.zeros((q.shape[1], n, n))
    for p, a in enumerate(lv):
        big[:, a["iy"] * m:(a["iy"] + 1) * m, a["ix"] * m:(a["ix"] + 1) * m] = q[p]
    return big


@pytest.mark.parametrize("a", [(1.0, 0.0), (1.0, 1.0), (0.0, -1.0)])
def test_exact_shift_at_cfl_one(a):
    m, level = 8, 2
    trees, pl, lv, mesh = _uniform_periodic(level, m)
    par = O.params(m, O.ADVECTION, ax=a[0], ay=a[1])
    h = 1.0 / (m << level)
    q = I.state_from(lv, m, lambda x, y: np.sin(2 * np.pi * x) + np.cos(6 * np.pi * y) * x, pl)
    big0 = _assemble(lv, q, m, level)
    for _ in range(3):
        q, nu = O.advance(mesh, par, q, h)
    assert abs(nu - 1.0) < 1e-15
    big = _assemble(lv, q, m, level)
    want = np.roll(big0, (3 * int(a[1]), 3 * int(a[0])), axis=(1, 2))
    assert np.max(np.abs(big - want)) <= 1e-14


def _lw1d(q, u, nu, steps, lim):
    """Independent 1D flux-limited Lax-Wendroff (LeVeque 2002, Sec. 6.12),
    periodic, u > 0: F_{i-1/2} = u Q_{i-1} + u/2 (1 - nu) phi(theta) dQ."""
    def phi(t):
        if lim == 4:
            return np.maximum(0, np.minimum(np.minimum((1 + t) / 2, 2), 2 * t))
        raise ValueError
    for _ in range(steps):
        dq = q - np.roll(q, 1)                  # at edge i-1/2
        up = np.roll(dq, 1)                     # edge i-3/2
        with np.errstate(divide="ignore", invalid="ignore"):
            th = np.where(dq != 0, up * dq / np.where(dq != 0, dq * dq, 1), 0)
        F = u * np.roll(q, 1) + 0.5 * u * (1 - nu) * np.where(dq != 0, phi(th), 0) * dq
        q = q - nu / u * (np.roll(F, -1) - F)
    return q


def test_one_dimensional_reduction():
    m, level = 8, 1
    trees, pl, lv, mesh = _uniform_periodic(level, m)
    u = 0.9
    par = O.params(m, O.ADVECTION, ax=u, ay=0.0)
    n = m << level
    h = 1.0 / n
    dt = 0.8 * h / u
    fn = lambda x, y: np.where(np.abs(x - 0.4) < 0.2, 1.0, 0.0) + 0.3 * np.sin(2 * np.pi * x) + 0 * y
    q = I.state_from(lv, m, fn, pl)
    row0 = _assemble(lv, q, m, level)[0, 0]
    for _ in range(7):
        q, _ = O.advance(mesh, par, q, dt)
    big = _assemble(lv, q, m, level)[0]
    want = _lw1d(row0.copy(), u, u * dt / h, 7, 4)
    for r in range(n):
        assert np.max(np.abs(big[r] - want)) <= 1e-14


def test_translation_converges():
    """Gaussian translated by a = (1, 0.5) on the periodic square; exact
    solution known in closed form.  MC clips extrema, so order >= 1.5."""
    errs = []
    a = (1.0, 0.5)
    T = 0.25
    for level in (2, 3, 4, 5):
        m = 8
        trees, pl, lv, mesh = _uniform_periodic(level, m)
        par = O.params(m, O.ADVECTION, ax=a[0], ay=a[1])
        h = 1.0 / (m << level)
        nsteps = int(np.ceil(T / (0.9 * h)))
        dt = T / nsteps
        q = I.state_from(lv, m, lambda x, y: I.periodic_gaussian(x, y, 0.5, 0.5), pl)
        for _ in range(nsteps):
            q, _ = O.advance(mesh, par, q, dt)
        ex = I.state_from(lv, m, lambda x, y: I.periodic_gaussian(
            x, y, (0.5 + a[0] * T) % 1.0, (0.5 + a[1] * T) % 1.0), pl)
        errs.append(np.sum(np.abs(q - ex)) * h * h)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert all(e1 > e2 for e1, e2 in zip(errs, errs[1:]))
    assert orders[-1] >= 1.5, (errs, orders)


def _dambreak_exact(x, t, ex):
    g = ex["g"]
    hl, hs, us = ex["h_left"], ex["h_star"], ex["u_star"]
    xi = (x - 0.5) / t
    h = np.full_like(x, ex["h_right"])
    h = np.where(xi < ex["shock_speed"], hs, h)
    rare = (xi >= ex["rarefaction_head"]) & (xi < ex["rarefaction_tail"])
    # inside the rarefaction: u - 2c = -2 sqrt(g hl) and u - c = xi
    c = (2 * np.sqrt(g * hl) - xi) / 3.0
    h = np.where(rare, c * c / g, h)
    h = np.where(xi < ex["rarefaction_head"], hl, h)
    return h


def test_dam_break_converges_to_exact():
    ex = json.load(open(os.path.join(GOLDEN, "dambreak_exact.json")))
    trees, pl = I.walled_square()
    T = 0.12
    errs, plateau = [], None
    for level in (2, 3, 4, 5):
        m = 8
        lv = O.sfc_sort(I.uniform_leaves(1, level))
        mesh = O.Mesh(trees, lv, m)
        par = O.params(m, O.SHALLOW, g=ex["g"])
        h = 1.0 / (m << level)
        nsteps = int(np.ceil(T / (0.5 * h)))
        dt = T / nsteps
        q = I.state_from(lv, m, lambda x, y: np.stack(
            [np.where(x < 0.5, 2.0, 1.0), 0 * x, 0 * x], axis=1), pl)
        for _ in range(nsteps):
            q, nu = O.advance(mesh, par, q, dt)
            assert nu < 1.0
        big = _assemble(lv, q, m, level)
        n = m << level
        x = (np.arange(n) + 0.5) * h
        row = big[0, n // 2]
        assert np.max(np.abs(big[0] - row[None, :])) <= 1e-13   # 1D data stays 1D
        assert np.max(np.abs(big[2])) <= 1e-13                 # no transverse momentum
        errs.append(np.sum(np.abs(row - _dambreak_exact(x, T, ex))) * h)
        mid = (x - 0.5) / T
        sel = (mid > ex["rarefaction_tail"] + 0.15) & (mid < ex["shock_speed"] - 0.15)
        plateau = np.mean(row[sel]) if sel.any() else None
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert all(e1 > e2 for e1, e2 in zip(errs, errs[1:])), errs
    assert np.mean(orders) >= 0.5, orders
    assert abs(plateau - ex["h_star"]) < 1e-3


@pytest.mark.parametrize("physics", [O.ADVECTION, O.SHALLOW])
def test_uniform_forest_equals_single_patch_bitwise(physics):
    level, m = 2, 8
    n = m << level
    if physics == O.ADVECTION:
        trees, pl = I.periodic_square()
        par_f = O.params(m, physics, ax=1.0, ay=0.5)
        par_1 = O.params(n, physics, ax=1.0, ay=0.5)
        fn = lambda x, y: I.gaussian(x, y)
        dt = 0.9 / n
    else:
        trees, pl = I.walled_square()
        par_f = O.params(m, physics)
        par_1 = O.params(n, physics)
        fn = lambda x, y: I.dam_break(x, y, 0.45, 0.55, 0.25)
        dt = 0.4 / n
    lv = O.sfc_sort(I.uniform_leaves(1, level))
    mesh = O.Mesh(trees, lv, m)
    one = O.sfc_sort(I.uniform_leaves(1, 0))
    mesh1 = O.Mesh(trees, one, n)
    q = I.state_from(lv, m, fn, pl)
    q1 = I.state_from(one, n, fn, pl)
    assert np.array_equal(_assemble(lv, q, m, level), q1[0])
    for _ in range(6):
        q, nu = O.advance(mesh, par_f, q, dt)
        q1, nu1 = O.advance(mesh1, par_1, q1, dt)
        assert nu == nu1
    assert np.array_equal(_assemble(lv, q, m, level), q1[0])


def test_mass_uniform_periodic():
    m, level = 8, 2
    trees, pl, lv, mesh = _uniform_periodic(level, m)
    par = O.params(m, O.ADVECTION, ax=1.0, ay=0.5)
    q = I.state_from(lv, m, lambda x, y: I.gaussian(x, y), pl)
    m0 = O.sums(mesh, par, O.framed(q, m))[0]
    for _ in range(100):
        q, _ = O.advance(mesh, par, q, 0.028125)
    m1 = O.sums(mesh, par, O.framed(q, m))[0]
    assert abs(m1 - m0) / abs(m0) <= 1e-13


def _adaptive_sw(seed=31):
    trees, pl = I.walled_square()
    raw = I.refine_near(1, 2, 4, [(0.5, 0.5)], pl, radius=1.2)
    lv = O.balance(trees, np.concatenate([raw]))
    return trees, pl, lv


@pytest.mark.parametrize("physics", [O.SHALLOW, O.ADVECTION])
def test_mass_conserved_adaptive_with_reflux(physics):
    m = 8
    if physics == O.SHALLOW:
        trees, pl, lv = _adaptive_sw()
        par = O.params(m, physics)
        fn = lambda x, y: I.dam_break(x, y, 0.5, 0.5, 0.25)
        dt = 0.3 / (m << 4)
    else:
        trees, pl = I.periodic_square()
        lv = O.balance(trees, I.random_leaves(8, 1, 2, 4, 20))
        par = O.params(m, physics, ax=0.7, ay=-0.4)
        fn = lambda x, y: I.gaussian(x, y, 0.4, 0.6)
        dt = 0.8 / (m << 4) / 0.7
    mesh = O.Mesh(trees, lv, m)
    assert len(set(lv["level"].tolist())) >= 2
    q0 = I.state_from(lv, m, fn, pl)
    m0 = O.sums(mesh, par, O.framed(q0, m))
    q, qnr = q0.copy(), q0.copy()
    for _ in range(40):
        q, _ = O.advance(mesh, par, q, dt, reflux=True)
        qnr, _ = O.advance(mesh, par, qnr, dt, reflux=False)
    m1 = O.sums(mesh, par, O.framed(q, m))
    mnr = O.sums(mesh, par, O.framed(qnr, m))
    assert abs(m1[0] - m0[0]) / abs(m0[0]) <= 1e-13
    drift_nr = abs(mnr[0] - m0[0]) / abs(m0[0])
    assert drift_nr > 1e-11          # without reflux the scheme leaks
    if physics == O.SHALLOW:
        # momentum: the walls exchange momentum with the fluid, but
        # the dam break stays symmetric about the centre: total momentum 0
        assert abs(m1[1]) < 1e-12 and abs(m1[2]) < 1e-12


def test_radial_dam_break_symmetry():
    m, level = 8, 2
    trees, pl = I.walled_square()
    lv = O.sfc_sort(I.uniform_leaves(1, level))
    mesh = O.Mesh(trees, lv, m)
    par = O.params(m, O.SHALLOW)
    q = I.state_from(lv, m, lambda x, y: I.dam_break(x, y), pl)
    n = m << level
    for _ in range(60):
        q, _ = O.advance(mesh, par, q, 0.3 / n)
    big = _assemble(lv, q, m, level)
    h, hu, hv = big
    err = max(np.max(np.abs(h - h.T)), np.max(np.abs(h - h[::-1, :])),
              np.max(np.abs(h - h[:, ::-1])), np.max(np.abs(hu - hv.T)),
              np.max(np.abs(hu + hu[:, ::-1])), np.max(np.abs(hv + hv[::-1, :])))
    assert err <= 1e-10


@pytest.mark.parametrize("sphere", [False, True])
def test_threads_do_not_change_results(sphere):
    """The ghost fill and the step's patch loop split whole patches over
    threads (for the CPU baseline's all-core timing): with 1 and with 4
    threads every value, nu_max and the nesting depth are bit for bit the
    same, on an adaptive forest with coarse-fine faces and reflux."""
    from paper_1308_1472_amd import fcx
    if sphere:
        trees = I.cubed_sphere()
        lv = fcx.balance(trees, I.random_leaves(5, 6, 1, 3, 10))
        m = 8
        q = I.sphere_bump(lv, m)
        par = O.params(m, O.SPHERE)
    else:
        trees, pl = I.walled_square()
        lv = O.balance(trees, I.random_leaves(5, 1, 2, 5, 40))
        m = 8
        q = I.state_from(lv, m, lambda x, y: I.dam_break(x, y), pl)
        par = O.params(m, O.SHALLOW)
    mesh = O.Mesh(trees, lv, m, sphere=sphere)
    out = []
    try:
        for t in (1, 4):
            O.set_threads(t)
            f = O.framed(q, m)
            depth = O.ghost_fill(mesh, par, f)
            fn, nu = O.step(mesh, par, f, 1e-3, True)
            out.append((f, fn, nu, depth))
    finally:
        O.set_threads(1)
    (f1, n1, nu1, d1), (f4, n4, nu4, d4) = out
    assert np.array_equal(f1, f4, equal_nan=True)
    assert np.array_equal(n1, n4, equal_nan=True)
    assert nu1 == nu4 and d1 == d4
