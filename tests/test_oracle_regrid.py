"""Pins of the oracle's tagging and regrid: tag rules on states whose
answer is known, refine-then-coarsen identity, mass invariance, exactness on
linear data, balance after every regrid, the initial-mesh loop."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I
from tests import helpers as H

M = 8


def test_tags_known_cases():
    trees, pl = I.walled_square()
    lv = O.sfc_sort(I.uniform_leaves(1, 2))
    mesh = O.Mesh(trees, lv, M)
    par = O.params(M, O.SHALLOW)
    # flat water: criterion false everywhere -> all families coarsen
    q = I.state_from(lv, M, lambda x, y: I.dam_break(x, y, hin=1.0), pl)
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    assert np.all(O.tags(mesh, par, f, 1, 0.1, 1, 4) == -1)
    assert np.all(O.tags(mesh, par, f, 1, 0.1, 2, 4) == 0)    # at lmin
    # a jump across x = 0.5 refines exactly the patches that see it through
    # their central differences (ghost cells included)
    q = I.state_from(lv, M, lambda x, y: np.stack(
        [np.where(x < 0.5, 2.0, 1.0), 0 * x, 0 * x], axis=1), pl)
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    tg = O.tags(mesh, par, f, 1, 0.1, 1, 4)
    want = np.where((lv["ix"] == 1) | (lv["ix"] == 2), 1, 0)
    # families with no refined member coarsen unless the parent sees the jump
    fam_sees_jump = np.isin(lv["ix"] // 2, [0, 1])   # all parents touch x=0.5
    assert np.all(tg[want == 1] == 1)
    assert np.all(tg[(want == 0) & ~fam_sees_jump] == -1)
    assert np.all(tg[(want == 0) & fam_sees_jump] != 1)
    # the max-min criterion of the paper looks at the interior only: a jump
    # at x = 0.3 lies inside the patches with ix = 1
    q = I.state_from(lv, M, lambda x, y: np.stack(
        [np.where(x < 0.3, 2.0, 1.0), 0 * x, 0 * x], axis=1), pl)
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    tg0 = O.tags(mesh, par, f, 0, 0.5, 1, 4)
    assert np.all(tg0[lv["ix"] == 1] == 1) and np.all(tg0[lv["ix"] != 1] != 1)
    assert np.all(tg0[lv["ix"] >= 2] == -1)
    # at lmax nothing is refined
    assert np.all(O.tags(mesh, par, f, 1, 0.1, 1, 2) != 1)


def test_tag_values_on_linear_data_and_agreement_with_tags():
    """h = 1 + a x + b y with walls far from the sampled cells: every
    interior central difference is exact, so the squared gradient of each
    patch and of each averaged parent is a^2 + b^2; max - min over a patch
    of side s with m cells is (|a| + |b|) s (m - 1) / m.  The tags are the
    decisions the values imply."""
    trees, pl = I.periodic_square()
    lv = O.sfc_sort(I.uniform_leaves(1, 3))
    mesh = O.Mesh(trees, lv, M)
    par = O.params(M, O.ADVECTION)
    a, b = 0.375, -0.25
    # periodic: a linear field jumps at the wrap; take patches away from it
    q = I.state_from(lv, M, lambda x, y: (1.0 + a * x + b * y)[:, None], pl)
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    ref, parent = O.tag_values(mesh, par, f, 1)
    inner = (lv["ix"] > 0) & (lv["ix"] < 7) & (lv["iy"] > 0) & (lv["iy"] < 7)
    np.testing.assert_allclose(ref[inner], a * a + b * b, rtol=1e-12)
    fam = ~np.isnan(parent)
    assert fam.sum() == 16
    inner_fam = fam & (lv["ix"] >= 2) & (lv["ix"] <= 4) & (lv["iy"] >= 2) & (lv["iy"] <= 4)
    np.testing.assert_allclose(parent[inner_fam], a * a + b * b, rtol=1e-12)
    ref0, _ = O.tag_values(mesh, par, f, 0)
    s = 1.0 / 8
    np.testing.assert_allclose(ref0[inner], (abs(a) + abs(b)) * s * (M - 1) / M,
                               rtol=1e-12)
    # tags follow the values: threshold between two distinct values
    for crit, vals in ((1, ref), (0, ref0)):
        thr = np.sqrt(a * a + b * b) * 0.999 if crit == 1 else ref0[inner][0] * 0.999
        tg = O.tags(mesh, par, f, crit, thr, 1, 5)
        t = thr * thr if crit == 1 else thr
        assert np.array_equal(tg == 1, vals > t)


def _regrid(mesh, par, q, tg, lmin, lmax, trees):
    f = O.framed(q, mesh.m)
    O.ghost_fill(mesh, par, f)
    lv2 = O.regrid(mesh, tg, lmin, lmax)
    mesh2 = O.Mesh(trees, lv2, mesh.m)
    f2 = O.transfer(mesh, mesh2, par, f)
    return mesh2, O.interior(f2, mesh.m)


@pytest.mark.parametrize("seed", [0, 1])
def test_refine_then_coarsen_is_identity(seed):
    trees, pl = I.periodic_square()
    lv = O.balance(trees, I.random_leaves(seed, 1, 1, 4, 15))
    mesh = O.Mesh(trees, lv, M)
    par = O.params(M, O.SHALLOW)
    rng = np.random.default_rng(seed)
    q = rng.uniform(1, 2, (len(lv), 3, M, M))
    m0 = O.sums(mesh, par, O.framed(q, M))
    mesh2, q2 = _regrid(mesh, par, q, np.ones(len(lv), np.int8), 0, 9, trees)
    assert len(mesh2) == 4 * len(lv)
    m1 = O.sums(mesh2, par, O.framed(q2, M))
    np.testing.assert_allclose(m1, m0, rtol=1e-14)
    mesh3, q3 = _regrid(mesh2, par, q2, -np.ones(len(mesh2), np.int8), 0, 9,
                        trees)
    assert np.array_equal(mesh3.leaves, mesh.leaves)
    assert np.max(np.abs(q3 - q)) <= 1e-15 * np.max(np.abs(q))


def test_regrid_linear_data_and_balance():
    trees, pl = I.walled_square()
    lv = O.balance(trees, I.random_leaves(4, 1, 2, 5, 20))
    mesh = O.Mesh(trees, lv, M)
    par = O.params(M)
    fn = lambda x, y: 0.2 + 0.7 * x + 1.3 * y
    q = I.state_from(lv, M, fn, pl)
    rng = np.random.default_rng(2)
    tg = rng.integers(-1, 2, len(lv)).astype(np.int8)
    mesh2, q2 = _regrid(mesh, par, q, tg, 1, 6, trees)
    lo, hi = H.leaf_boxes_plane(mesh2.leaves, pl)
    assert H.is_balanced_bruteforce(mesh2.leaves, lo, hi)
    want = I.state_from(mesh2.leaves, M, fn, pl)
    x, y = I.cell_centres(mesh2.leaves, M, pl)
    h = np.ldexp(1.0, -mesh2.leaves["level"].astype(int))[:, None, None] / M
    far = np.minimum.reduce([x, y, 1 - x, 1 - y]) > 6 * h
    err = np.abs(q2[:, 0] - want[:, 0])[far]
    assert err.max() <= 1e-14


def test_initial_mesh_loop_follows_the_dam():
    """Initial AMR mesh: uniform at lmin, tag, refine, re-evaluate the
    initial data, repeat to lmax (the dam edge ends at the finest level)."""
    trees, pl = I.walled_square()
    par = O.params(16, O.SHALLOW)
    lmin, lmax = 2, 4
    fn = lambda x, y: I.dam_break(x, y)
    lv = O.sfc_sort(I.uniform_leaves(1, lmin))
    for _ in range(lmax - lmin + 1):
        mesh = O.Mesh(trees, lv, 16)
        q = I.state_from(lv, 16, fn, pl)
        f = O.framed(q, 16)
        O.ghost_fill(mesh, par, f)
        tg = O.tags(mesh, par, f, 1, 0.1, lmin, lmax)
        lv2 = O.regrid(mesh, tg, lmin, lmax)
        if np.array_equal(lv2, lv):
            break
        lv = lv2
    mesh = O.Mesh(trees, lv, 16)
    assert mesh.balanced()
    x, y = I.cell_centres(lv, 16, pl)
    r = np.hypot(x - 0.5, y - 0.5)
    near = np.any(np.abs(r - 0.25) < 1.0 / 256, axis=(1, 2))
    assert np.all(lv["level"][near] == lmax)
    assert lmin <= lv["level"].min() < lmax
