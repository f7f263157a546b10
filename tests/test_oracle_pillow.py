"""Pins of the oracle's two-tree (pillow) sphere, the geometry of the
paper's Sec. 5 sphere example (one quadtree per hemisphere), and of the
rigid rotation on it, against facts outside the oracle:

- the cells of a uniform forest tile the sphere: total area 4 pi (from the
  capacities); every capacity positive (both trees right-handed), also in
  the ghost layers.  (Unlike the gnomonic cube map, this map does not send
  grid lines to great circles, so the midpoint of a coarse cell's edge,
  mapped as a fine cell's corner, lies off the coarse cell's great-circle
  edge: adaptive forests tile the sphere only up to that offset, which
  falls with the cell size);
- the map sends each tree's boundary to the equator and the glued faces to
  the same points (the map written out here: the circle of polar angle
  d pi / 2 for the square of half-width d);
- an edge on the equator seen from either tree has the identical length
  and the equal or opposite normal, bit for bit; ghost cells carry the
  capacity of the cell whose value they hold;
- the rotation's edge fluxes are the arc integrals of the closed-form
  velocity along the edges (corners mapped here), and the discrete field is
  exactly divergence free on every frame cell (no corner is left uncovered:
  the region beyond a square corner is the own tree's corner mirrored);
- under refinement a function of the axis coordinate stays steady and one
  turn returns the state, both to errors that fall at second order.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I
from tests.test_oracle_rotation import AXIS, _arc_flux

PI = np.pi
M = 8


def _mesh(lv, m=M):
    return O.Mesh(I.pillow_sphere(), lv, m, sphere=True)


def _pt(tree, xi, eta):
    """the map, written out"""
    x, y = 2 * xi - 1, 2 * eta - 1
    d = max(abs(x), abs(y))
    if d == 0:
        r = np.array([0.0, 0.0, 1.0])
    else:
        th = 0.5 * PI * d
        r = np.array([np.sin(th) * x, np.sin(th) * y, 0.0]) / np.hypot(x, y)
        r[2] = np.cos(th)
    if tree == 1:
        r[1:] = -r[1:]
    return r


@pytest.mark.parametrize("seed", [None, 1, 2])
def test_total_area_is_4pi_and_capacities_positive(seed):
    trees = I.pillow_sphere()
    lv = O.sfc_sort(I.uniform_leaves(2, 2)) if seed is None else \
        O.balance(trees, I.random_leaves(seed, 2, 1, 4, 16))
    mesh = _mesh(lv)
    tot = 0.0
    for p, a in enumerate(lv):
        dx = 2.0 ** -int(a["level"]) / M
        for j in range(-1, M + 3):
            for i in range(-1, M + 3):
                k = O.sphere_kappa(mesh, p, i, j)
                if (i in (-1, M + 2)) and (j in (-1, M + 2)):
                    continue           # outermost corners: never used
                assert k > 0
                if 1 <= i <= M and 1 <= j <= M:
                    tot += k * dx * dx
    assert abs(tot / (4 * PI) - 1) <= (1e-13 if seed is None else 3e-4)


def test_map_glues_the_trees_along_the_equator():
    rng = np.random.default_rng(1)
    for s in rng.uniform(0, 1, 20):
        for t in (0, 1):
            for xi, eta in ((0.0, s), (1.0, s), (s, 0.0), (s, 1.0)):
                assert _pt(t, xi, eta)[2] == 0.0 or abs(_pt(t, xi, eta)[2]) < 1e-16
        # faces 2 <-> 3 the same way, faces 0 <-> 0 and 1 <-> 1 reversed
        np.testing.assert_allclose(_pt(0, s, 0.0), _pt(1, s, 1.0), atol=1e-15)
        np.testing.assert_allclose(_pt(0, s, 1.0), _pt(1, s, 0.0), atol=1e-15)
        np.testing.assert_allclose(_pt(0, 0.0, s), _pt(1, 0.0, 1 - s), atol=1e-15)
        np.testing.assert_allclose(_pt(0, 1.0, s), _pt(1, 1.0, 1 - s), atol=1e-15)
    # the oracle's centres are the map's images of the computational centres
    lv = O.balance(I.pillow_sphere(), I.random_leaves(4, 2, 1, 3, 8))
    mesh = _mesh(lv)
    for p, a in enumerate(lv):
        h = 2.0 ** -int(a["level"]) / M
        for (i, j) in ((1, 1), (3, M), (M, 5)):
            xi = int(a["ix"]) * M * h + (i - 0.5) * h
            eta = int(a["iy"]) * M * h + (j - 0.5) * h
            np.testing.assert_allclose(O.sphere_centre(mesh, p, i, j), _pt(int(a["tree"]), xi, eta),
                                       atol=2e-16)


def test_shared_edges_are_bit_equal_across_the_equator():
    lv = O.sfc_sort(I.uniform_leaves(2, 1))
    mesh = _mesh(lv)
    key = {}
    for p, a in enumerate(lv):
        for f in range(4):
            for t in range(1, M + 1):
                if f < 2:
                    i, j, d = (1 if f == 0 else M + 1), t, 0
                else:
                    i, j, d = t, (1 if f == 2 else M + 1), 1
                g, n, tt = O.sphere_edge(mesh, p, d, i, j)
                c1 = O.sphere_centre(mesh, p, i, j)
                c0 = O.sphere_centre(mesh, p, i - 1, j) if d == 0 else O.sphere_centre(mesh, p, i, j - 1)
                # a corner cell meets the other tree's corner cell along two
                # edges (both on the equator): their tangents tell them apart
                k = tuple(np.round(c0 + c1, 9)) + tuple(np.round(np.abs(tt), 9))
                key.setdefault(k, []).append((g, n))
    shared = [v for v in key.values() if len(v) == 2]
    # every edge on a patch face: 8 patches x 4 faces x M edges, each seen twice
    assert len(shared) == 8 * 4 * M // 2
    for (g1, n1), (g2, n2) in shared:
        assert g1 == g2
        assert np.array_equal(n1, n2) or np.array_equal(n1, -n2)


def test_ghost_geometry_is_the_neighbours():
    lv = O.sfc_sort(I.uniform_leaves(2, 2))
    mesh = _mesh(lv)
    cen = {}
    for p in range(len(lv)):
        for j in range(1, M + 1):
            for i in range(1, M + 1):
                cen[tuple(np.round(O.sphere_centre(mesh, p, i, j), 12))] = O.sphere_kappa(mesh, p, i, j)
    hits = 0
    for p in range(len(lv)):
        for j in range(-1, M + 3):
            for i in range(-1, M + 3):
                if (1 <= i <= M and 1 <= j <= M) or ((i in (-1, M + 2)) and (j in (-1, M + 2))):
                    continue
                k = tuple(np.round(O.sphere_centre(mesh, p, i, j), 12))
                assert k in cen, (p, i, j)
                hits += 1
                assert abs(O.sphere_kappa(mesh, p, i, j) - cen[k]) <= 1e-14 * cen[k]
    assert hits == len(lv) * (8 * M + 12)


def test_rotation_fluxes_are_arc_integrals_and_divergence_free():
    trees = I.pillow_sphere()
    lv = O.balance(trees, I.random_leaves(6, 2, 1, 3, 12))
    mesh = _mesh(lv)
    T = 1.7
    par = O.params(M, O.ROTATION, period=T, axis=AXIS)
    w = np.array(AXIS) / np.linalg.norm(AXIS)
    omega = 2 * PI / T
    rng = np.random.default_rng(8)
    for _ in range(200):
        p = int(rng.integers(len(lv)))
        a = lv[p]
        d = int(rng.integers(2))
        i, j = (int(v) for v in rng.integers(1, M + 1, 2))
        h = 1.0 / ((1 << int(a["level"])) * M)
        xi0, eta0 = (int(a["ix"]) * M + i - 1) * h, (int(a["iy"]) * M + j - 1) * h
        t = int(a["tree"])
        A = _pt(t, xi0, eta0)
        B = _pt(t, xi0 + (d == 1) * h, eta0 + (d == 0) * h)
        cr = _pt(t, xi0 + h / 2, eta0 + h / 2)
        cl = _pt(t, xi0 + h / 2 - (d == 0) * h, eta0 + h / 2 - (d == 1) * h)
        nsign = 1.0 if np.dot(np.cross(A, B), cr - cl) > 0 else -1.0
        want = _arc_flux(A, B, omega, w, nsign) / h
        assert abs(O.rotation_edge(mesh, par, p, d, i, j) - want) <= 1e-11 * omega
    for p in range(len(lv)):
        scale = 1e-12 * omega * M * (1 << int(lv[p]["level"]))
        for j in range(0, M + 2):
            for i in range(0, M + 2):
                e = lambda dd, ii, jj: O.rotation_edge(mesh, par, p, dd, ii, jj)
                div = e(0, i + 1, j) - e(0, i, j) + e(1, i, j + 1) - e(1, i, j)
                assert abs(div) <= scale, (p, i, j, div)


def _run(level, q_fn, t_end, T, m=M, cfl=0.4):
    lv = O.sfc_sort(I.uniform_leaves(2, level))
    mesh = _mesh(lv, m)
    q = I.sphere_scalar(lv, m, q_fn, pillow=True)
    par = O.params(m, O.ROTATION, period=T, axis=AXIS)
    # the equator cells are the largest: about pi / 2 per level-0 side
    h = (PI / 2) / (m << level)
    nsteps = int(np.ceil(t_end * (2 * PI / T) / (cfl * h)))
    dt = t_end / nsteps
    q0 = q.copy()
    for _ in range(nsteps):
        q, nu = O.advance(mesh, par, q, dt)
        assert nu <= 1.0
    return q0, q


def _wr(r):
    w = np.array(AXIS) / np.linalg.norm(AXIS)
    return np.einsum("pkij,k->pij", r, w)


def test_rotation_on_the_pillow_converges():
    steady, turn = [], []
    c = np.array([0.6, 0.0, 0.8])
    blob = lambda r: np.exp(-4.0 * np.sum((r - c[None, :, None, None]) ** 2, axis=1))
    for level in (1, 2, 3):
        q0, q = _run(level, lambda r: np.cos(3 * _wr(r)), 0.25, 1.0)
        steady.append(np.mean(np.abs(q - q0)))
        q0, q = _run(level, blob, 1.0, 1.0)
        turn.append(np.mean(np.abs(q - q0)) / np.mean(np.abs(q0)))
    assert steady[0] / steady[1] > 3.0 and steady[1] / steady[2] > 3.0, steady
    assert turn[0] / turn[1] > 3.0 and turn[1] / turn[2] > 3.0, turn
    assert steady[-1] < 5e-3 and turn[-1] < 0.03


def test_corner_ghosts_are_the_own_corner_mirrored():
    """Beyond a square corner (where only the two trees' corner cells meet)
    the ghost cells hold the own tree's cells mirrored through the corner:
    frame cell (1 - a, 1 - b) of the corner patch holds its cell (a, b)."""
    trees = I.pillow_sphere()
    lv = O.sfc_sort(I.uniform_leaves(2, 1))
    mesh = _mesh(lv)
    par = O.params(M, O.ROTATION, axis=AXIS)
    q = np.random.default_rng(3).random((len(lv), 1, M, M))
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    seen = 0
    for p, a in enumerate(lv):
        n = 1 << int(a["level"])
        for cx in (0, 1):
            for cy in (0, 1):
                if int(a["ix"]) != cx * (n - 1) or int(a["iy"]) != cy * (n - 1):
                    continue
                seen += 1
                for da in (1, 2):
                    for db in (1, 2):
                        # own cell (i, j) counted from the corner, and its mirror
                        i = da if cx == 0 else M + 1 - da
                        j = db if cy == 0 else M + 1 - db
                        gi = 1 - da if cx == 0 else M + da
                        gj = 1 - db if cy == 0 else M + db
                        if (gi in (-1, M + 2)) and (gj in (-1, M + 2)):
                            continue           # outermost corner: never used
                        assert f[p, 0, gj + 1, gi + 1] == f[p, 0, j + 1, i + 1]
    assert seen == 8          # four corners in each of the two trees
