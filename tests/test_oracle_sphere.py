"""Pins of the oracle's cubed-sphere geometry and solver: total area 4 pi,
bit-equal shared edges across cube edges, ghost geometry equal to the
neighbour's, the Roe property of the rotated solver, lake at rest, exact
mass conservation on adaptive meshes, and invariance under a rotation of
the cube."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I

M = 8


def _mesh(leaves):
    return O.Mesh(I.cubed_sphere(), leaves, M, sphere=True)


def _area(mesh, leaves):
    tot = 0.0
    for p, a in enumerate(leaves):
        dx = 2.0 ** -int(a["level"]) / M
        for j in range(1, M + 1):
            for i in range(1, M + 1):
                tot += O.sphere_kappa(mesh, p, i, j) * dx * dx
    return tot


@pytest.mark.parametrize("seed", [None, 1, 2])
def test_total_area_is_4pi(seed):
    trees = I.cubed_sphere()
    lv = O.sfc_sort(I.uniform_leaves(6, 2)) if seed is None else \
        O.balance(trees, I.random_leaves(seed, 6, 1, 4, 20))
    assert abs(_area(_mesh(lv), lv) / (4 * np.pi) - 1) <= 1e-13


def test_edges_normals_and_tangents():
    lv = O.sfc_sort(I.uniform_leaves(6, 1))
    mesh = _mesh(lv)
    for p in range(len(lv)):
        for j in range(1, M + 1):
            for i in range(1, M + 2):
                for d in (0, 1):
                    ii, jj = (i, j) if d == 0 else (j, i)
                    g, n, t = O.sphere_edge(mesh, p, d, ii, jj)
                    lo = (ii - 1, jj) if d == 0 else (ii, jj - 1)
                    rl, rr = O.sphere_centre(mesh, p, *lo), O.sphere_centre(mesh, p, ii, jj)
                    assert np.dot(n, rr - rl) > 0               # towards higher index
                    assert abs(np.dot(n, n) - 1) < 1e-15 and abs(np.dot(t, t) - 1) < 1e-15
                    assert abs(np.dot(n, t)) < 1e-15
                    mid = rl + rr
                    assert abs(np.dot(n, mid)) < 1e-2 * np.linalg.norm(mid)
                    # arc length close to the centre distance in the other direction
                    assert 0.5 < g * 2.0 ** -1 / M / np.arccos(np.clip(np.dot(rl, rr), -1, 1)) < 2


def test_shared_edges_are_bit_equal_across_cube_edges():
    """Every patch face on a cube edge: the same physical edges seen from the
    neighbouring face have the identical length and the opposite or equal
    normal, bit for bit."""
    trees = I.cubed_sphere()
    lv = O.sfc_sort(I.uniform_leaves(6, 1))
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
                # identify the edge by the two cell centres it separates
                c1 = O.sphere_centre(mesh, p, i, j)
                c0 = O.sphere_centre(mesh, p, i - 1, j) if d == 0 else O.sphere_centre(mesh, p, i, j - 1)
                k = tuple(np.round(c0 + c1, 9))
                key.setdefault(k, []).append((g, n))
    shared = [v for v in key.values() if len(v) == 2]
    assert len(shared) == 6 * 4 * 2 * M // 2 + 6 * 4 * M  # all edges on patch faces
    for (g1, n1), (g2, n2) in shared:
        assert g1 == g2
        assert np.array_equal(n1, n2) or np.array_equal(n1, -n2)


def test_ghost_geometry_is_the_neighbours():
    lv = O.sfc_sort(I.uniform_leaves(6, 1))
    mesh = _mesh(lv)
    cen = {}
    for p in range(len(lv)):
        for j in range(1, M + 1):
            for i in range(1, M + 1):
                cen[tuple(np.round(O.sphere_centre(mesh, p, i, j), 12))] = \
                    O.sphere_kappa(mesh, p, i, j) * 4 ** -int(lv[p]["level"])
    hits = 0
    for p in range(len(lv)):
        for j in range(-1, M + 3):
            for i in range(-1, M + 3):
                if 1 <= i <= M and 1 <= j <= M:
                    continue
                k = tuple(np.round(O.sphere_centre(mesh, p, i, j), 12))
                if k in cen:
                    hits += 1
                    kap = O.sphere_kappa(mesh, p, i, j) * 4 ** -int(lv[p]["level"])
                    assert abs(kap - cen[k]) <= 1e-14 * cen[k]
    assert hits > 24 * 4 * 2 * M


def test_rotated_riemann_roe_property():
    par = O.params(M, O.SPHERE, g=1.3)
    rng = np.random.default_rng(0)
    for _ in range(20):
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        r = rng.normal(size=3); r -= np.dot(r, n) * n; r /= np.linalg.norm(r)
        t = np.cross(r, n)
        gam = rng.uniform(0.5, 2)
        ql = np.concatenate([[rng.uniform(0.5, 2)], rng.normal(size=3) * 0.3])
        qr = np.concatenate([[rng.uniform(0.5, 2)], rng.normal(size=3) * 0.3])
        W, s, am, ap, fl = O.riemann_sphere(par, gam, n, t, ql, qr)

        def flux(q):
            h, mn, mt = q[0], q[1:] @ n, q[1:] @ t
            return np.array([mn, mn * mn / h + 0.5 * 1.3 * h * h, mn * mt / h])
        df = gam * (flux(qr) - flux(ql))
        tot = am + ap
        np.testing.assert_allclose([tot[0], tot[1:] @ n, tot[1:] @ t], df, rtol=1e-12, atol=1e-13)
        assert abs(tot[1:] @ r) < 1e-13                     # no radial part
        assert fl == pytest.approx(0.5 * gam * ((ql[1:] + qr[1:]) @ n) - 0.5 * (ap[0] - am[0]))
        np.testing.assert_allclose(W.sum(axis=0)[0], qr[0] - ql[0], rtol=1e-12, atol=1e-14)


def test_lake_at_rest_is_bitwise_unchanged():
    trees = I.cubed_sphere()
    lv = O.balance(trees, I.random_leaves(4, 6, 1, 4, 15))
    mesh = _mesh(lv)
    par = O.params(M, O.SPHERE)
    q = np.zeros((len(lv), 4, M, M))
    q[:, 0] = 1.0
    q0 = q.copy()
    for _ in range(3):
        q, _ = O.advance(mesh, par, q, 0.004)
    assert np.array_equal(q, q0)


@pytest.mark.parametrize("transverse", [0, 2])
def test_mass_is_conserved_exactly(transverse):
    trees = I.cubed_sphere()
    lv = O.balance(trees, I.random_leaves(3, 6, 2, 3, 12))
    mesh = _mesh(lv)
    par = O.params(M, O.SPHERE, transverse=transverse)
    q = I.sphere_bump(lv, M)
    # the bump on a cube vertex stresses the three-face corners
    q += I.sphere_bump(lv, M, lat=np.arcsin(1 / np.sqrt(3)), lon=np.pi / 4, amp=0.05)
    f = O.framed(q, M); O.ghost_fill(mesh, par, f)
    m0 = O.sums(mesh, par, f)[0]
    dt = 0.35 * (np.pi / 2) / (M * 8) / 1.1
    for _ in range(60):
        q, nu = O.advance(mesh, par, q, dt)
    assert nu < 1.0
    f = O.framed(q, M); O.ghost_fill(mesh, par, f)
    assert abs(O.sums(mesh, par, f)[0] / m0 - 1) <= 1e-13
    # momentum stays tangent
    r = I.sphere_centres(lv, M)
    assert np.abs(np.einsum("pkij,pkij->pij", q[:, 1:], r)).max() < 1e-15


def _rotate_index(lv):
    """Image under the rotation by 90 degrees about z of every leaf and cell
    of a uniform forest: (leaf index, cell permutation) per leaf."""
    n = 1 << int(lv[0]["level"])
    where = {(int(a["tree"]), int(a["ix"]), int(a["iy"])): p for p, a in enumerate(lv)}
    out = []
    for a in lv:
        t, x, y = int(a["tree"]), int(a["ix"]), int(a["iy"])
        if t < 4:
            out.append((where[((t + 1) % 4, x, y)], "id"))
        elif t == 4:   # (xi, eta) -> (1 - eta, xi)
            out.append((where[(4, n - 1 - y, x)], "r4"))
        else:          # (xi, eta) -> (eta, 1 - xi)
            out.append((where[(5, y, n - 1 - x)], "r5"))
    return out


def test_rotation_of_the_cube_maps_solutions():
    lv = O.sfc_sort(I.uniform_leaves(6, 2))
    mesh = _mesh(lv)
    par = O.params(M, O.SPHERE)
    qa = I.sphere_bump(lv, M, lat=0.3, lon=0.5)
    qb = I.sphere_bump(lv, M, lat=0.3, lon=0.5 + np.pi / 2)
    dt = 0.3 * (np.pi / 2) / (M * 4)
    for _ in range(8):
        qa, _ = O.advance(mesh, par, qa, dt)
        qb, _ = O.advance(mesh, par, qb, dt)
    R = np.array([[0.0, -1, 0], [1, 0, 0], [0, 0, 1]])
    err, scale = 0.0, np.abs(qa[:, 0] - 1).max()
    for p, (q_img, how) in enumerate(_rotate_index(lv)):
        a = qa[p]
        if how == "r4":     # cell (i, j) -> (m+1-j, i)
            a = np.stack([np.rot90(c, -1) for c in a])
        elif how == "r5":   # cell (i, j) -> (j, m+1-i)
            a = np.stack([np.rot90(c, 1) for c in a])
        b = qb[q_img]
        err = max(err, np.abs(a[0] - b[0]).max(),
                  np.abs(np.einsum("kl,lij->kij", R, a[1:]) - b[1:]).max())
    assert err <= 1e-12 * max(scale, 1e-3), err


def _ld_point(tree, xi, eta):
    """Sphere point of reference coordinates (xi, eta) of a tree in x87
    extended precision (the gnomonic equiangular map, written out here)."""
    c, u, v = (np.array(w, dtype=np.longdouble) for w in I.CUBE_FACES[tree])
    q = np.longdouble(np.pi) / 4
    a = np.tan((np.longdouble(xi) - np.longdouble(0.5)) * 2 * q)
    b = np.tan((np.longdouble(eta) - np.longdouble(0.5)) * 2 * q)
    p = c + a * u + b * v
    return p / np.sqrt(np.sum(p * p))


def _ld_quad_area(A, B, C, D):
    """Area of the spherical quadrilateral ABCD as two triangles, each by
    Van Oosterom and Strackee with the triple product over its short sides,
    in extended precision."""
    def tri(a, b, c):
        w = np.cross(b - a, c - a)
        return 2 * np.arctan2(np.sum(a * w),
                              1 + np.sum(a * b) + np.sum(b * c) + np.sum(c * a))
    return tri(A, B, C) + tri(A, C, D)


@pytest.mark.parametrize("level,m", [(6, 32), (9, 8)])
def test_small_cell_areas_to_relative_rounding(level, m):
    """Capacities of small cells (angular size about 8e-4 and 4e-4) times
    the computational cell area equal the cells' areas computed
    independently in extended precision to 2e-12 relative: the oracle keeps
    relative accuracy on small cells (rounding of the corner points gives
    about eps / h; a triple product formed without the short sides would
    give eps / h^2, 2e-11 measured here)."""
    trees = I.cubed_sphere()
    rng = np.random.default_rng(level)
    n = 1 << level
    picks = [(int(t), int(x), int(y)) for t, x, y in
             zip(rng.integers(0, 6, 4), rng.integers(0, n, 4), rng.integers(0, n, 4))]
    leaves = O.sfc_sort(np.array([(t, level, x, y) for t, x, y in picks], dtype=I.LEAF_DTYPE))
    # a single-leaf-per-tree forest is not a tiling: use one leaf at a time
    # inside a forest made of that leaf's tree refined along its path
    worst = 0.0
    for t, x, y in picks:
        lv = [(t2, 0, 0, 0) for t2 in range(6) if t2 != t]
        # the path from the root to (level, x, y): siblings at every level
        for l in range(1, level + 1):
            px, py = x >> (level - l), y >> (level - l)
            for c in range(4):
                cx, cy = 2 * (px >> 1) + (c & 1), 2 * (py >> 1) + (c >> 1)
                if (cx, cy) != (px, py) or l == level:
                    lv.append((t, l, cx, cy))
        raw = np.array(lv, dtype=I.LEAF_DTYPE)
        bal = O.balance(trees, raw)
        mesh = O.Mesh(trees, bal, m, sphere=True)
        p = int(np.nonzero((bal["tree"] == t) & (bal["level"] == level) &
                           (bal["ix"] == x) & (bal["iy"] == y))[0][0])
        h = 1.0 / (m << level)
        for (i, j) in ((1, 1), (m // 2, m // 3 + 1), (m, m)):
            xi0 = (x * m + i - 1) * h
            eta0 = (y * m + j - 1) * h
            A = _ld_point(t, xi0, eta0)
            B = _ld_point(t, xi0 + h, eta0)
            C = _ld_point(t, xi0 + h, eta0 + h)
            D = _ld_point(t, xi0, eta0 + h)
            want = _ld_quad_area(A, B, C, D)
            got = O.sphere_kappa(mesh, p, i, j) * h * h
            worst = max(worst, float(abs(np.longdouble(got) / want - 1)))
    assert worst <= 2e-12, worst
