"""Pins of the oracle's ghost fill (copy / average / limited interpolation by
the location rule): exactness on linear data, mean preservation of the
interpolation, constants, no nested interpolation, equality with a uniform
grid's periodic frame."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I

M = 8


def _ghost_mask(m):
    g = np.ones((m + 4, m + 4), bool)
    g[2:m + 2, 2:m + 2] = False
    for a in (0, m + 3):
        for b in (0, m + 3):
            g[a, b] = False      # outermost corners are never read
    return g


def _frame_centres(leaves, m, pl):
    return I.cell_centres(leaves, m, pl, ghosts=2)


@pytest.mark.parametrize("domain", ["walled", "brick_oriented"])
@pytest.mark.parametrize("seed", [3, 4, 5])
def test_linear_data_exact(domain, seed):
    if domain == "walled":
        trees, pl = I.walled_square()
        nt, ext = 1, (1.0, 1.0)
    else:
        trees, pl = I.brick(2, 2, orient_codes=[0, 1, 6, 3])
        nt, ext = 4, (2.0, 2.0)
    lv = O.balance(trees, I.random_leaves(seed, nt, 2, 5, 30))
    mesh = O.Mesh(trees, lv, M)
    par = O.params(M)
    fn = lambda x, y: 0.3 + 1.7 * x - 0.9 * y
    q = I.state_from(lv, M, fn, pl)
    f = O.framed(q, M)
    depth = O.ghost_fill(mesh, par, f)
    assert depth <= 1
    gx, gy = _frame_centres(lv, M, pl)
    expect = fn(gx, gy)
    h = np.ldexp(1.0, -lv["level"].astype(int))[:, None, None] / M
    dist = np.minimum.reduce([gx, gy, ext[0] - gx, ext[1] - gy])
    use = _ghost_mask(M)[None] & (dist > 4 * h)
    got = f[:, 0]
    err = np.abs(got - expect)[use]
    assert use.sum() > 100
    assert err.max() <= 1e-14 * np.abs(expect[use]).max()


@pytest.mark.parametrize("seed", [6, 7])
def test_interpolated_means_equal_coarse_cell(seed):
    trees, pl = I.periodic_square()
    lv = O.balance(trees, I.random_leaves(seed, 1, 2, 5, 25))
    mesh = O.Mesh(trees, lv, M)
    par = O.params(M)
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((len(lv), 1, M, M))
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    n_checked = 0
    for p, a in enumerate(lv):
        size = O.SIDE >> int(a["level"])
        cs = size // M
        x0, y0 = int(a["ix"]) * size, int(a["iy"]) * size
        # 2x2 ghost blocks along each face: centre of the block = centre of
        # one coarse cell if the neighbour there is coarser
        for face in range(4):
            for k in range(M // 2 + 1):
                t0 = 2 * k - 1          # block covers cells t0, t0+1
                if face < 2:
                    gi = (-1, 0) if face == 0 else (M + 1, M + 2)
                    gj = (t0, t0 + 1)
                else:
                    gj = (-1, 0) if face == 2 else (M + 1, M + 2)
                    gi = (t0, t0 + 1)
                if min(gi + gj) < -1 or max(gi + gj) > M + 2:
                    continue
                if (gi[0] < 1 or gi[0] > M) and (gj[0] < 1 or gj[0] > M):
                    continue        # corner block holds an unread cell
                cx = x0 + (gi[0] - 1) * cs + cs   # block centre
                cy = y0 + (gj[0] - 1) * cs + cs
                L = mesh.locate(int(a["tree"]), cx, cy)
                if L < 0 or lv["level"][L] != a["level"] - 1:
                    continue
                b = lv[L]
                sb = O.SIDE >> int(b["level"])
                csb = sb // M
                # coordinates wrap on the periodic square
                ux = (cx % O.SIDE) - int(b["ix"]) * sb
                uy = (cy % O.SIDE) - int(b["iy"]) * sb
                ic, jc = ux // csb, uy // csb
                qc = q[L, 0, jc, ic]
                blk = [f[p, 0, j + 1, i + 1] for i in gi for j in gj]
                assert abs(np.mean(blk) - qc) <= 1e-15 * (1 + abs(qc)) * 4
                n_checked += 1
    assert n_checked > 20


@pytest.mark.parametrize("domain", ["walled", "periodic", "sphere"])
def test_constant_preserved_bitwise(domain):
    if domain == "walled":
        trees, _ = I.walled_square()
        nt, par = 1, O.params(M, O.SHALLOW)
    elif domain == "periodic":
        trees, _ = I.periodic_square()
        nt, par = 1, O.params(M)
    else:
        trees = I.cubed_sphere()
        nt, par = 6, O.params(M)
    lv = O.balance(trees, I.random_leaves(11, nt, 1, 5, 40))
    mesh = O.Mesh(trees, lv, M)
    c = np.array([1.234567, 0.0, 0.0])[:par.meqn]
    q = np.broadcast_to(c[None, :, None, None], (len(lv), par.meqn, M, M)).copy()
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    g = _ghost_mask(M)
    for k in range(par.meqn):
        vals = f[:, k][np.broadcast_to(g, (len(lv),) + g.shape)]
        assert np.all(vals == c[k])


def test_uniform_forest_frame_is_periodic_wrap():
    level = 2
    trees, _ = I.periodic_square()
    lv = O.sfc_sort(I.uniform_leaves(1, level))
    mesh = O.Mesh(trees, lv, M)
    par = O.params(M)
    n = M << level
    rng = np.random.default_rng(0)
    big = rng.standard_normal((n, n))        # [y, x]
    q = np.zeros((len(lv), 1, M, M))
    for p, a in enumerate(lv):
        q[p, 0] = big[a["iy"] * M:(a["iy"] + 1) * M, a["ix"] * M:(a["ix"] + 1) * M]
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    g = _ghost_mask(M)
    for p, a in enumerate(lv):
        ys = (np.arange(-2, M + 2) + a["iy"] * M) % n
        xs = (np.arange(-2, M + 2) + a["ix"] * M) % n
        want = big[np.ix_(ys, xs)]
        assert np.array_equal(f[p, 0][g], want[g])


def test_reflecting_wall_frame():
    trees, _ = I.walled_square()
    lv = O.sfc_sort(I.uniform_leaves(1, 1))
    mesh = O.Mesh(trees, lv, M)
    par = O.params(M, O.SHALLOW)
    rng = np.random.default_rng(1)
    q = rng.uniform(1, 2, (len(lv), 3, M, M))
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    p = 0                                   # lower-left patch: walls 0 and 2
    for k, s in ((0, 1), (1, -1), (2, 1)):
        # xi-low wall: Q(1-k) = Q(k), hu negated
        assert np.array_equal(f[p, k, 2:M + 2, 1], s * f[p, k, 2:M + 2, 2])
        assert np.array_equal(f[p, k, 2:M + 2, 0], s * f[p, k, 2:M + 2, 3])
    for k, s in ((0, 1), (1, 1), (2, -1)):
        assert np.array_equal(f[p, k, 1, 2:M + 2], s * f[p, k, 2, 2:M + 2])
    # domain corner: doubly reflected
    assert f[p, 1, 1, 1] == -f[p, 1, 2, 2] and f[p, 2, 1, 1] == -f[p, 2, 2, 2]
