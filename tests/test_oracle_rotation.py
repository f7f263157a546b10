"""Pins of the oracle's advection by a rigid rotation of the cubed sphere
(ROTATION: the colour equation with u = Omega w x r, the flow of the
paper's Sec. 5 sphere example), against facts outside the oracle:

- the flux of an edge is the integral of u.n along the great-circle arc
  between the edge's corners (Gauss-Legendre quadrature of the closed-form
  velocity here, with the corners mapped here from the gnomonic map and the
  normal turned towards the higher-index cell): fixes the sign, the
  corners, Omega = 2 pi / T, the axis normalisation and the division by
  the computational cell size;
- the discrete field is exactly divergence free (the fluxes of a cell's
  four edges telescope) on every cell of the patch frames but the corner
  cells at a cube vertex, whose region no tree covers (there the own face
  mapping extended meets the canonical corners, and those cells only
  receive transverse parts);
- any function of w.r is a steady solution (the flow runs along circles
  about the axis), so the scheme changes such a state only by its
  truncation error, which falls under refinement; a wrong sign or axis
  would move it at O(1);
- after one full turn the state returns to the initial one up to the
  truncation error, which falls under refinement;
- a uniform state is kept exactly;
- turning the cube by 90 degrees about z (the rotation axis) maps the
  computation onto itself: the results of a state and of its turned copy
  agree cell by cell.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I

PI = np.pi
M = 8
AXIS = (0.3, -0.4, 0.866)     # tilted: the flow crosses cube edges and vertices


def _mesh(lv, m=M):
    return O.Mesh(I.cubed_sphere(), lv, m, sphere=True)


def _arc_flux(a, b, omega, w, nsign):
    """integral of (omega w x r).n ds along the great-circle arc a -> b,
    n = nsign (a x b)/|a x b| (constant on the arc)"""
    n = np.cross(a, b)
    n = nsign * n / np.linalg.norm(n)
    th = np.arccos(np.clip(np.dot(a, b), -1, 1))
    x, wq = np.polynomial.legendre.leggauss(8)
    tot = 0.0
    for xk, wk in zip(x, wq):
        s = 0.5 * (xk + 1) * th
        r = (np.sin(th - s) * a + np.sin(s) * b) / np.sin(th)
        tot += 0.5 * wk * th * np.dot(omega * np.cross(w, r), n)
    return tot


@pytest.mark.parametrize("T", [1.0, 3.7])
def test_edge_flux_is_the_arc_integral_of_the_normal_velocity(T):
    trees = I.cubed_sphere()
    lv = O.balance(trees, I.random_leaves(5, 6, 1, 3, 12))
    mesh = _mesh(lv)
    par = O.params(M, O.ROTATION, period=T, axis=AXIS)
    w = np.array(AXIS) / np.linalg.norm(AXIS)
    omega = 2 * PI / T
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(300):
        p = int(rng.integers(len(lv)))
        a = lv[p]
        d = int(rng.integers(2))
        i, j = (int(v) for v in rng.integers(1, M + 1, 2))
        n = 1 << int(a["level"])
        h = 1.0 / (n * M)
        xi0, eta0 = (int(a["ix"]) * M + i - 1) * h, (int(a["iy"]) * M + j - 1) * h
        # the low-side edge of cell (i, j) and the centres on its two sides
        A = I.sphere_point(int(a["tree"]), xi0, eta0)
        B = I.sphere_point(int(a["tree"]), xi0 + (d == 1) * h, eta0 + (d == 0) * h)
        cr = I.sphere_point(int(a["tree"]), xi0 + h / 2, eta0 + h / 2)
        cl = I.sphere_point(int(a["tree"]), xi0 + h / 2 - (d == 0) * h,
                            eta0 + h / 2 - (d == 1) * h)
        nab = np.cross(A, B)
        nsign = 1.0 if np.dot(nab, cr - cl) > 0 else -1.0
        want = _arc_flux(A, B, omega, w, nsign) / h
        got = O.rotation_edge(mesh, par, p, d, i, j)
        worst = max(worst, abs(got - want) / omega)
    assert worst <= 1e-11


def test_discrete_field_is_divergence_free():
    trees = I.cubed_sphere()
    lv = O.balance(trees, I.random_leaves(3, 6, 1, 3, 10))
    mesh = _mesh(lv)
    par = O.params(M, O.ROTATION, period=1.0, axis=AXIS)
    for p in range(len(lv)):
        a = lv[p]
        n = 1 << int(a["level"])
        for j in range(0, M + 2):
            for i in range(0, M + 2):
                if i in (0, M + 1) and j in (0, M + 1):
                    # frame corner: skipped where the patch corner is a cube vertex
                    cx = int(a["ix"]) + (i > 0) in (0, n)
                    cy = int(a["iy"]) + (j > 0) in (0, n)
                    if cx and cy:
                        continue
                div = (O.rotation_edge(mesh, par, p, 0, i + 1, j) - O.rotation_edge(mesh, par, p, 0, i, j)
                       + O.rotation_edge(mesh, par, p, 1, i, j + 1) - O.rotation_edge(mesh, par, p, 1, i, j))
                assert abs(div) <= 1e-12 * 2 * PI * M * (1 << int(lv[p]["level"]))


def _run(level, q_fn, t_end, T, m=M, cfl=0.4):
    lv = O.sfc_sort(I.uniform_leaves(6, level))
    mesh = _mesh(lv, m)
    q = I.sphere_scalar(lv, m, q_fn)
    par = O.params(m, O.ROTATION, period=T, axis=AXIS)
    # the largest speed is Omega times the largest edge-length factor,
    # about 1.2 / (level-0 patch size) on the equiangular cube
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


def test_functions_of_the_axis_coordinate_are_steady():
    errs = []
    for level in (0, 1, 2):
        q0, q = _run(level, lambda r: np.cos(3 * _wr(r)), 0.25, 1.0)
        errs.append(np.mean(np.abs(q - q0)))
    assert errs[-1] < 3e-3
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3


def test_one_turn_returns_the_state():
    c = np.array([0.6, 0.0, 0.8])
    blob = lambda r: np.exp(-4.0 * np.sum((r - c[None, :, None, None]) ** 2, axis=1))
    errs = []
    for level in (0, 1, 2):
        q0, q = _run(level, blob, 1.0, 1.0)
        errs.append(np.mean(np.abs(q - q0)) / np.mean(np.abs(q0)))
    assert errs[-1] < 0.02
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_uniform_state_is_kept_exactly():
    q0, q = _run(1, lambda r: 0.0 * r[:, 0] + 0.625, 0.1, 1.0)
    assert np.array_equal(q, q0)


def _rotate_index(lv):
    """image of every leaf of a uniform forest under the turn by 90 degrees
    about z: (leaf index, cell permutation)"""
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


def test_turning_the_cube_maps_solutions():
    lv = O.sfc_sort(I.uniform_leaves(6, 1))
    mesh = _mesh(lv)
    par = O.params(M, O.ROTATION, period=1.0, axis=(0.0, 0.0, 1.0))
    f = lambda r: np.exp(-3.0 * ((r[:, 0] - 0.5) ** 2 + (r[:, 1] - 0.2) ** 2 + (r[:, 2] - 0.6) ** 2))
    qa = I.sphere_scalar(lv, M, f)
    # the same state turned by 90 degrees about z: f(R^T r)
    qb = I.sphere_scalar(lv, M, lambda r: f(np.stack([r[:, 1], -r[:, 0], r[:, 2]], axis=1)))
    dt = 0.3 * (PI / 2) / (M * 2) / (2 * PI)
    for _ in range(6):
        qa, _ = O.advance(mesh, par, qa, dt)
        qb, _ = O.advance(mesh, par, qb, dt)
    err = 0.0
    for p, (pb, how) in enumerate(_rotate_index(lv)):
        a = qa[p, 0]
        b = qb[pb, 0]
        if how == "r4":     # cell (i, j) of the image is (m-1-j, i) of b's patch
            b = np.rot90(b, 1)
        elif how == "r5":
            b = np.rot90(b, -1)
        err = max(err, np.max(np.abs(a - b)))
    assert err <= 1e-13


def test_transverse_parts_use_the_receiving_cells_edges():
    """One step from a single unit cell (no limiter, transverse mode 1: the
    diagonal neighbour downstream is reached only by the transverse parts).
    It takes 1/2 dt^2 / (kappa_d dx^2) times the sum over the two paths of
    (flux of the normal edge) x (flux of the receiving cell's edge that faces
    the diagonal cell) / kappa of the receiving cell; the fluxes are the arc
    integrals formed here, the capacities the pinned geometry's."""
    m = 16
    lv = O.sfc_sort(I.uniform_leaves(6, 0))
    mesh = _mesh(lv, m)
    T = 1.0
    par = O.params(m, O.ROTATION, limiter=0, transverse=1, period=T, axis=AXIS)
    w = np.array(AXIS) / np.linalg.norm(AXIS)
    omega = 2 * PI / T
    h = 1.0 / m
    p = 0
    tree = int(lv[p]["tree"])

    def flux(d, i, j):      # low-side d-edge of cell (i, j), over h
        xi0, eta0 = (i - 1) * h, (j - 1) * h
        A = I.sphere_point(tree, xi0, eta0)
        B = I.sphere_point(tree, xi0 + (d == 1) * h, eta0 + (d == 0) * h)
        cr = I.sphere_point(tree, xi0 + h / 2, eta0 + h / 2)
        cl = I.sphere_point(tree, xi0 + h / 2 - (d == 0) * h, eta0 + h / 2 - (d == 1) * h)
        nsign = 1.0 if np.dot(np.cross(A, B), cr - cl) > 0 else -1.0
        return _arc_flux(A, B, omega, w, nsign) / h

    # a cell whose flow runs towards higher i and j on all four paths' edges
    cell = None
    for j in range(3, m - 2):
        for i in range(3, m - 2):
            if min(flux(0, i + 1, j), flux(1, i + 1, j + 1),
                   flux(1, i, j + 1), flux(0, i + 1, j + 1)) > 0.05 * omega:
                cell = (i, j)
                break
        if cell:
            break
    assert cell is not None
    i, j = cell
    q = np.zeros((len(lv), 1, m, m))
    q[p, 0, j - 1, i - 1] = 1.0
    dt = 0.2 * h / omega
    qn, _ = O.advance(mesh, par, q, dt)
    k = lambda a, b: O.sphere_kappa(mesh, p, a, b)
    want = 0.5 * dt * dt / (k(i + 1, j + 1) * h * h) * (
        flux(0, i + 1, j) * flux(1, i + 1, j + 1) / k(i + 1, j)
        + flux(1, i, j + 1) * flux(0, i + 1, j + 1) / k(i, j + 1))
    got = qn[p, 0, j, i]
    assert abs(got - want) <= 1e-10 * abs(want), (got, want)
