"""Pins of the oracle's prescribed-flow advection (SWIRL: the colour equation
q_t + u q_x + v q_y = 0 with (u, v) = (psi_y, -psi_x) from a stream function;
a stand-in for the unpublished field of the paper's Sec. 5 advection
example), against facts outside the oracle:

- each edge's normal velocity is psi's difference over the edge, so it
  matches the analytic derivative of the stream function at the edge's
  midpoint to second order, and the discrete field is exactly divergence
  free (the four edges of a cell telescope);
- any function of the stream function is a steady solution of the
  equation (the flow runs along psi's contours), so the scheme may change
  such a state only by its truncation error: second order under refinement.
  A velocity with the wrong sign or swapped components crosses the contours
  and makes an O(1) change;
- the flow reverses at half its period: after a whole period the state
  returns to the initial one up to the truncation error (second order);
- a uniform state is kept exactly (every jump is zero);
- one step from a single unit cell reaches its diagonal neighbour only
  through the transverse parts (LeVeque 1997): their value, formed here from
  the closed-form stream function, fixes which edge of the receiving cell
  each part uses (in a smooth field the wrong edge is only a second-order
  change, which the convergence checks above would not see).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I

PI = np.pi


def _u_exact(x, y, t, T):
    return np.sin(PI * x) ** 2 * np.sin(2 * PI * y) * np.cos(PI * t / T)


def _v_exact(x, y, t, T):
    return -np.sin(2 * PI * x) * np.sin(PI * y) ** 2 * np.cos(PI * t / T)


@pytest.mark.parametrize("t", [0.0, 0.3, 0.77])
def test_edge_velocity_is_the_stream_function_derivative(t):
    T = 1.5
    par = O.params(8, O.SWIRL, period=T)
    rng = np.random.default_rng(4)
    errs = []
    for h in (1 / 32, 1 / 64, 1 / 128):
        e = 0.0
        for _ in range(40):
            a, b = rng.uniform(0, 1 - h, 2)
            u = O.swirl_edge(par, 0, a, b, b + h, t)
            v = O.swirl_edge(par, 1, a, b, b + h, t)
            e = max(e, abs(u - _u_exact(a, b + h / 2, t, T)),
                    abs(v - _v_exact(b + h / 2, a, t, T)))
        errs.append(e)
    # second order: the error of a centred difference quotient, at most
    # h^2 / 24 max |psi'''| (|psi'''| <= 4 pi^2 here)
    for e, h in zip(errs, (1 / 32, 1 / 64, 1 / 128)):
        assert e <= h * h / 24 * 4 * PI * PI * 1.01
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_stream_function_values():
    par = O.params(8, O.SWIRL, period=2.0)
    for x, y, t in [(0.5, 0.5, 0.0), (0.25, 0.75, 0.5), (0.1, 0.9, 1.3)]:
        want = np.sin(PI * x) ** 2 * np.sin(PI * y) ** 2 * np.cos(PI * t / 2.0) / PI
        assert abs(O.swirl_psi(par, x, y, t) - want) <= 1e-15
    # zero on the square's boundary
    for s in np.linspace(0, 1, 7):
        assert abs(O.swirl_psi(par, 0.0, s, 0.1)) <= 1e-30
        assert abs(O.swirl_psi(par, s, 1.0, 0.1)) <= 1e-30


def test_discrete_field_is_divergence_free():
    par = O.params(8, O.SWIRL, period=1.0)
    rng = np.random.default_rng(5)
    for _ in range(200):
        h = 2.0 ** -rng.integers(3, 9)
        x, y = rng.uniform(0, 1 - h, 2)
        t = rng.uniform(0, 2)
        div = (O.swirl_edge(par, 0, x + h, y, y + h, t) - O.swirl_edge(par, 0, x, y, y + h, t)
               + O.swirl_edge(par, 1, y + h, x, x + h, t) - O.swirl_edge(par, 1, y, x, x + h, t))
        assert abs(div) <= 1e-13


def _run(level, m, q_fn, t_end, T, cfl=0.45):
    trees, pl = I.walled_square()
    lv = O.sfc_sort(I.uniform_leaves(1, level))
    mesh = O.Mesh(trees, lv, m)
    q = I.state_from(lv, m, q_fn, pl)
    h = 1.0 / (m << level)
    nsteps = int(np.ceil(t_end / (cfl * h)))
    dt = t_end / nsteps
    par = O.params(m, O.SWIRL, period=T)
    q0 = q.copy()
    t = 0.0
    for _ in range(nsteps):
        par.time = t
        q, nu = O.advance(mesh, par, q, dt)
        assert nu <= 1.0
        t += dt
    return q0, q


def test_functions_of_psi_are_steady_to_second_order():
    psi_s = lambda x, y: np.sin(PI * x) ** 2 * np.sin(PI * y) ** 2
    errs = []
    for level in (2, 3, 4):
        q0, q = _run(level, 8, psi_s, 0.25, 1.0e9)
        errs.append(np.mean(np.abs(q - q0)))
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_the_flow_returns_the_state_after_one_period():
    blob = lambda x, y: np.exp(-((x - 0.5) ** 2 + (y - 0.7) ** 2) / 0.02)
    errs = []
    for level in (2, 3, 4):
        q0, q = _run(level, 8, blob, 1.0, 1.0)
        errs.append(np.mean(np.abs(q - q0)) / np.mean(np.abs(q0)))
    assert errs[-1] < 0.02
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_uniform_state_is_kept_exactly():
    q0, q = _run(2, 8, lambda x, y: 0.0 * x + 0.375, 0.1, 1.0)
    assert np.array_equal(q, q0)


def _psi_np(x, y):
    return np.sin(PI * x) ** 2 * np.sin(PI * y) ** 2 / PI


@pytest.mark.parametrize("where", ["upper_right", "lower_left"])
def test_transverse_terms_use_the_receiving_cells_edges(where):
    """One step from a single unit cell (no limiter, transverse mode 1: the
    diagonal neighbour is reached only by the transverse parts).  The cell
    on the diagonal downstream takes 1/2 (dt/dx)^2 times the sum over the
    two paths of (normal edge velocity) x (transverse velocity of the edge
    of the receiving cell that faces the diagonal cell); the velocities are
    formed here from the closed-form stream function."""
    m, level = 16, 0
    trees, pl = I.walled_square()
    lv = O.sfc_sort(I.uniform_leaves(1, level))
    mesh = O.Mesh(trees, lv, m)
    h = 1.0 / m
    # cell (i, j) (1-based) spans [(i-1)h, ih] x [(j-1)h, jh]
    i, j = (13, 4) if where == "upper_right" else (4, 13)
    q = np.zeros((1, 1, m, m))
    q[0, 0, j - 1, i - 1] = 1.0
    par = O.params(m, O.SWIRL, limiter=0, transverse=1, period=1e12)
    dt = 0.4 * h
    qn, _ = O.advance(mesh, par, q, dt)
    r = dt / h

    def u(xe, yb):      # x-edge at x = xe spanning [yb, yb + h]
        return (_psi_np(xe, yb + h) - _psi_np(xe, yb)) / h

    def v(ye, xb):      # y-edge at y = ye spanning [xb, xb + h]
        return -(_psi_np(xb + h, ye) - _psi_np(xb, ye)) / h

    if where == "upper_right":
        # u > 0 and v > 0 here: the cell (i+1, j+1) receives
        u1, v1 = u(i * h, (j - 1) * h), v(j * h, i * h)            # x path
        v2, u2 = v(j * h, (i - 1) * h), u(i * h, j * h)            # y path
        assert min(u1, v1, v2, u2) > 0
        want = 0.5 * r * r * (u1 * v1 + v2 * u2)
        got = qn[0, 0, j, i]
    else:
        # u < 0 and v < 0: the cell (i-1, j-1) receives
        u1, v1 = u((i - 1) * h, (j - 1) * h), v((j - 1) * h, (i - 2) * h)
        v2, u2 = v((j - 1) * h, (i - 1) * h), u((i - 1) * h, (j - 2) * h)
        assert max(u1, v1, v2, u2) < 0
        want = 0.5 * r * r * (u1 * v1 + v2 * u2)
        got = qn[0, 0, j - 2, i - 2]
    assert abs(got - want) <= 1e-14 * abs(want), (got, want)
