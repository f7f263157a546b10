"""GPU tests of the CFL rule's reject-and-redo (an attempt whose largest
Courant number exceeds cfl_max leaves the state unchanged and the next one
uses dt * cfl_desired / nu), of per-forest status words in batches, and of
the old-to-new patch map of a regrid, against the CPU oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import fcx
from paper_1308_1472_amd import inputs as I
from tests.gpu_drive import oracle_attempt, oracle_params, say, smooth_sw_state

pytestmark = pytest.mark.gpu


def _maxrel(a, b):
    top = max(np.max(np.abs(b)), 1e-300)
    return max(np.max(np.abs(a[:, k] - b[:, k])) / max(np.max(np.abs(b[:, k])), 1e-3 * top)
               for k in range(b.shape[1]))


def _dam_break_forest(m=8):
    trees, pl = I.walled_square()
    lv = fcx.balance(trees, I.refine_near(1, 2, 4, [(0.5, 0.5)], pl, radius=1.2))
    q0 = I.state_from(lv, m, lambda x, y: I.dam_break(x, y), pl)
    return trees, pl, lv, q0


def _nu_of(mesh, par, q, dt):
    return O.advance(mesh, par, q, dt)[1]


@pytest.mark.parametrize("precision", [64, 32])
def test_advance_rejects_and_redoes(precision):
    """fcx_advance with dt 1.4 times the largest stable one: the attempt is
    rejected (q_new bit-equal to q, dt reduced by cfl_desired / nu, status
    bit 3), the next attempt is accepted and equals the oracle's step with
    the reduced dt; counters follow.  With the rule off the first step is
    kept and flagged with bit 0."""
    import torch
    say(f"[redo] advance precision={precision}")
    m = 8
    trees, pl, lv, q0 = _dam_break_forest(m)
    mesh = O.Mesh(trees, lv, m)
    par = O.params(m, O.SHALLOW)
    probe = 1e-4
    dt0 = 1.4 * probe / _nu_of(mesh, par, q0, probe)
    q1, nu0, dt1, ok = oracle_attempt(mesh, par, q0, dt0)
    assert not ok and nu0 > 1.3
    q2, nu1, dt2, ok2 = oracle_attempt(mesh, par, q1, dt1)
    assert ok2 and abs(nu1 - 0.9) < 1e-9
    dtype = torch.float64 if precision == 64 else torch.float32
    for redo in (1, 0):
        ctx = fcx.Context(fcx.config(m, precision, fcx.FCX_SHALLOW, redo=redo), trees)
        ctx.upload_forest(lv)
        q = torch.from_numpy(q0.ravel().copy()).to(dtype).cuda()
        qn = torch.full_like(q, float("nan"))
        dt = torch.full((1,), dt0, dtype=torch.float64, device="cuda")
        nu = torch.zeros_like(dt)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        ctx.advance(q, qn, dt, nu, st)
        torch.cuda.synchronize()
        tol = 1e-13 if precision == 64 else 1e-5
        assert abs(dt.item() / dt1 - 1) <= tol
        if redo:
            assert torch.equal(qn, q)
            assert st.item() == 8
            assert ctx.step_stats() == (0, 1, 0)
            ctx.advance(qn, q, dt, nu, st)
            P = len(lv)
            got = q.double().cpu().numpy().reshape(P, 3, m, m)
            if precision == 64:
                assert _maxrel(got, q2) <= 1e-12
                assert abs(dt.item() / dt2 - 1) <= 1e-12
            else:
                assert np.abs(got - q2).sum() / np.abs(q2).sum() <= 1e-5
            assert st.item() == 8
            assert ctx.step_stats() == (1, 1, P * m * m)
        else:
            assert not torch.equal(qn, q)
            assert st.item() == 1
            assert ctx.step_stats() == (1, 0, len(lv) * m * m)


@pytest.mark.parametrize("fused", [True, False])
def test_run_loop_redo_matches_oracle(fused):
    """fcx_run from a dt 1.3 times the stable one, a regrid every 3
    attempts, levels 2-4: forest, dt, state and counters equal the oracle's
    attempts under the same rule (plain steps: the redo copy is taken by
    the separate next-dt launch)."""
    import torch
    say(f"[redo] run loop fused={fused}")
    m, lmin, lmax, every, thr, steps = 8, 2, 4, 3, 0.3, 9
    trees, pl, lv0, q0 = _dam_break_forest(m)
    cfg = fcx.config(m, 64, fcx.FCX_SHALLOW)
    par = oracle_params(cfg)
    mesh = O.Mesh(trees, lv0, m)
    dt0 = 1.3 * 1e-4 / _nu_of(mesh, par, q0, 1e-4)
    # the oracle's attempts
    lv, q, dt = lv0, q0.copy(), dt0
    oks, cells = [], 0
    for n in range(steps):
        if n > 0 and n % every == 0:
            f = O.framed(q, m)
            O.ghost_fill(mesh, par, f)
            tg = O.tags(mesh, par, f, 1, thr, lmin, lmax)
            lv = O.regrid(mesh, tg, lmin, lmax)
            mesh2 = O.Mesh(trees, lv, m)
            q = O.interior(O.transfer(mesh, mesh2, par, f), m)
            mesh = mesh2
        q, nu, dt, ok = oracle_attempt(mesh, par, q, dt)
        oks.append(ok)
        cells += ok * len(lv) * m * m
    assert oks.count(False) >= 1
    ctx = fcx.Context(cfg, trees)
    ctx.upload_forest(lv0)
    dtt = torch.full((1,), dt0, dtype=torch.float64, device="cuda")
    nut = torch.zeros_like(dtt)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pmax = 1 << (2 * lmax)
    bufs = [torch.empty(pmax * 3 * m * m, dtype=torch.float64, device="cuda")
            for _ in range(2)]
    bufs[0][:q0.size].copy_(torch.from_numpy(q0.ravel()))
    ghost = torch.empty(pmax * 3 * (8 * m + 16), dtype=torch.float64, device="cuda")
    which, got_cells = ctx.run(bufs[0], bufs[1], ghost, steps, 0, every, 1, thr, lmin,
                               lmax, dtt, nut, st, fused=fused)
    assert np.array_equal(ctx.leaves(), lv)
    got = bufs[which][:ctx.state_elems()].cpu().numpy().reshape(q.shape)
    assert _maxrel(got, q) <= 1e-12
    assert abs(dtt.item() / dt - 1) <= 1e-12
    assert got_cells == cells
    assert ctx.step_stats() == (oks.count(True), oks.count(False), cells)
    assert st.item() == 8


def _batch_of_three(precision):
    import torch
    specs = [(fcx.FCX_ADVECTION, 8, "periodic", 1), (fcx.FCX_SHALLOW, 16, "walled", 2),
             (fcx.FCX_SHALLOW, 8, "walled", 4)]
    ctxs, states, meshes, pars = [], [], [], []
    for phys, m, dom, seed in specs:
        trees, pl = I.periodic_square() if dom == "periodic" else I.walled_square()
        lv = fcx.balance(trees, I.random_leaves(seed, 1, 2, 4, 10))
        cfg = fcx.config(m, precision, phys, ax=0.7, ay=-0.3)
        ctx = fcx.Context(cfg, trees)
        ctx.upload_forest(lv)
        ctxs.append(ctx)
        if phys == fcx.FCX_SHALLOW:
            states.append(smooth_sw_state(lv, m, pl, seed))
        else:
            states.append(I.state_from(lv, m, lambda x, y: I.gaussian(x, y, 0.4, 0.5, 0.02),
                                       pl))
        meshes.append(O.Mesh(trees, lv, m))
        pars.append(oracle_params(fcx.config(m, 64, phys, ax=0.7, ay=-0.3)))
    batch = fcx.Batch(ctxs)
    dtype = torch.float64 if precision == 64 else torch.float32
    qb = torch.empty(batch.state_elems(), dtype=dtype, device="cuda")
    for f, q in enumerate(states):
        o = batch.state_offset(f)
        qb[o:o + q.size].copy_(torch.from_numpy(q.ravel()))
    return batch, ctxs, states, meshes, pars, qb


def test_batch_rejects_one_forest():
    """A batch step where only forest 1's dt is too large: forest 1 keeps
    its state bit for bit, its dt shrinks by cfl_desired / nu and only its
    status carries bit 3; the other forests advance as the oracle does;
    the per-forest counters say so; the redo attempt then matches the
    oracle's step with the reduced dt."""
    import torch
    say("[redo] batch")
    batch, ctxs, states, meshes, pars, q0 = _batch_of_three(64)
    dts = []
    for f in range(3):
        nu1 = _nu_of(meshes[f], pars[f], states[f], 1e-4)
        dts.append((1.5 if f == 1 else 0.5) * 1e-4 / nu1)
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    nu = torch.zeros(3, dtype=torch.float64, device="cuda")
    st = torch.zeros(3, dtype=torch.int32, device="cuda")
    qn = torch.empty_like(q0)
    batch.step(q0, qn, dt, nu, st)
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [0, 8, 0]
    for f, c in enumerate(ctxs):
        o = batch.state_offset(f)
        got = qn[o:o + c.state_elems()].cpu().numpy().reshape(states[f].shape)
        want, nu_o, dt_o, ok = oracle_attempt(meshes[f], pars[f], states[f], dts[f])
        assert ok == (f != 1)
        if f == 1:
            assert np.array_equal(got, states[f])
        else:
            assert _maxrel(got, want) <= 1e-12
        assert abs(dt[f].item() / dt_o - 1) <= 1e-13
    stats = batch.step_stats()
    assert stats[:, :2].tolist() == [[1, 0], [0, 1], [1, 0]]
    assert stats[1, 2] == 0 and stats[0, 2] == ctxs[0].num_patches() * 64
    # the redo of forest 1
    q2 = torch.empty_like(q0)
    dt_before = dt.cpu().numpy().copy()
    batch.step(qn, q2, dt, nu, st)
    o = batch.state_offset(1)
    got = q2[o:o + ctxs[1].state_elems()].cpu().numpy().reshape(states[1].shape)
    want, nu_o, _, ok = oracle_attempt(meshes[1], pars[1], states[1], dt_before[1])
    assert ok and abs(nu_o - 0.9) < 1e-9
    assert _maxrel(got, want) <= 1e-12
    assert batch.step_stats()[1, :2].tolist() == [1, 1]


def test_batch_negative_depth_is_reported_by_its_forest():
    """A non-positive depth in forest 2 of a batch raises bit 1 of forest 2's
    status only (each forest has its own error word)."""
    import torch
    say("[batch] per-forest error word")
    batch, ctxs, states, meshes, pars, q0 = _batch_of_three(64)
    o = batch.state_offset(2)
    m = ctxs[2].cfg.m
    q0[o + 5 * m + 3] = -1.0                  # patch 0, h at cell (4, 6)
    dt = torch.full((3,), 1e-4, dtype=torch.float64, device="cuda")
    nu = torch.zeros(3, dtype=torch.float64, device="cuda")
    st = torch.zeros(3, dtype=torch.int32, device="cuda")
    qn = torch.empty_like(q0)
    batch.step(q0, qn, dt, nu, st)
    s = st.cpu().tolist()
    assert s[0] == 0 and s[1] == 0 and s[2] & 2


def _old_to_new_from_leaves(old, new):
    """The map from the two leaf lists alone: kept leaves by identity, a
    refined leaf by the index of its first child, a merged leaf -1."""
    idx = {tuple(int(v) for v in a): i for i, a in enumerate(new)}
    out = []
    for a in old:
        t, lvl, x, y = (int(v) for v in a)
        if (t, lvl, x, y) in idx:
            out.append(idx[(t, lvl, x, y)])
        elif (t, lvl + 1, 2 * x, 2 * y) in idx:
            k = idx[(t, lvl + 1, 2 * x, 2 * y)]
            assert all(idx.get((t, lvl + 1, 2 * x + (c & 1), 2 * y + (c >> 1))) == k + c
                       for c in range(4))
            out.append(-2 - k)
        else:
            assert (t, lvl - 1, x >> 1, y >> 1) in idx
            out.append(-1)
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("seed", [2, 9])
def test_regrid_old_to_new_map(seed):
    """fcx_regrid_apply's old_to_new equals the map derived from the
    oracle's old and new leaves (kept, refined into k..k+3, merged), over
    three regrids with random tags; fcx_regrid gives the same for its
    criterion tags."""
    import torch
    say(f"[regrid] old_to_new seed={seed}")
    trees, pl = I.walled_square()
    lv = O.balance(trees, I.random_leaves(seed, 1, 2, 5, 30))
    cfg = fcx.config(8, 64, fcx.FCX_SHALLOW)
    ctx = fcx.Context(cfg, trees)
    ctx.upload_forest(lv)
    rng = np.random.default_rng(seed)
    seen = {"kept": 0, "refined": 0, "merged": 0}
    for r in range(3):
        old = ctx.leaves()
        tg = rng.integers(-1, 2, len(old)).astype(np.int8)
        n, o2n = ctx.regrid_apply(tg, 1, 6, old_to_new=True)
        new = O.regrid(O.Mesh(trees, old, 8), tg, 1, 6)
        assert n == len(new) and np.array_equal(ctx.leaves(), new)
        want = _old_to_new_from_leaves(old, new)
        assert np.array_equal(o2n, want), r
        seen["kept"] += int((o2n >= 0).sum())
        seen["refined"] += int((o2n <= -2).sum())
        seen["merged"] += int((o2n == -1).sum())
    assert min(seen.values()) > 0, seen
    # the one-call regrid on the criterion tags
    old = ctx.leaves()
    q = smooth_sw_state(old, 8, pl, seed)
    qt = torch.from_numpy(q.ravel().copy()).cuda()
    g = torch.empty(ctx.ghost_elems(), dtype=torch.float64, device="cuda")
    n, o2n = ctx.regrid(qt, g, 1, 0.5, 1, 6, old_to_new=True)
    mesh = O.Mesh(trees, old, 8)
    f = O.framed(q, 8)
    O.ghost_fill(mesh, oracle_params(cfg), f)
    new = O.regrid(mesh, O.tags(mesh, oracle_params(cfg), f, 1, 0.5, 1, 6), 1, 6)
    assert np.array_equal(ctx.leaves(), new)
    assert np.array_equal(o2n, _old_to_new_from_leaves(old, new))
