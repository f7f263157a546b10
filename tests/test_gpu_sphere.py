"""GPU parity of the cubed-sphere path against the CPU oracle: geometry
tables, ghost fill with capacity-weighted averages, the rotated-Roe step
with reflux and cube-edge mass sync (FP64 to 1e-12, FP32 to 1e-5 in relative
L1), exact mass conservation and the lake at rest; refinement tags, regrid
with the conservative capacity-weighted transfer, and the run loop with
regrids."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import fcx
from paper_1308_1472_amd import inputs as I
from tests.gpu_drive import Gpu, ghost_to_frame, needed_mask, oracle_params, say

pytestmark = pytest.mark.gpu

M = 8


def _forest(seed, lmin=1, lmax=3, n=12):
    trees = I.cubed_sphere()
    if seed is None:
        return trees, fcx.sfc_sort(I.uniform_leaves(6, lmin))
    return trees, fcx.balance(trees, I.random_leaves(seed, 6, lmin, lmax, n))


def _oracle_geo(mesh, lv):
    """(P, 18, m+4, m+4) geometry tables from the oracle."""
    P = len(lv)
    g = np.zeros((P, 18, M + 4, M + 4))
    for p in range(P):
        for j in range(-1, M + 3):
            for i in range(-1, M + 3):
                g[p, 0, j + 1, i + 1] = O.sphere_kappa(mesh, p, i, j)
                for d in (0, 1):
                    gam, n, t = O.sphere_edge(mesh, p, d, i, j)
                    g[p, 4 + 7 * d, j + 1, i + 1] = gam
                    g[p, 5 + 7 * d:8 + 7 * d, j + 1, i + 1] = n
                    g[p, 8 + 7 * d:11 + 7 * d, j + 1, i + 1] = t
    return g


@pytest.mark.parametrize("seed", [None, 5])
def test_geometry_matches_oracle(seed):
    say(f"[sphere] geometry seed={seed}")
    trees, lv = _forest(seed)
    ctx = fcx.Context(fcx.config(M, 64, fcx.FCX_SPHERE), trees)
    ctx.upload_forest(lv)
    got = ctx.sphere_geometry().cpu().numpy()
    mesh = O.Mesh(trees, lv, M, sphere=True)
    want = _oracle_geo(mesh, lv)
    # frames 1-3 are interleaved centres on the device: compare separately
    FR = (M + 4) ** 2
    cen = got[:, 1:4].reshape(len(lv), 3 * FR).reshape(len(lv), FR, 3)
    for p in range(len(lv)):
        for f in range(FR):
            i, j = f % (M + 4) - 1, f // (M + 4) - 1
            np.testing.assert_allclose(cen[p, f], O.sphere_centre(mesh, p, i, j),
                                       rtol=0, atol=1e-14)
    # kappa and the edge frames: interleaved 7 per cell on the device
    np.testing.assert_allclose(got[:, 0], want[:, 0], rtol=1e-13)
    for d in (0, 1):
        e = got[:, 4 + 7 * d:11 + 7 * d].reshape(len(lv), 7 * FR).reshape(len(lv), FR, 7)
        w = want[:, 4 + 7 * d:11 + 7 * d].reshape(len(lv), 7, FR).transpose(0, 2, 1)
        np.testing.assert_allclose(e, w, rtol=1e-13, atol=1e-14)


def test_ghost_fill_matches_oracle():
    say("[sphere] ghost fill")
    trees, lv = _forest(7, 1, 3, 14)
    cfg = fcx.config(M, 64, fcx.FCX_SPHERE)
    g = Gpu(cfg, trees, lv)
    q = I.sphere_bump(lv, M)
    rng = np.random.default_rng(0)
    q[:, 1:] = 0.05 * rng.normal(size=q[:, 1:].shape)
    g.set_state(q)
    g.fill()
    got = ghost_to_frame(g.ghosts(), g.state(), M)
    f = O.framed(q, M)
    O.ghost_fill(O.Mesh(trees, lv, M, sphere=True), oracle_params(cfg), f)
    mk = needed_mask(M)
    assert np.max(np.abs(got[:, :, mk] - f[:, :, mk])) <= 1e-13


def _run(precision, trees, lv, q0, nsteps, dt):
    cfg = fcx.config(M, precision, fcx.FCX_SPHERE)
    g = Gpu(cfg, trees, lv)
    g.set_state(q0)
    nus = []
    for _ in range(nsteps):
        nu, _ = g.step(dt)
        nus.append(nu)
    return g, cfg, nus


def _oracle_run(trees, lv, q0, nsteps, dt, cfg):
    mesh = O.Mesh(trees, lv, M, sphere=True)
    par = oracle_params(cfg)
    q = q0.copy()
    nus = []
    for _ in range(nsteps):
        q, nu = O.advance(mesh, par, q, dt)
        nus.append(nu)
    return q, nus, mesh, par


def test_fp64_step_matches_oracle():
    say("[sphere] fp64 steps")
    trees, lv = _forest(3, 2, 3, 12)
    q0 = I.sphere_bump(lv, M) + I.sphere_bump(lv, M, lat=np.arcsin(1 / np.sqrt(3)),
                                              lon=np.pi / 4, amp=0.05)
    dt = 0.3 * (np.pi / 2) / (M * 8) / 1.5
    g, cfg, nus = _run(64, trees, lv, q0, 6, dt)
    want, nus_o, mesh, par = _oracle_run(trees, lv, q0, 6, dt, cfg)
    got = g.state()
    for k in range(4):
        scale = max(np.abs(want[:, k]).max(), 1e-3)
        assert np.abs(got[:, k] - want[:, k]).max() <= 1e-12 * scale, k
    np.testing.assert_allclose(nus, nus_o, rtol=1e-12)
    # mass through the library's capacity-weighted sums
    s0 = O.sums(mesh, par, _filled(mesh, par, q0))[0]
    assert abs(g.conservation_sums()[0] / s0 - 1) <= 1e-13


def _filled(mesh, par, q):
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    return f


def test_fp32_step_within_1e5_of_oracle():
    say("[sphere] fp32 steps")
    trees, lv = _forest(4, 2, 3, 10)
    q0 = I.sphere_bump(lv, M)
    dt = 0.3 * (np.pi / 2) / (M * 8) / 1.5
    g, cfg, _ = _run(32, trees, lv, q0, 8, dt)
    want, _, _, _ = _oracle_run(trees, lv, q0, 8, dt, fcx.config(M, 64, fcx.FCX_SPHERE))
    got = g.state()
    rel = np.abs(got[:, 0] - want[:, 0]).sum() / np.abs(want[:, 0]).sum()
    assert rel <= 1e-5, rel


def test_mass_and_lake_at_rest_on_the_gpu():
    say("[sphere] mass + lake")
    trees, lv = _forest(9, 1, 4, 20)
    q0 = I.sphere_bump(lv, M, lat=np.arcsin(1 / np.sqrt(3)), lon=np.pi / 4)
    dt = 0.3 * (np.pi / 2) / (M * 16) / 1.5
    g, cfg, nus = _run(64, trees, lv, q0, 1, dt)
    m0 = g.conservation_sums()[0]
    for _ in range(40):
        g.step(dt)
    assert abs(g.conservation_sums()[0] / m0 - 1) <= 1e-13
    assert max(nus) < 1
    lake = np.zeros_like(q0)
    lake[:, 0] = 1.0
    g2, _, _ = _run(64, trees, lv, lake, 3, dt)
    assert np.array_equal(g2.state(), lake)


def test_unsupported_sphere_calls_fail_loudly():
    import torch
    trees, lv = _forest(None)
    ctx = fcx.Context(fcx.config(M, 64, fcx.FCX_SPHERE), trees)
    ctx.upload_forest(lv)
    q = torch.zeros(ctx.state_elems(), dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(fcx.FcxError):
        ctx.fused_step(q, torch.zeros_like(q), dt, torch.zeros_like(dt))
    with pytest.raises(fcx.FcxError):
        fcx.Batch([ctx])


def _gap_thresholds(values, squared):
    """Two thresholds in the widest relative gaps between distinct criterion
    values (lower and upper half), so that no decision sits within rounding
    of a threshold; values at rounding-noise level (flat water) are left
    out of the search."""
    v = values[np.isfinite(values)]
    v = np.unique(v[v > 1e-8 * v.max()])
    out = []
    for lo, hi in ((0.15, 0.5), (0.5, 0.85)):
        a, b = int(lo * (len(v) - 1)), int(hi * (len(v) - 1))
        r = v[a + 1:b + 1] / v[a:b]
        k = a + int(np.argmax(r))
        t = np.sqrt(v[k] * v[k + 1])
        assert v[k + 1] / v[k] > 1 + 1e-6
        out.append(np.sqrt(t) if squared else t)
    return out


def _sphere_state(lv, seed):
    q = I.sphere_bump(lv, M) + I.sphere_bump(lv, M, lat=0.3, lon=2.0, amp=0.2)
    rng = np.random.default_rng(seed)
    q[:, 1:] = 0.05 * rng.normal(size=q[:, 1:].shape)
    return q


def test_regrid_tags_match_oracle():
    say("[sphere] tags")
    trees, lv = _forest(7, 1, 3, 14)
    cfg = fcx.config(M, 64, fcx.FCX_SPHERE)
    q = _sphere_state(lv, 1)
    g = Gpu(cfg, trees, lv)
    g.set_state(q)
    mesh = O.Mesh(trees, lv, M, sphere=True)
    par = oracle_params(cfg)
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    seen = set()
    for crit in (1, 0):
        ref, parent = O.tag_values(mesh, par, f, crit)
        for thr in _gap_thresholds(np.concatenate([ref, parent]), crit == 1):
            got = g.tags(crit, thr, 1, 4)
            want = O.tags(mesh, par, f, crit, thr, 1, 4)
            assert np.array_equal(got, want), (crit, thr)
            seen.update(np.unique(want).tolist())
    assert seen == {-1, 0, 1}


def test_regrid_transfer_matches_oracle_and_conserves_mass():
    say("[sphere] regrid transfer")
    import torch
    trees, lv = _forest(11, 1, 3, 14)
    cfg = fcx.config(M, 64, fcx.FCX_SPHERE)
    q = _sphere_state(lv, 2)
    rng = np.random.default_rng(4)
    tg = rng.integers(-1, 2, len(lv)).astype(np.int8)
    g = Gpu(cfg, trees, lv)
    g.set_state(q)
    sums = torch.zeros(4, dtype=torch.float64, device="cuda")
    g.ctx.conservation_sums(g.q, sums)
    before = sums.cpu().numpy().copy()
    g.regrid(tg, 1, 4)
    g.ctx.conservation_sums(g.q, sums)
    after = sums.cpu().numpy()
    mesh = O.Mesh(trees, lv, M, sphere=True)
    par = oracle_params(cfg)
    f = O.framed(q, M)
    O.ghost_fill(mesh, par, f)
    lv2 = O.regrid(mesh, tg, 1, 4)
    assert np.array_equal(g.ctx.leaves(), lv2)
    assert len(lv2) != len(lv)
    want = O.interior(O.transfer(mesh, O.Mesh(trees, lv2, M, sphere=True), par, f), M)
    got = g.state()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert abs(after[0] - before[0]) <= 1e-13 * abs(before[0])


def test_run_loop_with_regrids_equals_single_calls():
    """fcx_run on the sphere (plain steps, a criterion regrid every 2 steps)
    gives bit for bit the forest, state and dt of the same single calls, and
    keeps the mass to rounding."""
    import torch
    say("[sphere] run loop")
    trees, lv = _forest(13, 1, 3, 10)
    lmin, lmax, steps, every, thr = 1, 4, 7, 2, 0.6
    cfg = fcx.config(M, 64, fcx.FCX_SPHERE)
    q0 = _sphere_state(lv, 3)
    dt0 = 0.2 * (np.pi / 2) / (M << lmax)

    def fresh():
        ctx = fcx.Context(cfg, trees)
        ctx.upload_forest(lv)
        dt = torch.full((1,), dt0, dtype=torch.float64, device="cuda")
        return ctx, dt, torch.zeros_like(dt), torch.zeros(1, dtype=torch.int32, device="cuda")

    ctx, dt, nu, st = fresh()
    q = torch.from_numpy(q0.ravel().copy()).cuda()
    sums = torch.zeros(4, dtype=torch.float64, device="cuda")
    ctx.conservation_sums(q, sums)
    mass0 = sums[0].item()
    regrids = 0
    for n in range(steps):
        if n > 0 and n % every == 0:
            gh = torch.empty(ctx.ghost_elems(), dtype=torch.float64, device="cuda")
            before = ctx.num_patches()
            ctx.regrid(q, gh, 1, thr, lmin, lmax)
            regrids += ctx.num_patches() != before
            q2 = torch.empty(ctx.state_elems(), dtype=torch.float64, device="cuda")
            ctx.regrid_transfer(q, gh, q2)
            q = q2
        qn = torch.empty_like(q)
        gh = torch.empty(ctx.ghost_elems(), dtype=torch.float64, device="cuda")
        ctx.ghost_fill(q, gh)
        ctx.patch_step(q, gh, qn, dt, nu)
        ctx.reflux(q, qn, dt)
        if nu.item() > cfg.cfl_max:              # the redo rule, on the host
            qn = q
        ctx.next_dt(nu, dt, st)
        q = qn
    assert regrids > 0
    want, want_lv, want_dt = q.cpu().numpy(), ctx.leaves(), dt.item()
    ctx.conservation_sums(q, sums)
    assert abs(sums[0].item() - mass0) <= 1e-12 * abs(mass0)
    ctx, dt, nu, st = fresh()
    cap = 6 * (1 << (2 * lmax)) * 4 * M * M
    bufs = [torch.empty(cap, dtype=torch.float64, device="cuda") for _ in range(2)]
    bufs[0][:q0.size].copy_(torch.from_numpy(q0.ravel()))
    ghost = torch.empty(6 * (1 << (2 * lmax)) * 4 * (8 * M + 16), dtype=torch.float64,
                        device="cuda")
    which, cells = ctx.run(bufs[0], bufs[1], ghost, steps, 0, every, 1, thr, lmin, lmax,
                           dt, nu, st, fused=False)
    got = bufs[which][:ctx.state_elems()].cpu().numpy()
    assert np.array_equal(ctx.leaves(), want_lv)
    assert np.array_equal(got, want) and dt.item() == want_dt
    with pytest.raises(fcx.FcxError):
        ctx.run(bufs[which], bufs[1 - which], ghost, 1, steps, 0, 1, thr, lmin, lmax,
                dt, nu, st, fused=True)


@pytest.mark.parametrize("precision", [64, 32])
def test_geometry_after_regrids_equals_a_fresh_upload(precision):
    """The geometry a regrid builds for the new forest (tables and, in FP32,
    a step that reads the FP32 copy of them) equals bit for bit that of a
    context uploaded afresh with the same leaves: a patch's tables depend
    only on its tree, level and position."""
    say(f"[sphere] geometry after regrids precision={precision}")
    import torch
    trees, lv = _forest(5, 1, 3, 14)
    cfg = fcx.config(M, precision, fcx.FCX_SPHERE)
    g = Gpu(cfg, trees, lv)
    g.set_state(_sphere_state(lv, 3))
    rng = np.random.default_rng(7)
    kept = 0
    for _ in range(2):
        old = g.ctx.leaves()
        g.regrid(rng.integers(-1, 2, g.ctx.num_patches()).astype(np.int8), 1, 4)
        new = g.ctx.leaves()
        kept += len(set(map(tuple, old.tolist())) & set(map(tuple, new.tolist())))
    assert kept > 0
    fresh = Gpu(cfg, trees, g.ctx.leaves())
    assert torch.equal(g.ctx.sphere_geometry(), fresh.ctx.sphere_geometry())
    q = g.state()
    fresh.set_state(q)
    g.set_state(q)
    h = 1.0 / (M << 4)
    g.step(0.2 * h)
    fresh.step(0.2 * h)
    assert np.array_equal(g.state(), fresh.state())
