"""GPU parity: every C-ABI call of the HIP path against the CPU FP64 oracle on
identical seeded inputs.  FP64 bar: 1e-12 relative, per component, to that
component's max|q| (the target the method's double-precision path is held
to; a component whose largest value is below 1e-3 of the largest
component's is measured against that floor instead); FP32 bar: 1e-5
relative L1 per component against the FP64 oracle on the same mesh
schedule."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import fcx
from paper_1308_1472_amd import inputs as I
from tests.gpu_drive import (Gpu, ghost_to_frame, needed_mask, oracle_attempt,
                             oracle_params, say, smooth_sw_state)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def _rel(a, b, axis=1):
    """Largest over components (axis `axis`) of max|a - b| / max|b|, the
    scale floored at 1e-3 of the largest component's."""
    a = np.moveaxis(np.asarray(a, float), axis, 0)
    b = np.moveaxis(np.asarray(b, float), axis, 0)
    top = max(np.max(np.abs(b)), 1e-300)
    worst = 0.0
    for ak, bk in zip(a, b):
        scale = max(np.max(np.abs(bk)), 1e-3 * top)
        worst = max(worst, np.max(np.abs(ak - bk)) / scale)
    return worst


def _forest(domain, seed, lmin=2, lmax=5, nsplit=30):
    if domain == "walled":
        trees, pl = I.walled_square(); nt = 1
    elif domain == "periodic":
        trees, pl = I.periodic_square(); nt = 1
    elif domain == "brick":
        trees, pl = I.brick(2, 2, orient_codes=[0, 1, 6, 3]); nt = 4
    elif domain == "brick_sw":
        trees, pl = I.brick(2, 1); nt = 2
    raw = I.random_leaves(seed, nt, lmin, lmax, nsplit)
    lv = O.balance(trees, raw)
    assert np.array_equal(lv, fcx.balance(trees, raw))
    return trees, pl, lv


CASES = [("walled", fcx.FCX_SHALLOW, 8), ("periodic", fcx.FCX_ADVECTION, 8),
         ("brick", fcx.FCX_ADVECTION, 16), ("brick_sw", fcx.FCX_SHALLOW, 16),
         ("walled", fcx.FCX_SHALLOW, 32)]


def _setup(domain, phys, m, seed):
    trees, pl, lv = _forest(domain, seed)
    cfg = fcx.config(m, 64, phys, ax=0.8, ay=-0.55)
    if phys == fcx.FCX_SHALLOW:
        q = smooth_sw_state(lv, m, pl, seed)
    else:
        q = I.state_from(lv, m, lambda x, y: I.gaussian(x, y, 0.4, 0.6, 0.02)
                         + 0.3 * np.sin(5 * x) * np.cos(3 * y), pl)
    return trees, pl, lv, cfg, q


@pytest.mark.parametrize("domain,phys,m", CASES)
def test_ghost_fill_matches_oracle(domain, phys, m):
    say(f"[ghost] {domain} phys={phys} m={m}")
    trees, pl, lv, cfg, q = _setup(domain, phys, m, 7)
    gpu = Gpu(cfg, trees, lv)
    gpu.set_state(q)
    gpu.fill()
    got = ghost_to_frame(gpu.ghosts(), q, m)
    mesh = O.Mesh(trees, lv, m)
    f = O.framed(q, m)
    O.ghost_fill(mesh, oracle_params(cfg), f)
    mk = needed_mask(m)
    assert _rel(got[:, :, mk], f[:, :, mk]) <= 1e-15


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("reflux", [False, True])
@pytest.mark.parametrize("domain,phys,m", CASES)
def test_one_step_matches_oracle(domain, phys, m, fused, reflux):
    say(f"[step] {domain} phys={phys} m={m} fused={fused} reflux={reflux}")
    trees, pl, lv, cfg, q = _setup(domain, phys, m, 11)
    gpu = Gpu(cfg, trees, lv)
    gpu.set_state(q)
    h = 1.0 / (m << 5)
    dt = 0.4 * h
    nu, _ = gpu.step(dt, fused=fused, reflux=reflux)
    got = gpu.state()
    mesh = O.Mesh(trees, lv, m)
    par = oracle_params(cfg)
    f = O.framed(q, m)
    O.ghost_fill(mesh, par, f)
    fn, nu_o = O.step(mesh, par, f, dt, reflux)
    want = O.interior(fn, m)
    assert _rel(got, want) <= FP64_TOL
    assert abs(nu - nu_o) <= 1e-14 * nu_o


def _advection_16_patches_run(fused):
    trees, pl = I.periodic_square()
    lv = O.sfc_sort(I.uniform_leaves(1, 2))
    cfg = fcx.config(8, 64, fcx.FCX_ADVECTION, ax=1.0, ay=0.5)
    q0 = I.state_from(lv, 8, lambda x, y: I.gaussian(x, y), pl)
    gpu = Gpu(cfg, trees, lv)
    gpu.set_state(q0)
    for _ in range(100):
        gpu.step(0.028125, fused=fused)
    return trees, lv, cfg, q0, gpu.state()


@pytest.mark.parametrize("fused", [False, True])
def test_advection_16_patches_100_steps(fused):
    """16 patches of 8x8, a = (1, 0.5), periodic, CFL 0.9, MC + transverse."""
    say(f"[cfg-small] fused={fused}")
    trees, lv, cfg, q0, got = _advection_16_patches_run(fused)
    mesh = O.Mesh(trees, lv, 8)
    par = oracle_params(cfg)
    q = q0
    for _ in range(100):
        q, _ = O.advance(mesh, par, q, 0.028125)
    assert _rel(got, q) <= FP64_TOL


def _sw_adaptive_oracle(trees, pl, m, lmin, lmax, nsteps, regrid_every,
                        fn, thr=0.1, dt0=None):
    """Oracle reference run: initial mesh loop, CFL-controlled dt with the
    reject-and-redo rule, regrid every `regrid_every` attempts."""
    par = O.params(m, O.SHALLOW)
    lv = O.sfc_sort(I.uniform_leaves(len(trees), lmin))
    for _ in range(lmax - lmin + 1):
        mesh = O.Mesh(trees, lv, m)
        f = O.framed(I.state_from(lv, m, fn, pl), m)
        O.ghost_fill(mesh, par, f)
        lv2 = O.regrid(mesh, O.tags(mesh, par, f, 1, thr, lmin, lmax), lmin, lmax)
        if np.array_equal(lv2, lv):
            break
        lv = lv2
    mesh = O.Mesh(trees, lv, m)
    q = I.state_from(lv, m, fn, pl)
    hist = {"leaves": [lv.copy()], "tags": [], "dt": [], "nu": [], "ok": []}
    dt = dt0
    for n in range(nsteps):
        if n > 0 and n % regrid_every == 0:
            f = O.framed(q, m)
            O.ghost_fill(mesh, par, f)
            tg = O.tags(mesh, par, f, 1, thr, lmin, lmax)
            hist["tags"].append(tg)
            lv = O.regrid(mesh, tg, lmin, lmax)
            mesh2 = O.Mesh(trees, lv, m)
            q = O.interior(O.transfer(mesh, mesh2, par, f), m)
            mesh = mesh2
            hist["leaves"].append(lv.copy())
        hist["dt"].append(dt)
        q, nu, dt, ok = oracle_attempt(mesh, par, q, dt)
        hist["nu"].append(nu)
        hist["ok"].append(ok)
    return lv, q, hist, mesh


@pytest.mark.parametrize("fused", [False, True])
def test_adaptive_shallow_water_run_matches_oracle(fused):
    """Radial dam break with reflecting walls on an adaptive forest: tags,
    meshes, dt sequence and state all match over 16 steps with regrid every
    4 (levels 2-4, m = 8)."""
    say(f"[adaptive] fused={fused}")
    trees, pl = I.walled_square()
    m, lmin, lmax = 8, 2, 4
    fn = lambda x, y: I.dam_break(x, y)
    dt0 = 0.5 / (m << lmax) / 1.8
    lv_o, q_o, hist, _ = _sw_adaptive_oracle(trees, pl, m, lmin, lmax, 16, 4, fn,
                                             dt0=dt0)
    cfg = fcx.config(m, 64, fcx.FCX_SHALLOW)
    gpu = Gpu(cfg, trees, hist["leaves"][0])
    gpu.set_state(I.state_from(hist["leaves"][0], m, fn, pl))
    gpu.dt.fill_(dt0)
    r = 0
    for n in range(16):
        if n > 0 and n % 4 == 0:
            tg = gpu.tags(1, 0.1, lmin, lmax)
            assert np.array_equal(tg, hist["tags"][r])
            gpu.regrid(tg, lmin, lmax)
            r += 1
            assert np.array_equal(gpu.ctx.leaves(), hist["leaves"][r])
        nu, used = gpu.step(fused=fused, auto_dt=True)
        assert abs(used - hist["dt"][n]) <= 1e-13 * hist["dt"][n]
        assert abs(nu - hist["nu"][n]) <= 1e-13 * hist["nu"][n]
    # the CFL flag is raised exactly when the oracle saw a Courant number > 1
    assert int(gpu.status.item()) == int(max(hist["nu"]) > 1.0)
    assert _rel(gpu.state(), q_o) <= FP64_TOL


def test_tags_bit_exact_on_identical_state():
    say("[tags]")
    for seed in range(3):
        trees, pl, lv, cfg, q = _setup("walled", fcx.FCX_SHALLOW, 16, 40 + seed)
        gpu = Gpu(cfg, trees, lv)
        gpu.set_state(q)
        mesh = O.Mesh(trees, lv, 16)
        par = oracle_params(cfg)
        f = O.framed(q, 16)
        O.ghost_fill(mesh, par, f)
        for crit, thr in ((1, 0.5), (1, 2.0), (0, 0.05), (0, 0.3)):
            got = gpu.tags(crit, thr, 2, 5)
            want = O.tags(mesh, par, f, crit, thr, 2, 5)
            assert np.array_equal(got, want), (crit, thr)


def test_regrid_transfer_matches_oracle():
    say("[transfer]")
    trees, pl, lv, cfg, q = _setup("walled", fcx.FCX_SHALLOW, 8, 5)
    rng = np.random.default_rng(3)
    tg = rng.integers(-1, 2, len(lv)).astype(np.int8)
    gpu = Gpu(cfg, trees, lv)
    gpu.set_state(q)
    gpu.regrid(tg, 1, 6)
    mesh = O.Mesh(trees, lv, 8)
    par = oracle_params(cfg)
    f = O.framed(q, 8)
    O.ghost_fill(mesh, par, f)
    lv2 = O.regrid(mesh, tg, 1, 6)
    assert np.array_equal(gpu.ctx.leaves(), lv2)
    want = O.interior(O.transfer(mesh, O.Mesh(trees, lv2, 8), par, f), 8)
    assert _rel(gpu.state(), want) <= 1e-15


def test_one_call_regrid_equals_the_separate_calls():
    """fcx_regrid (ghost fill, criterion tags, apply) gives the oracle's
    tags-then-regrid forest, and the transfer on its ghost fill the oracle's
    state."""
    import torch
    say("[regrid one call]")
    trees, pl, lv, cfg, q = _setup("walled", fcx.FCX_SHALLOW, 16, 7)
    gpu = Gpu(cfg, trees, lv)
    gpu.set_state(q)
    mesh = O.Mesh(trees, lv, 16)
    par = oracle_params(cfg)
    f = O.framed(q, 16)
    O.ghost_fill(mesh, par, f)
    tg = O.tags(mesh, par, f, 1, 0.5, 1, 6)
    assert (tg != 0).any()
    q_old, g_old = gpu.q, gpu.ghost
    n = gpu.ctx.regrid(q_old, g_old, 1, 0.5, 1, 6)
    lv2 = O.regrid(mesh, tg, 1, 6)
    assert n == len(lv2) and np.array_equal(gpu.ctx.leaves(), lv2)
    gpu._alloc()
    gpu.ctx.regrid_transfer(q_old, g_old, gpu.q)
    torch.cuda.synchronize()
    want = O.interior(O.transfer(mesh, O.Mesh(trees, lv2, 16), par, f), 16)
    assert _rel(gpu.state(), want) <= 1e-15


@pytest.mark.parametrize("seed", [3, 8])
def test_tables_after_a_regrid_equal_a_fresh_build(seed):
    """After a regrid the patch tables are updated incrementally (patches
    whose neighbourhood is unchanged keep their records, renumbered) and
    reordered for the device; read back, they equal entry for entry the
    tables of a fresh upload of the same leaves."""
    say(f"[tables] seed={seed}")
    trees, pl = I.walled_square()
    cfg = fcx.config(16, 64, fcx.FCX_SHALLOW)
    ctx = fcx.Context(cfg, trees)
    ctx.upload_forest(fcx.balance(trees, I.random_leaves(seed, 1, 2, 5, 40)))
    rng = np.random.default_rng(seed)
    items = 0
    for r in range(3):
        tg = rng.integers(-1, 2, ctx.num_patches()).astype(np.int8)
        ctx.regrid_apply(tg, 1, 6)
        got = ctx.patch_table()
        ref = fcx.Context(cfg, trees)
        ref.upload_forest(ctx.leaves())
        want = ref.patch_table()
        for k in ("counts", "recs", "phislot", "family", "items", "aux"):
            assert np.array_equal(got[k], want[k]), (r, k)
        items += len(want["items"])
    assert items > 0


def _two_way_coarse_corners(lv):
    """Number of (leaf, corner) pairs whose two faces at that corner both
    border finer leaves: the corner cell takes a reflux correction from an
    xi face and from an eta face."""
    have = {(int(a["level"]), int(a["ix"]), int(a["iy"])) for a in lv}
    n = 0
    for a in lv:
        l, x, y = int(a["level"]), int(a["ix"]), int(a["iy"])
        finer = [(l + 1, 2 * x - 1, 2 * y) in have, (l + 1, 2 * x + 2, 2 * y) in have,
                 (l + 1, 2 * x, 2 * y - 1) in have, (l + 1, 2 * x, 2 * y + 2) in have]
        n += sum(finer[fx] and finer[2 + fy] for fx in (0, 1) for fy in (0, 1))
    return n


@pytest.mark.parametrize("precision,m", [(64, 16), (32, 16), (32, 8), (32, 32), (64, 32)])
def test_advance_equals_the_three_calls(precision, m):
    """fcx_advance (update, reflux and next dt in one launch: the tile that
    completes an item's arrivals applies its reflux) gives bit for bit the
    state, dt and flags of fcx_fused_step + fcx_reflux + fcx_next_dt, on a
    mesh where coarse corner cells take both an xi and an eta correction,
    with one tile per patch (m = 8, 16) and four (m = 32); the last step
    exceeds cfl_max so the flag path runs too."""
    import torch
    say(f"[advance] precision={precision} m={m}")
    trees, pl = I.walled_square()
    lv = fcx.balance(trees, I.random_leaves(21, 1, 2, 5, 40))
    assert _two_way_coarse_corners(lv) > 0
    q0 = smooth_sw_state(lv, m, pl, 5)
    # the last step's Courant number exceeds cfl_max: with the redo rule off
    # it is kept and flagged, as by the separate calls
    cfg = fcx.config(m, precision, fcx.FCX_SHALLOW, redo=0)
    dtype = torch.float64 if precision == 64 else torch.float32
    dt0 = 0.3 / (m << 5)
    results = []
    for one_call in (False, True):
        ctx = fcx.Context(cfg, trees)
        ctx.upload_forest(lv)
        q = torch.from_numpy(q0.ravel().copy()).to(dtype).cuda()
        dt = torch.full((1,), dt0, dtype=torch.float64, device="cuda")
        nu = torch.zeros_like(dt)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        hist = []
        for n in range(6):
            if n == 5:
                dt.mul_(2.0)
            qn = torch.empty_like(q)
            if one_call:
                ctx.advance(q, qn, dt, nu, st)
            else:
                ctx.fused_step(q, qn, dt, nu)
                ctx.reflux(q, qn, dt)
                ctx.next_dt(nu, dt, st)
            q = qn
            hist.append((dt.item(), st.item(), nu.item()))
        results.append((q.cpu().numpy(), hist))
    (qa, ha), (qb, hb) = results
    assert np.array_equal(qa, qb, equal_nan=True)
    assert ha == hb
    assert ha[-1][1] & 1 and not ha[-2][1] & 1


@pytest.mark.parametrize("fused", [True, False])
def test_native_run_loop_equals_single_calls(fused):
    """fcx_run (steps with a regrid every 3) gives bit for bit the state,
    forest, dt and flags of the same sequence of single calls."""
    import torch
    say(f"[run loop] fused={fused}")
    trees, pl = I.walled_square()
    m, lmin, lmax = 8, 2, 4
    lv = fcx.balance(trees, I.random_leaves(4, 1, 2, 4, 10))
    q0 = I.state_from(lv, m, lambda x, y: I.dam_break(x, y, 0.45, 0.5, 0.2), pl)
    cfg = fcx.config(m, 64, fcx.FCX_SHALLOW)
    dt0 = 0.4 / (m << lmax) / 1.5
    steps = 10

    def fresh():
        ctx = fcx.Context(cfg, trees)
        ctx.upload_forest(lv)
        dt = torch.full((1,), dt0, dtype=torch.float64, device="cuda")
        return ctx, dt, torch.zeros_like(dt), torch.zeros(1, dtype=torch.int32, device="cuda")

    # single calls
    ctx, dt, nu, st = fresh()
    q = torch.from_numpy(q0.ravel().copy()).cuda()
    for n in range(steps):
        if n > 0 and n % 3 == 0:
            g = torch.empty(ctx.ghost_elems(), dtype=torch.float64, device="cuda")
            ctx.regrid(q, g, 1, 0.3, lmin, lmax)
            q2 = torch.empty(ctx.state_elems(), dtype=torch.float64, device="cuda")
            ctx.regrid_transfer(q, g, q2)
            q = q2
        qn = torch.empty_like(q)
        if fused:
            ctx.advance(q, qn, dt, nu, st)
        else:
            g = torch.empty(ctx.ghost_elems(), dtype=torch.float64, device="cuda")
            ctx.ghost_fill(q, g)
            ctx.patch_step(q, g, qn, dt, nu)
            ctx.reflux(q, qn, dt)
            if nu.item() > cfg.cfl_max:          # the redo rule, on the host
                qn = q
            ctx.next_dt(nu, dt, st)
        q = qn
    want, want_lv, want_dt = q.cpu().numpy(), ctx.leaves(), dt.item()
    # the run loop
    ctx, dt, nu, st = fresh()
    cap = (1 << (2 * lmax)) * 3 * m * m
    bufs = [torch.empty(cap, dtype=torch.float64, device="cuda") for _ in range(2)]
    bufs[0][:q0.size].copy_(torch.from_numpy(q0.ravel()))
    ghost = torch.empty((1 << (2 * lmax)) * 3 * (8 * m + 16), dtype=torch.float64,
                        device="cuda")
    which, cells = ctx.run(bufs[0], bufs[1], ghost, steps, 0, 3, 1, 0.3, lmin, lmax,
                           dt, nu, st, fused=fused)
    got = bufs[which][:ctx.state_elems()].cpu().numpy()
    assert np.array_equal(ctx.leaves(), want_lv)
    assert np.array_equal(got, want) and dt.item() == want_dt
    assert cells > 0
    # a capacity that is too small is refused
    with pytest.raises(fcx.FcxError):
        ctx.run(bufs[which][:10], bufs[1 - which], ghost, 1, steps, 0, 1, 0.3, lmin, lmax,
                dt, nu, st, fused=fused)


def test_conservation_sums_match_oracle():
    say("[sums]")
    for domain, phys, m in CASES:
        trees, pl, lv, cfg, q = _setup(domain, phys, m, 3)
        gpu = Gpu(cfg, trees, lv)
        gpu.set_state(q)
        got = gpu.conservation_sums()
        want = O.sums(O.Mesh(trees, lv, m), oracle_params(cfg), O.framed(q, m))
        np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15 * np.abs(want).max())


@pytest.mark.parametrize("m", [8, 16, 32])
@pytest.mark.parametrize("fused", [False, True])
def test_fp32_within_1e5_of_fp64_oracle(fused, m):
    """FP32 state and fluxes (FP64 dt, CFL and sums) against the FP64 oracle
    on the same mesh and dt schedule: one 8x8 tile per patch (m = 8), one
    16x16 tile (m = 16) and four (m = 32)."""
    say(f"[fp32] fused={fused} m={m}")
    trees, pl = I.walled_square()
    lmin, lmax = 2, 4
    fn = lambda x, y: I.dam_break(x, y)
    dt0 = 0.5 / (m << lmax) / 1.8
    lv_o, q_o, hist, _ = _sw_adaptive_oracle(trees, pl, m, lmin, lmax, 12, 4, fn,
                                             dt0=dt0)
    cfg = fcx.config(m, 32, fcx.FCX_SHALLOW)
    gpu = Gpu(cfg, trees, hist["leaves"][0])
    gpu.set_state(I.state_from(hist["leaves"][0], m, fn, pl))
    r = 0
    for n in range(12):
        if n > 0 and n % 4 == 0:
            gpu.regrid(hist["tags"][r], lmin, lmax)
            r += 1
            assert np.array_equal(gpu.ctx.leaves(), hist["leaves"][r])
        if hist["ok"][n]:                    # attempts the oracle kept
            gpu.step(hist["dt"][n], fused=fused)
    got = gpu.state()
    for k in range(3):
        err = np.sum(np.abs(got[:, k] - q_o[:, k])) / np.sum(np.abs(q_o[:, k]))
        assert err <= 1e-5, (k, err)


def test_mass_conserved_on_gpu_adaptive():
    say("[mass]")
    trees, pl = I.walled_square()
    raw = I.refine_near(1, 2, 4, [(0.5, 0.5)], pl, radius=1.2)
    lv = fcx.balance(trees, raw)
    cfg = fcx.config(16, 64, fcx.FCX_SHALLOW)
    gpu = Gpu(cfg, trees, lv)
    gpu.set_state(I.state_from(lv, 16, lambda x, y: I.dam_break(x, y), pl))
    m0 = gpu.conservation_sums()
    gpu.dt.fill_(0.3 / 256)
    for _ in range(100):
        gpu.step(fused=True, auto_dt=True)
    m1 = gpu.conservation_sums()
    assert abs(m1[0] - m0[0]) / m0[0] <= 1e-12
    assert int(gpu.status.item()) == 0


def test_error_paths():
    say("[errors]")
    import torch
    trees, pl = I.walled_square()
    cfg = fcx.config(8, 64, fcx.FCX_SHALLOW)
    ctx = fcx.Context(cfg, trees)
    # unbalanced forest
    lv = [tuple(a) for a in I.uniform_leaves(1, 1).tolist()]
    lv.remove((0, 1, 0, 0))
    lv += [(0, 3, x, y) for x in range(4) for y in range(4)]
    lv = fcx.sfc_sort(np.array(lv, dtype=fcx.LEAF_DTYPE))
    with pytest.raises(fcx.FcxError) as e:
        ctx.upload_forest(lv)
    assert e.value.code == -2
    # unsorted leaves
    with pytest.raises(fcx.FcxError) as e:
        ctx.upload_forest(I.uniform_leaves(1, 2)[::-1].copy())
    assert e.value.code == -1
    # calls before an upload
    q = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        ctx.ghost_fill(q, q)
    ctx.upload_forest(fcx.sfc_sort(I.uniform_leaves(1, 1)))
    g = Gpu(cfg, trees, fcx.sfc_sort(I.uniform_leaves(1, 1)))
    rc = fcx.lib().fcx_patch_step(g.ctx.h, g.q.data_ptr(), g.ghost.data_ptr(),
                                  g.q.data_ptr(), g.dt.data_ptr(),
                                  g.numax.data_ptr(), None)
    assert rc == -1                                  # aliasing rejected
    # a non-positive depth is reported through the status word
    q = np.ones((4, 3, 8, 8))
    q[2, 0, 3, 3] = -1.0
    g.set_state(q)
    g.dt.fill_(1e-3)
    g.step(auto_dt=True)
    assert int(g.status.item()) & 2
    # CFL above cfl_max is flagged
    g2 = Gpu(cfg, trees, fcx.sfc_sort(I.uniform_leaves(1, 1)))
    g2.set_state(np.ones((4, 3, 8, 8)) * np.array([1.0, 0.0, 0.0])[None, :, None, None])
    g2.dt.fill_(0.2)                                 # nu = 0.2 * 16 * 1 > 1
    g2.step(auto_dt=True)
    assert int(g2.status.item()) & 1


def test_single_patch_and_periodic_self_neighbour():
    """Edge case: one patch (level 0) whose every neighbour is itself."""
    say("[single]")
    trees, pl = I.periodic_square()
    lv = fcx.sfc_sort(I.uniform_leaves(1, 0))
    cfg = fcx.config(16, 64, fcx.FCX_ADVECTION, ax=0.7, ay=0.3)
    q = I.state_from(lv, 16, lambda x, y: I.gaussian(x, y), pl)
    gpu = Gpu(cfg, trees, lv)
    gpu.set_state(q)
    gpu.step(0.9 / 16 / 0.7, fused=True)
    want, _ = O.advance(O.Mesh(trees, lv, 16), oracle_params(cfg), q, 0.9 / 16 / 0.7)
    assert _rel(gpu.state(), want) <= FP64_TOL
