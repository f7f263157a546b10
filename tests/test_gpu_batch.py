"""GPU tests of batches of independent forests: one launch per tile class over
forests of different patch size and physics equals each forest's own
fused step and the CPU oracle; graph replays equal eager steps; every tuning
gives the same state; per-forest dt and sums."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import fcx
from paper_1308_1472_amd import inputs as I
from tests.gpu_drive import oracle_params, say, smooth_sw_state

pytestmark = pytest.mark.gpu

# (physics, m, domain, seed)
FORESTS = [(fcx.FCX_ADVECTION, 8, "periodic", 1), (fcx.FCX_SHALLOW, 16, "walled", 2),
           (fcx.FCX_ADVECTION, 32, "periodic", 3), (fcx.FCX_SHALLOW, 8, "walled", 4),
           (fcx.FCX_SHALLOW, 32, "walled", 5)]


def _make(precision=64):
    import torch
    ctxs, meshes, states, pars = [], [], [], []
    for phys, m, dom, seed in FORESTS:
        trees, pl = I.periodic_square() if dom == "periodic" else I.walled_square()
        lv = fcx.balance(trees, I.random_leaves(seed, 1, 2, 5, 12))
        cfg = fcx.config(m, precision, phys, ax=0.6 + 0.1 * seed, ay=-0.3)
        ctx = fcx.Context(cfg, trees)
        ctx.upload_forest(lv)
        if phys == fcx.FCX_SHALLOW:
            q = smooth_sw_state(lv, m, pl, seed)
        else:
            q = I.state_from(lv, m, lambda x, y: I.gaussian(x, y, 0.3 + 0.1 * seed, 0.5, 0.02), pl)
        ctxs.append(ctx)
        meshes.append((trees, lv))
        states.append(q)
        pars.append(oracle_params(cfg))
    batch = fcx.Batch(ctxs)
    dtype = torch.float64 if precision == 64 else torch.float32
    qb = torch.empty(batch.state_elems(), dtype=dtype, device="cuda")
    for f, q in enumerate(states):
        o = batch.state_offset(f)
        qb[o:o + q.size].copy_(torch.from_numpy(q.ravel()))
    return batch, ctxs, meshes, states, pars, qb


def _split(batch, ctxs, qb):
    out = []
    for f, c in enumerate(ctxs):
        o = batch.state_offset(f)
        n = c.state_elems()
        out.append(qb[o:o + n].double().cpu().numpy().reshape(
            c.num_patches(), c.meqn, c.cfg.m, c.cfg.m))
    return out


def _dts(n):
    # Courant number about 0.4 on the finest cells (level 5) of each forest
    return np.array([0.4 / (FORESTS[f][1] << 5) / 1.6 * (1 + 0.05 * f)
                     for f in range(n)])


def test_batch_step_matches_single_forests_and_oracle():
    import torch
    say("[batch] step vs forests vs oracle")
    batch, ctxs, meshes, states, pars, qb = _make()
    n = batch.n
    dts = _dts(n)
    dt = torch.tensor(dts, device="cuda")
    nu = torch.zeros(n, dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    qn = torch.empty_like(qb)
    batch.step(qb, qn, dt, nu, st)
    got = _split(batch, ctxs, qn)
    nus = nu.cpu().numpy()
    for f, ctx in enumerate(ctxs):
        # the forest's own fused step + reflux
        q = torch.from_numpy(states[f].ravel().copy()).cuda()
        q2 = torch.empty_like(q)
        d1 = torch.tensor([dts[f]], device="cuda")
        nu1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.fused_step(q, q2, d1, nu1)
        ctx.reflux(q, q2, d1)
        own = q2.cpu().numpy().reshape(got[f].shape)
        assert np.array_equal(got[f], own), f
        trees, lv = meshes[f]
        want, nu_o = O.advance(O.Mesh(trees, lv, ctx.cfg.m), pars[f], states[f], dts[f])
        assert np.max(np.abs(got[f] - want)) <= 1e-12 * np.max(np.abs(want))
        # next dt per forest: dt * 0.9 / nu
        assert abs(dt[f].item() - dts[f] * 0.9 / nu_o) <= 1e-12 * dts[f]
    assert int(st.sum().item()) == 0


@pytest.mark.parametrize("persistent", [0, 1])
def test_graph_replays_equal_eager_steps(persistent):
    """Replays of a captured graph equal eager steps, in both launch forms
    (the persistent one clears its work counters with a captured kernel)."""
    import torch
    say(f"[batch] graph replay persistent={persistent}")
    batch, ctxs, meshes, states, pars, q0 = _make(32)
    batch.set_tuning(16, 64, 256, persistent)
    n = batch.n
    mk = lambda: (torch.tensor(_dts(n), device="cuda"),
                  torch.zeros(n, dtype=torch.float64, device="cuda"),
                  torch.zeros(n, dtype=torch.int32, device="cuda"))
    # eager reference: 6 steps
    qa, qb = q0.clone(), torch.empty_like(q0)
    dt, nu, st = mk()
    for k in range(6):
        batch.step(qa, qb, dt, nu, st)
        qa, qb = qb, qa
    eager = qa.clone()
    # graph of 2 steps, replayed 3 times with eager work in between
    ga, gb = q0.clone(), torch.empty_like(q0)
    dt2, nu2, st2 = mk()
    batch.capture(2, ga, gb, dt2, nu2, st2)
    checks = []
    for r in range(3):
        batch.replay()
        torch.cuda.synchronize()
        scratch = torch.randn(1000, device="cuda").sum()   # eager work
        torch.cuda.synchronize()
        checks.append(ga.clone())
        del scratch
    # every replay: the state after 2(r+1) eager steps
    qa, qb = q0.clone(), torch.empty_like(q0)
    dt, nu, st = mk()
    for r in range(3):
        for k in range(2):
            batch.step(qa, qb, dt, nu, st)
            qa, qb = qb, qa
        assert torch.equal(checks[r], qa), r
    assert torch.equal(checks[-1], eager)
    assert torch.equal(dt2, dt)


def test_every_tuning_gives_the_same_state():
    import torch
    say("[batch] tunings")
    batch, ctxs, meshes, states, pars, q0 = _make()
    n = batch.n
    ref = None
    for tb in (8, 16):
        for t8 in (64, 128):
            for t16 in (256, 512):
                for pers in (0, 1):
                    batch.set_tuning(tb, t8, t16, pers)
                    dt = torch.tensor(_dts(n), device="cuda")
                    nu = torch.zeros(n, dtype=torch.float64, device="cuda")
                    st = torch.zeros(n, dtype=torch.int32, device="cuda")
                    qn = torch.empty_like(q0)
                    batch.step(q0, qn, dt, nu, st)
                    if ref is None:
                        ref = qn.clone()
                    else:
                        err = (qn - ref).abs().max().item()
                        assert err <= 1e-13 * ref.abs().max().item(), (tb, t8, t16, pers)


def test_batch_sums_match_oracle():
    import torch
    say("[batch] sums")
    batch, ctxs, meshes, states, pars, q0 = _make()
    out = torch.zeros(4 * batch.n, dtype=torch.float64, device="cuda")
    batch.sums(q0, out)
    got = out.cpu().numpy().reshape(batch.n, 4)
    for f, c in enumerate(ctxs):
        trees, lv = meshes[f]
        want = O.sums(O.Mesh(trees, lv, c.cfg.m), pars[f], O.framed(states[f], c.cfg.m))
        # momentum sums nearly cancel: absolute bar at the scale of sum |q|
        np.testing.assert_allclose(got[f, :c.meqn], want, rtol=1e-14, atol=1e-15)
        assert np.all(got[f, c.meqn:] == 0)


# Advection forests of uniform leaves (every halo a strip copy) with every
# velocity sign, walls and translated trees, and enough tiles that each
# wavefront of the strip-halo launch walks several items (on 256 CUs: 5120
# wavefronts for 16 x 16 tiles, 6144 for 8 x 8) and some walks cross from one
# forest into the next.  The 16 x 16 class mixes limiters (limiter and
# transverse mode read at run time), the 8 x 8 class is MC only (fixed when
# compiling).  (m, domain, level, ax, ay, limiter)
LONG_RUNS = [(16, "periodic", 6, 0.8, 0.55, 4), (16, "walled", 6, -0.7, 0.45, 4),
             (32, "periodic", 5, 0.6, -0.9, 4), (16, "brick", 5, -0.5, -0.65, 1),
             (8, "walled", 6, 0.9, -0.2, 4), (8, "periodic", 6, -0.3, 0.75, 4),
             (8, "periodic", 5, 0.0, -0.7, 4)]


@pytest.mark.parametrize("precision", [64, 32])
def test_long_runs_of_strip_halo_tiles(precision):
    """Each forest of the batch equals its own fused step and reflux bit for
    bit, with the same next dt (the Courant number is carried per forest
    along a walk); two of them also against the oracle."""
    import torch
    say(f"[batch] long runs of strip-halo tiles precision={precision}")
    ctxs, meshes, states, pars, dts = [], [], [], [], []
    for k, (m, dom, level, ax, ay, lim) in enumerate(LONG_RUNS):
        if dom == "brick":
            trees, pl = I.brick(3, 2, periodic=(True, False)); nt = 6
        elif dom == "walled":
            trees, pl = I.walled_square(); nt = 1
        else:
            trees, pl = I.periodic_square(); nt = 1
        lv = fcx.sfc_sort(I.uniform_leaves(nt, level))
        cfg = fcx.config(m, precision, fcx.FCX_ADVECTION, ax=ax, ay=ay, limiter=lim)
        ctx = fcx.Context(cfg, trees)
        ctx.upload_forest(lv)
        q = I.state_from(lv, m, lambda x, y: I.gaussian(x, y, 0.3 + 0.05 * k, 0.55, 0.02)
                         + 0.2 * np.sin(4 * x + k) * np.cos(3 * y), pl)
        ctxs.append(ctx)
        meshes.append((trees, lv))
        states.append(q)
        pars.append(oracle_params(cfg))
        dts.append(0.45 / ((m << level) * max(abs(ax), abs(ay))))
    batch = fcx.Batch(ctxs)
    dtype = torch.float64 if precision == 64 else torch.float32
    qb = torch.empty(batch.state_elems(), dtype=dtype, device="cuda")
    for f, q in enumerate(states):
        o = batch.state_offset(f)
        qb[o:o + q.size].copy_(torch.from_numpy(q.ravel()))
    n = batch.n
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    nu = torch.zeros(n, dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    qn = torch.empty_like(qb)
    batch.step(qb, qn, dt, nu, st)
    got = _split(batch, ctxs, qn)
    assert int(st.sum().item()) == 0
    for f, ctx in enumerate(ctxs):
        q = torch.from_numpy(states[f].ravel().copy()).to(dtype).cuda()
        q2 = torch.empty_like(q)
        d1 = torch.tensor([dts[f]], dtype=torch.float64, device="cuda")
        nu1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.fused_step(q, q2, d1, nu1)
        ctx.reflux(q, q2, d1)
        own = q2.double().cpu().numpy().reshape(got[f].shape)
        if LONG_RUNS[f][0] == 8 or LONG_RUNS[f][5] != 4:
            assert np.array_equal(got[f], own), f
        else:
            # an MC forest in a class that reads the limiter at run time:
            # the arithmetic is the same, the compiler's fused multiply-adds
            # are not all
            err = np.max(np.abs(got[f] - own)) / np.max(np.abs(own))
            assert err <= (1e-15 if precision == 64 else 1e-6), (f, err)
        assert abs(dt[f].item() - dts[f] * 0.9 / nu1.item()) <= 1e-15 * dts[f], f
        if f in (2, 4):
            trees, lv = meshes[f]
            want, nu_o = O.advance(O.Mesh(trees, lv, ctx.cfg.m), pars[f], states[f], dts[f])
            # (FP32 tiles take the velocity in FP32)
            assert abs(nu1.item() - nu_o) <= (1e-14 if precision == 64 else 1e-6) * nu_o
            if precision == 64:
                assert np.max(np.abs(got[f] - want)) <= 1e-12 * np.max(np.abs(want))
            else:
                assert np.sum(np.abs(got[f] - want)) <= 1e-5 * np.sum(np.abs(want))


def test_autotuner_picks_a_valid_config(tmp_path, monkeypatch):
    from paper_1308_1472_amd import autotune
    say("[batch] autotune")
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    batch, ctxs, meshes, states, pars, q0 = _make(32)
    before = q0.clone()
    best, timings = autotune.tune(batch, q0, steps=2, reps=1)
    combos = 1
    for vals in autotune.SPACE.values():
        combos *= len(vals)
    assert len(timings) == combos == 16 and all(v > 0 for v in timings.values())
    import torch
    assert torch.equal(q0, before)           # state untouched
    best2, _ = autotune.tune(batch, q0)      # second call: from the cache
    assert best2 == best
