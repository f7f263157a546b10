"""GPU parity of the advection tile (staged in the frame where both velocity
components are non-negative) against the CPU FP64 oracle: every sign
combination of (a_x, a_y), zero components, every limiter and transverse
mode, plain and fused halos, coarse-fine faces (the reflux reads the tile's
face terms), single- and multi-tile patches, multi-tree forests with rotated
neighbours.  FP64 within 1e-12 relative to max|q|; Courant number within
1e-14; FP32 within 1e-5 relative L1."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import fcx
from paper_1308_1472_amd import inputs as I
from tests.gpu_drive import Gpu, oracle_params, say

pytestmark = pytest.mark.gpu

SIGNS = [(0.8, 0.55), (-0.8, 0.55), (0.8, -0.55), (-0.8, -0.55), (0.0, 0.7),
         (-0.6, 0.0), (0.0, -0.7)]


def _case(domain, m, seed, uniform=False):
    if domain == "brick":
        trees, pl = I.brick(2, 2, orient_codes=[0, 1, 6, 3]); nt = 4
    elif domain == "walled":
        trees, pl = I.walled_square(); nt = 1
    elif domain == "extrap":
        trees, pl = I.walled_square(bc=I.BC_EXTRAP); nt = 1
    elif domain == "brick_translated":
        trees, pl = I.brick(3, 2, periodic=(True, False)); nt = 6
    else:
        trees, pl = I.periodic_square(); nt = 1
    if uniform:
        lv = fcx.sfc_sort(I.uniform_leaves(nt, 2))
    else:
        lv = fcx.balance(trees, I.random_leaves(seed, nt, 2, 4, 20))
    q = I.state_from(lv, m, lambda x, y: I.gaussian(x, y, 0.45, 0.55, 0.03)
                     + 0.3 * np.sin(5 * x) * np.cos(3 * y)
                     + 0.2 * (x > 0.6) * (y < 0.35), pl)
    return trees, lv, q


def _compare(cfg, trees, lv, q, fused, steps=2):
    m = cfg.m
    gpu = Gpu(cfg, trees, lv)
    gpu.set_state(q)
    mesh = O.Mesh(trees, lv, m)
    par = oracle_params(cfg)
    dt = 0.45 / (m << 4)
    want = q
    for _ in range(steps):
        nu, _ = gpu.step(dt, fused=fused, reflux=True)
        f = O.framed(want, m)
        O.ghost_fill(mesh, par, f)
        fn, nu_o = O.step(mesh, par, f, dt, True)
        want = O.interior(fn, m)
        assert abs(nu - nu_o) <= 1e-6 * nu_o if cfg.precision == 32 else \
            abs(nu - nu_o) <= 1e-14 * nu_o
    got = gpu.state()
    if cfg.precision == 64:
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert err <= 1e-12, err
    else:
        err = np.sum(np.abs(got - want)) / np.sum(np.abs(want))
        assert err <= 1e-5, err
    return err


@pytest.mark.parametrize("ax,ay", SIGNS)
@pytest.mark.parametrize("m,tile", [(8, 0), (16, 0), (32, 16), (32, 8)])
def test_velocity_signs(ax, ay, m, tile):
    say(f"[advect] signs ax={ax} ay={ay} m={m} tile={tile}")
    trees, lv, q = _case("periodic", m, 3)
    for fused in (False, True):
        _compare(fcx.config(m, 64, fcx.FCX_ADVECTION, ax=ax, ay=ay, tile=tile),
                 trees, lv, q, fused)


@pytest.mark.parametrize("limiter", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("transverse", [0, 1, 2])
def test_limiters_and_transverse_modes(limiter, transverse):
    say(f"[advect] limiter={limiter} transverse={transverse}")
    trees, lv, q = _case("periodic", 16, 5)
    for ax, ay in [(0.7, -0.45), (-0.35, 0.9)]:
        _compare(fcx.config(16, 64, fcx.FCX_ADVECTION, limiter=limiter,
                            transverse=transverse, ax=ax, ay=ay),
                 trees, lv, q, True)


@pytest.mark.parametrize("ax,ay", SIGNS[:4])
def test_rotated_trees(ax, ay):
    """Four trees glued with rotations: the fused halo takes the general
    gather for most ghost cells."""
    say(f"[advect] brick ax={ax} ay={ay}")
    trees, lv, q = _case("brick", 16, 7)
    for fused in (False, True):
        _compare(fcx.config(16, 64, fcx.FCX_ADVECTION, ax=ax, ay=ay), trees, lv, q, fused)


@pytest.mark.parametrize("m", [8, 16, 32])
def test_fp32(m):
    say(f"[advect] fp32 m={m}")
    trees, lv, q = _case("periodic", m, 9)
    for ax, ay in SIGNS[:4]:
        _compare(fcx.config(m, 32, fcx.FCX_ADVECTION, ax=ax, ay=ay), trees, lv, q, True,
                 steps=3)


@pytest.mark.parametrize("limiter", [0, 1, 2, 3, 4])
def test_fp32_limiters(limiter):
    """FP32 tiles: minmod and MC take their median-of-three forms."""
    say(f"[advect] fp32 limiter={limiter}")
    trees, lv, q = _case("periodic", 16, 13)
    for ax, ay in [(0.7, -0.45), (-0.35, 0.9)]:
        _compare(fcx.config(16, 32, fcx.FCX_ADVECTION, limiter=limiter, ax=ax, ay=ay),
                 trees, lv, q, True, steps=3)


@pytest.mark.parametrize("domain", ["walled", "extrap", "brick_translated", "periodic"])
@pytest.mark.parametrize("uniform", [True, False])
@pytest.mark.parametrize("m", [8, 16, 32])
def test_walls_and_same_level_halos(domain, uniform, m):
    """Reflecting and extrapolating walls and translated neighbours: the
    fused halo's strip copies (uniform source per strip) and corner cells,
    every velocity sign, against the oracle."""
    say(f"[advect] halo domain={domain} uniform={uniform} m={m}")
    trees, lv, q = _case(domain, m, 11, uniform)
    for ax, ay in SIGNS[:4]:
        for fused in (True, False):
            _compare(fcx.config(m, 64, fcx.FCX_ADVECTION, ax=ax, ay=ay), trees, lv, q, fused)
