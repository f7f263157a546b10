"""CPU-side checks of the C ABI: the library loads, exports every entry point
that include/fcx.h declares, and its host-only integer work (SFC order, 2:1
balance) agrees exactly with the oracle's independent implementation."""
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import fcx
from paper_1308_1472_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "fcx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fcx_[a-z_0-9]+)\s*\(", text)))


def test_header_matches_binding_list():
    assert _header_functions() == sorted(fcx.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = fcx.lib()
    for name in _header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", fcx.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (fcx_\w+)", out))
    assert set(_header_functions()) <= exported
    assert lib.fcx_version() == 1


@pytest.mark.parametrize("seed", range(4))
def test_sfc_sort_matches_oracle(seed):
    raw = I.random_leaves(seed, 3, 1, 7, 80)
    rng = np.random.default_rng(seed)
    raw = raw[rng.permutation(len(raw))]
    a = fcx.sfc_sort(raw)
    b = O.sfc_sort(raw)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("domain", ["walled", "periodic", "brick", "sphere"])
@pytest.mark.parametrize("seed", range(3))
def test_balance_matches_oracle(domain, seed):
    if domain == "walled":
        trees, _ = I.walled_square(); nt = 1
    elif domain == "periodic":
        trees, _ = I.periodic_square(); nt = 1
    elif domain == "brick":
        trees, _ = I.brick(2, 2, orient_codes=[0, 1, 6, 3]); nt = 4
    else:
        trees = I.cubed_sphere(); nt = 6
    raw = I.random_leaves(100 + seed, nt, 1, 7, 60)
    a = fcx.balance(trees, raw)
    b = O.balance(trees, raw)
    assert np.array_equal(a, b)


def test_balance_rejects_bad_connectivity():
    trees, _ = I.walled_square()
    bad = trees.copy()
    bad["bc"][0, 0] = 0
    bad["nbr_tree"][0, 0] = 0
    bad["nbr_face"][0, 0] = 1
    with pytest.raises(fcx.FcxError) as e:
        fcx.balance(bad, I.uniform_leaves(1, 1))
    assert e.value.code == -1


@pytest.mark.parametrize("domain", ["walled", "periodic", "brick", "sphere"])
@pytest.mark.parametrize("seed", range(4))
def test_regrid_leaves_matches_oracle(domain, seed):
    """Host regrid (incremental balance) against the oracle's plain
    refine / merge / full re-balance, on random tags."""
    if domain == "walled":
        trees, _ = I.walled_square(); nt = 1
    elif domain == "periodic":
        trees, _ = I.periodic_square(); nt = 1
    elif domain == "brick":
        trees, _ = I.brick(2, 2, orient_codes=[0, 1, 6, 3]); nt = 4
    else:
        trees = I.cubed_sphere(); nt = 6
    lv = O.balance(trees, I.random_leaves(200 + seed, nt, 1, 6, 50))
    rng = np.random.default_rng(seed)
    for lmin, lmax in ((1, 7), (2, 5)):
        tg = rng.choice(np.array([-1, -1, 0, 1], np.int8), len(lv))
        a = fcx.regrid_leaves(trees, lv, tg, lmin, lmax)
        b = O.regrid(O.Mesh(trees, lv, 8), tg, lmin, lmax)
        assert np.array_equal(a, b)


def test_committed_tagger_weights_load_safely():
    import json
    from paper_1308_1472_amd import learned as L
    z = np.load(L.WEIGHTS, allow_pickle=False)
    assert z["params"].shape == (fcx.MLP_PARAMS,) and z["params"].dtype == np.float32
    assert z["norm"].shape == (2 * fcx.MLP_INPUTS,) and np.all(z["norm"][16:] > 0)
    meta = json.loads(str(z["meta"]))
    assert meta["labels"] == "n+4" and meta["train_seeds"] == 180
    assert np.all(np.isfinite(z["params"]))
