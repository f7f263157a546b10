"""Pins of the oracle's forest: SFC order, the paper's mesh bookkeeping,
2:1 balance checked by brute-force geometry (independent of the oracle's
probe-based test), minimality of the balanced refinement."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_1472_amd import inputs as I
from tests import helpers as H

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_morton_order_of_children():
    lv = O.sfc_sort(I.uniform_leaves(1, 1)[::-1])
    assert [(a["ix"], a["iy"]) for a in lv] == [(0, 0), (1, 0), (0, 1), (1, 1)]
    lv = O.sfc_sort(I.uniform_leaves(2, 2)[::-1])
    assert list(lv["tree"][:16]) == [0] * 16
    # Z-curve: leaf (2,1) precedes (1,2) at level 2
    k = {(a["ix"], a["iy"]): n for n, a in enumerate(lv[:16])}
    assert k[(0, 0)] < k[(1, 0)] < k[(0, 1)] < k[(1, 1)] < k[(2, 0)]
    assert k[(3, 1)] < k[(0, 2)]


def test_paper_mesh_facts():
    facts = json.load(open(os.path.join(GOLDEN, "paper_mesh_facts.json")))
    for r in facts["patches_at_level"]:
        if r["level"] > 6:
            # count without building the forest
            assert r["trees"] * 4 ** r["level"] == r["patches"]
            continue
        lv = O.sfc_sort(I.uniform_leaves(r["trees"], r["level"]))
        trees = I.brick(r["trees"], 1)[0]
        mesh = O.Mesh(trees, lv, 8)
        assert len(mesh) == r["patches"]
    for r in facts["effective_resolution"]:
        lv = I.uniform_leaves(1, r["level"])
        x, _ = I.cell_centres(lv, r["m"])
        assert len(np.unique(x)) == r["cells_per_side"]


def test_invalid_forests_rejected():
    trees, _ = I.walled_square()
    lv = O.sfc_sort(I.uniform_leaves(1, 2))
    with pytest.raises(ValueError):
        O.Mesh(trees, lv[:-1], 8)                  # hole
    with pytest.raises(ValueError):
        O.Mesh(trees, lv[::-1].copy(), 8)          # not SFC-sorted
    with pytest.raises(ValueError):
        O.Mesh(trees, lv, 6)                       # m not a power of two
    bad = trees.copy()
    bad["bc"][0, 0] = 0
    bad["nbr_tree"][0, 0] = 0
    bad["nbr_face"][0, 0] = 1                      # one-sided connection
    with pytest.raises(ValueError):
        O.Mesh(bad, lv, 8)


DOMAINS = ["walled", "periodic", "brick_oriented", "sphere"]


def _domain(name):
    if name == "walled":
        t, pl = I.walled_square()
        return t, pl, 1, None
    if name == "periodic":
        t, pl = I.periodic_square()
        return t, pl, 1, (1.0, 1.0)
    if name == "brick_oriented":
        t, pl = I.brick(2, 2, orient_codes=[0, 1, 6, 3])
        return t, pl, 4, None
    return I.cubed_sphere(), None, 6, None


def _boxes(name, leaves, pl):
    if name == "sphere":
        return H.leaf_boxes_cube(leaves)
    return H.leaf_boxes_plane(leaves, pl)


@pytest.mark.parametrize("name", DOMAINS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_balance_bruteforce(name, seed):
    trees, pl, nt, period = _domain(name)
    raw = I.random_leaves(seed, nt, 1, 6, 40 if nt > 1 else 60)
    out = O.balance(trees, raw)
    lo, hi = _boxes(name, out, pl)
    assert H.is_balanced_bruteforce(out, lo, hi, period)
    assert H.covers(raw, out)
    mesh = O.Mesh(trees, out, 8)
    assert mesh.balanced()
    # minimality: undoing any refinement that balance introduced breaks
    # balance (or the refinement of the input)
    rawset = {tuple(int(v) for v in a) for a in raw}
    keys = [tuple(int(v) for v in a) for a in out]
    idx = {k: n for n, k in enumerate(keys)}
    checked = 0
    for k in keys:
        t, l, x, y = k
        if l == 0 or (x & 1) or (y & 1) or k in rawset:
            continue
        fam = [(t, l, x + (c & 1), y + (c >> 1)) for c in range(4)]
        if not all(f in idx for f in fam):
            continue
        if any(f in rawset for f in fam):
            continue
        parent = np.array([(t, l - 1, x >> 1, y >> 1)], dtype=I.LEAF_DTYPE)
        if not H.covers(raw, parent):
            continue
        keep = np.array([a for a in keys if a not in fam], dtype=I.LEAF_DTYPE)
        cand = np.concatenate([keep, parent])
        lo2, hi2 = _boxes(name, cand, pl)
        assert not H.is_balanced_bruteforce(cand, lo2, hi2, period)
        checked += 1
        if checked >= 12:
            break


def test_unbalanced_detected():
    trees, _ = I.walled_square()
    lv = I.uniform_leaves(1, 1)
    # refine the first child twice: level-3 leaves touch level-1 leaves
    lv = [tuple(a) for a in lv.tolist()]
    lv.remove((0, 1, 0, 0))
    for c in range(4):
        lv.append((0, 2, c & 1, c >> 1))
    lv.remove((0, 2, 1, 1))
    for c in range(4):
        lv.append((0, 3, 2 + (c & 1), 2 + (c >> 1)))
    lv = O.sfc_sort(np.array(lv, dtype=I.LEAF_DTYPE))
    mesh = O.Mesh(trees, lv, 8)
    assert not mesh.balanced()
    out = O.balance(trees, lv)
    assert O.Mesh(trees, out, 8).balanced()
    assert len(out) > len(lv)
