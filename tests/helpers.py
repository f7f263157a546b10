"""Shared helpers for the tests: brute-force geometry checks written
independently of both the oracle and the HIP library."""
from __future__ import annotations

import numpy as np

from paper_1308_1472_amd import inputs as I


def leaf_boxes_plane(leaves, placement):
    """Closed boxes [x0,x1]x[y0,y1] of leaves in the global plane."""
    h = np.ldexp(1.0, -leaves["level"].astype(np.int64))
    x0, y0 = leaves["ix"] * h, leaves["iy"] * h
    cs = []
    for dx, dy in ((0, 0), (1, 0), (0, 1), (1, 1)):
        gx, gy = placement.to_global(leaves["tree"], x0 + dx * h, y0 + dy * h)
        cs.append(np.stack([gx, gy], axis=1))
    cs = np.stack(cs, axis=1)
    return cs.min(axis=1), cs.max(axis=1)


def leaf_boxes_cube(leaves):
    """Closed 3D boxes of leaves drawn on the surface of the cube [-1,1]^3."""
    h = np.ldexp(1.0, -leaves["level"].astype(np.int64))
    out_lo, out_hi = [], []
    for k, a in enumerate(leaves):
        c, u, v = (np.array(w, float) for w in I.CUBE_FACES[a["tree"]])
        pts = []
        for dx, dy in ((0, 0), (1, 0), (0, 1), (1, 1)):
            x = (a["ix"] + dx) * h[k]
            y = (a["iy"] + dy) * h[k]
            pts.append(c + (2 * x - 1) * u + (2 * y - 1) * v)
        pts = np.array(pts)
        out_lo.append(pts.min(axis=0))
        out_hi.append(pts.max(axis=0))
    return np.array(out_lo), np.array(out_hi)


def touching_pairs(lo, hi, period=None, tol=1e-12):
    """Index pairs (a < b) of closed boxes that intersect; `period` wraps
    the plane (periodic square)."""
    n = len(lo)
    pairs = set()
    shifts = [np.zeros(lo.shape[1])]
    if period is not None:
        shifts = []
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                shifts.append(np.array([sx * period[0], sy * period[1]]))
    for s in shifts:
        ok = np.ones((n, n), bool)
        for d in range(lo.shape[1]):
            ok &= (lo[:, None, d] <= hi[None, :, d] + s[d] + tol)
            ok &= (lo[None, :, d] + s[d] <= hi[:, None, d] + tol)
        a, b = np.nonzero(ok)
        for x, y in zip(a.tolist(), b.tolist()):
            if x < y:
                pairs.add((x, y))
            elif y < x:
                pairs.add((y, x))
    return pairs


def is_balanced_bruteforce(leaves, lo, hi, period=None) -> bool:
    lev = leaves["level"]
    for a, b in touching_pairs(lo, hi, period):
        if abs(int(lev[a]) - int(lev[b])) > 1:
            return False
    return True


def covers(coarse, fine) -> bool:
    """Every fine leaf lies inside (or equals) some coarse leaf."""
    cs = {(int(a["tree"]), int(a["level"]), int(a["ix"]), int(a["iy"]))
          for a in coarse}
    for a in fine:
        t, l, x, y = (int(v) for v in a)
        found = False
        while l >= 0:
            if (t, l, x, y) in cs:
                found = True
                break
            l, x, y = l - 1, x >> 1, y >> 1
        if not found:
            return False
    return True
