"""Seeded synthetic inputs: forests, tree connectivities and initial data.

This module generates inputs only.  It holds none of the method's
arithmetic: no ghost filling, no Riemann solves, no balancing, no SFC
ordering, no tagging.  Leaf arrays it returns are in generation order and
may be unbalanced; each side (the HIP library and the CPU oracle) sorts and
balances them with its own code.  Both sides receive identical arrays from
here.

Conventions (shared with the method's description, arXiv 1308.1472 Sec. 2):
every tree is the reference square [0,1]^2; a leaf (tree, level, ix, iy)
covers [ix, ix+1] 2^-level x [iy, iy+1] 2^-level of its tree and houses an
m x m patch; cell (i, j), i, j = 1..m, has its centre at
((ix + (i - 1/2)/m) 2^-level, (iy + (j - 1/2)/m) 2^-level).

Interior state arrays have shape (P, meqn, m, m) indexed [p, k, j-1, i-1].
"""
from __future__ import annotations

import math

import numpy as np

LEAF_DTYPE = np.dtype([("tree", "<i4"), ("level", "<i4"), ("ix", "<i4"),
                       ("iy", "<i4")])
TREE_DTYPE = np.dtype([("nbr_tree", "<i4", (4,)), ("nbr_face", "<i4", (4,)),
                       ("orient", "<i4", (4,)), ("bc", "<i4", (4,))])

BC_CONNECTED, BC_WALL, BC_EXTRAP = 0, 1, 2


# --------------------------------------------------------------------------
# tree placements and the connectivities they induce
# --------------------------------------------------------------------------
class Placement:
    """Affine placement of each tree's reference square in the plane:
    global = origin + A @ (xi, eta) with A a signed permutation matrix.
    Used to build a brick connectivity and to evaluate initial data in one
    global coordinate system."""

    def __init__(self, origins, mats):
        self.origins = np.asarray(origins, dtype=np.float64)
        self.mats = np.asarray(mats, dtype=np.float64)

    @property
    def ntrees(self):
        return len(self.origins)

    def to_global(self, tree, xi, eta):
        A = self.mats[tree]
        o = self.origins[tree]
        gx = o[..., 0] + A[..., 0, 0] * xi + A[..., 0, 1] * eta
        gy = o[..., 1] + A[..., 1, 0] * xi + A[..., 1, 1] * eta
        return gx, gy


_ORIENTS = [
    ((1, 0), (0, 1)), ((0, -1), (1, 0)), ((-1, 0), (0, -1)), ((0, 1), (-1, 0)),
    ((-1, 0), (0, 1)), ((1, 0), (0, -1)), ((0, 1), (1, 0)), ((0, -1), (-1, 0)),
]


def brick_placement(nx: int, ny: int, orient_codes=None) -> Placement:
    """nx x ny unit squares; tree t = tx + nx*ty sits at (tx, ty).  Each
    tree's reference square may be rotated/reflected (codes 0..7)."""
    origins, mats = [], []
    for ty in range(ny):
        for tx in range(nx):
            t = tx + nx * ty
            code = 0 if orient_codes is None else int(orient_codes[t])
            A = np.array(_ORIENTS[code], dtype=np.float64)
            # choose the origin so that the image of [0,1]^2 is the cell
            corners = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], float) @ A.T
            o = np.array([tx, ty], float) - corners.min(axis=0)
            origins.append(o)
            mats.append(A)
    return Placement(origins, mats)


def _face_segment(pl: Placement, t: int, f: int):
    a, s = f // 2, f % 2
    if a == 0:
        p0, p1 = (s, 0.0), (s, 1.0)
    else:
        p0, p1 = (0.0, s), (1.0, s)
    g0 = np.array(pl.to_global(t, *p0))
    g1 = np.array(pl.to_global(t, *p1))
    return g0, g1


def connectivity_from_placement(pl: Placement, periodic=(False, False),
                                extent=None, bc=BC_WALL) -> np.ndarray:
    """Glue trees whose faces coincide (optionally modulo a periodic box of
    size `extent`).  Unmatched faces get the physical boundary `bc`."""
    n = pl.ntrees
    if extent is None:
        allc = []
        for t in range(n):
            for f in range(4):
                g0, g1 = _face_segment(pl, t, f)
                allc += [g0, g1]
        allc = np.array(allc)
        extent = allc.max(axis=0) - allc.min(axis=0)
    trees = np.zeros(n, dtype=TREE_DTYPE)
    trees["nbr_tree"] = -1
    trees["nbr_face"] = -1
    trees["bc"] = bc

    def canon(p):
        q = np.array(p, float)
        for d in range(2):
            if periodic[d]:
                q[d] = q[d] % extent[d]
        return tuple(np.round(q, 9))

    for t in range(n):
        for f in range(4):
            a0, a1 = _face_segment(pl, t, f)
            ka0, ka1 = canon(a0), canon(a1)
            for t2 in range(n):
                for f2 in range(4):
                    if t2 == t and f2 == f:
                        continue
                    b0, b1 = _face_segment(pl, t2, f2)
                    kb0, kb1 = canon(b0), canon(b1)
                    if (ka0, ka1) == (kb0, kb1):
                        o = 0
                    elif (ka0, ka1) == (kb1, kb0):
                        o = 1
                    else:
                        continue
                    # faces must bound the two trees from opposite sides
                    trees["nbr_tree"][t, f] = t2
                    trees["nbr_face"][t, f] = f2
                    trees["orient"][t, f] = o
                    trees["bc"][t, f] = BC_CONNECTED
    return trees


def periodic_square() -> tuple[np.ndarray, Placement]:
    pl = brick_placement(1, 1)
    trees = np.zeros(1, dtype=TREE_DTYPE)
    trees["nbr_tree"] = 0
    trees["nbr_face"] = [[1, 0, 3, 2]]
    trees["orient"] = 0
    trees["bc"] = BC_CONNECTED
    return trees, pl


def walled_square(bc=BC_WALL) -> tuple[np.ndarray, Placement]:
    pl = brick_placement(1, 1)
    trees = np.zeros(1, dtype=TREE_DTYPE)
    trees["nbr_tree"] = -1
    trees["nbr_face"] = -1
    trees["bc"] = bc
    return trees, pl


def brick(nx, ny, orient_codes=None, periodic=(False, False), bc=BC_WALL):
    pl = brick_placement(nx, ny, orient_codes)
    trees = connectivity_from_placement(pl, periodic=periodic,
                                        extent=np.array([nx, ny], float), bc=bc)
    return trees, pl


# --------------------------------------------------------------------------
# cubed sphere: six trees, gnomonic equiangular map
# --------------------------------------------------------------------------
# Face k of the cube is spanned by (centre c, axis u, axis v); a reference
# point (xi, eta) maps to the cube point c + tan(a) u + tan(b) v with
# a, b = pi/2 (xi - 1/2), pi/2 (eta - 1/2), then to the unit sphere.
CUBE_FACES = [
    ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((0, 1, 0), (-1, 0, 0), (0, 0, 1)),
    ((-1, 0, 0), (0, -1, 0), (0, 0, 1)),
    ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
    ((0, 0, 1), (0, 1, 0), (-1, 0, 0)),
    ((0, 0, -1), (0, 1, 0), (1, 0, 0)),
]


def sphere_point(tree, xi, eta):
    c, u, v = (np.array(w, float) for w in CUBE_FACES[tree])
    ta = np.tan(0.5 * np.pi * (np.asarray(xi) - 0.5))
    tb = np.tan(0.5 * np.pi * (np.asarray(eta) - 0.5))
    p = (c[:, None] * np.ones_like(ta).ravel()[None, :]
         + u[:, None] * ta.ravel()[None, :] + v[:, None] * tb.ravel()[None, :])
    p = p / np.linalg.norm(p, axis=0)[None, :]
    return p.reshape((3,) + np.shape(ta))


def cubed_sphere() -> np.ndarray:
    """Connectivity of the six cube faces, found by matching face edges of
    the cube (shared edges have identical end points)."""
    def edge(t, f):
        a, s = f // 2, f % 2
        if a == 0:
            e0, e1 = (s, 0.0), (s, 1.0)
        else:
            e0, e1 = (0.0, s), (1.0, s)
        c, u, v = (np.array(w, float) for w in CUBE_FACES[t])
        def corner(x, y):
            return tuple(np.round(c + (2 * x - 1) * u + (2 * y - 1) * v, 9))
        return corner(*e0), corner(*e1)

    trees = np.zeros(6, dtype=TREE_DTYPE)
    trees["bc"] = BC_CONNECTED
    for t in range(6):
        for f in range(4):
            a0, a1 = edge(t, f)
            found = False
            for t2 in range(6):
                if t2 == t:
                    continue
                for f2 in range(4):
                    b0, b1 = edge(t2, f2)
                    if (a0, a1) == (b0, b1):
                        o = 0
                    elif (a0, a1) == (b1, b0):
                        o = 1
                    else:
                        continue
                    trees["nbr_tree"][t, f] = t2
                    trees["nbr_face"][t, f] = f2
                    trees["orient"][t, f] = o
                    found = True
            assert found
    return trees


# --------------------------------------------------------------------------
# leaves
# --------------------------------------------------------------------------
def uniform_leaves(ntrees: int, level: int) -> np.ndarray:
    n = 1 << level
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    out = []
    for t in range(ntrees):
        a = np.zeros(n * n, dtype=LEAF_DTYPE)
        a["tree"] = t
        a["level"] = level
        a["ix"] = ix.ravel()
        a["iy"] = iy.ravel()
        out.append(a)
    return np.concatenate(out)


def random_leaves(seed: int, ntrees: int, lmin: int, lmax: int,
                  nsplit: int) -> np.ndarray:
    """Uniform at lmin, then `nsplit` random splits of leaves below lmax.
    Generally NOT 2:1 balanced."""
    rng = np.random.default_rng(seed)
    leaves = [tuple(r) for r in uniform_leaves(ntrees, lmin).tolist()]
    for _ in range(nsplit):
        cand = [k for k, a in enumerate(leaves) if a[1] < lmax]
        if not cand:
            break
        k = cand[int(rng.integers(len(cand)))]
        t, l, x, y = leaves.pop(k)
        for c in range(4):
            leaves.append((t, l + 1, 2 * x + (c & 1), 2 * y + (c >> 1)))
    return np.array(leaves, dtype=LEAF_DTYPE)


def refine_near(ntrees: int, lmin: int, lmax: int, points, placement,
                radius: float) -> np.ndarray:
    """Refine every leaf whose centre is within radius * 2^-level of one of
    the given global points, from lmin to lmax (unbalanced in general)."""
    pts = np.asarray(points, float).reshape(-1, 2)
    leaves = [tuple(r) for r in uniform_leaves(ntrees, lmin).tolist()]
    for _ in range(lmax - lmin):
        nxt = []
        for (t, l, x, y) in leaves:
            h = 2.0 ** -l
            gx, gy = placement.to_global(t, (x + 0.5) * h, (y + 0.5) * h)
            d = np.min(np.hypot(pts[:, 0] - gx, pts[:, 1] - gy))
            if l < lmax and d < radius * h:
                for c in range(4):
                    nxt.append((t, l + 1, 2 * x + (c & 1), 2 * y + (c >> 1)))
            else:
                nxt.append((t, l, x, y))
        leaves = nxt
    return np.array(leaves, dtype=LEAF_DTYPE)


# --------------------------------------------------------------------------
# cell centres and initial data
# --------------------------------------------------------------------------
def cell_centres(leaves: np.ndarray, m: int, placement: Placement | None = None,
                 ghosts: int = 0):
    """Reference (or global, with a placement) coordinates of the cell
    centres, shape (P, m+2g, m+2g) indexed [p, j, i]."""
    idx = (np.arange(-ghosts, m + ghosts) + 0.5) / m
    h = np.ldexp(1.0, -leaves["level"].astype(np.int64))[:, None, None]
    xi = (leaves["ix"][:, None, None] + idx[None, None, :]) * h
    eta = (leaves["iy"][:, None, None] + idx[None, :, None]) * h
    xi, eta = np.broadcast_arrays(xi, eta)
    if placement is None:
        return xi.copy(), eta.copy()
    t = leaves["tree"][:, None, None]
    return placement.to_global(np.broadcast_to(t, xi.shape), xi, eta)


def gaussian(x, y, cx=0.5, cy=0.5, width2=0.01):
    return np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / width2)


def periodic_gaussian(x, y, cx, cy, width2=0.01, images=1):
    out = np.zeros_like(x)
    for sx in range(-images, images + 1):
        for sy in range(-images, images + 1):
            out += gaussian(x, y, cx + sx, cy + sy, width2)
    return out


def dam_break(x, y, cx=0.5, cy=0.5, r=0.25, hin=2.0, hout=1.0):
    """(h, hu, hv) with h = hin inside the disc r^2 > dx^2 + dy^2."""
    inside = (x - cx) ** 2 + (y - cy) ** 2 < r * r
    h = np.where(inside, hin, hout)
    return np.stack([h, np.zeros_like(h), np.zeros_like(h)], axis=1)


def state_from(leaves, m, fn, placement=None, meqn=None):
    """Evaluate fn(x, y) at cell centres -> (P, meqn, m, m)."""
    x, y = cell_centres(leaves, m, placement)
    v = fn(x, y)
    v = np.asarray(v, dtype=np.float64)
    if v.ndim == 3:
        v = v[:, None]
    if meqn is not None:
        assert v.shape[1] == meqn
    return np.ascontiguousarray(v)


# --------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood 2014) for per-forest seeds of batches
# --------------------------------------------------------------------------
class SplitMix64:
    MASK = (1 << 64) - 1

    def __init__(self, seed: int):
        self.state = seed & self.MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def batch_forest_spec(seed: int) -> dict:
    """Description of one forest of a batch of independent forests:
    physics by seed parity, m in {8, 16, 32}, target patch count
    log-uniform in 16..16384, and random initial-data parameters."""
    g = SplitMix64(seed)
    physics = "advection" if seed % 2 == 0 else "shallow"
    m = (8, 16, 32)[g.next_u64() % 3]
    target = int(round(math.exp(math.log(16) + g.uniform() *
                                (math.log(16384) - math.log(16)))))
    spec = {"seed": seed, "physics": physics, "m": m, "target": target}
    cx, cy = 0.3 + 0.4 * g.uniform(), 0.3 + 0.4 * g.uniform()
    if physics == "advection":
        ang = 2 * math.pi * g.uniform()
        rad = math.sqrt(g.uniform())
        spec.update(ax=rad * math.cos(ang), ay=rad * math.sin(ang), cx=cx,
                    cy=cy, width2=0.002 + 0.02 * g.uniform())
    else:
        spec.update(cx=cx, cy=cy, r=0.15 + 0.15 * g.uniform(),
                    hin=1.5 + 1.5 * g.uniform())
    return spec


def batch_forest(seed: int, lmin: int = 2, lmax: int = 8):
    """One forest of a batch: (spec, trees, placement, leaves, initial-data
    function).  Mesh: uniform at lmin, then repeatedly refine the leaves
    closest to the feature (the Gaussian's centre, or the dam's rim) below
    lmax until there are at least spec["target"] leaves (not balanced)."""
    spec = batch_forest_spec(seed)
    if spec["physics"] == "advection":
        trees, pl = periodic_square()
        cx, cy = spec["cx"], spec["cy"]
        def dist(x, y):
            return np.hypot(x - cx, y - cy)
        w2 = spec["width2"]
        fn = lambda x, y: periodic_gaussian(x, y, cx, cy, w2)
    else:
        trees, pl = walled_square()
        cx, cy, r = spec["cx"], spec["cy"], spec["r"]
        def dist(x, y):
            return np.abs(np.hypot(x - cx, y - cy) - r)
        fn = lambda x, y: dam_break(x, y, cx, cy, r, spec["hin"], 1.0)
    leaves = [tuple(a) for a in uniform_leaves(1, lmin).tolist()]
    target = spec["target"]
    while len(leaves) < target:
        arr = np.array(leaves, dtype=LEAF_DTYPE)
        h = np.ldexp(1.0, -arr["level"].astype(np.int64))
        d = dist((arr["ix"] + 0.5) * h, (arr["iy"] + 0.5) * h)
        d = np.where(arr["level"] < lmax, d, np.inf)
        order = np.lexsort((np.arange(len(arr)), d))
        k = max(1, -(-(target - len(leaves)) // 3))
        pick = [int(i) for i in order[:k] if np.isfinite(d[i])]
        if not pick:
            break
        chosen = set(pick)
        nxt = []
        for i, (t, l, x, y) in enumerate(leaves):
            if i in chosen:
                for c in range(4):
                    nxt.append((t, l + 1, 2 * x + (c & 1), 2 * y + (c >> 1)))
            else:
                nxt.append((t, l, x, y))
        leaves = nxt
    return spec, trees, pl, np.array(leaves, dtype=LEAF_DTYPE), fn


def dam_break_spec(seed: int) -> dict:
    """Random radial dam break of the learned-tagging runs: centre in
    [0.3, 0.7]^2, radius in [0.15, 0.3], inner depth in [1.5, 3]."""
    g = SplitMix64(0x5EED_DA4B_0000 + seed)
    return {"centre": (0.3 + 0.4 * g.uniform(), 0.3 + 0.4 * g.uniform()),
            "radius": 0.15 + 0.15 * g.uniform(), "h_in": 1.5 + 1.5 * g.uniform()}


def pillow_sphere() -> np.ndarray:
    """Connectivity of the two-tree (pillow) sphere: tree t's faces 0 and 1
    meet the other tree's faces 0 and 1 with the tangential coordinate
    reversed, its face 2 meets the other's face 3 and its face 3 the other's
    face 2, the same way."""
    trees = np.zeros(2, dtype=TREE_DTYPE)
    trees["bc"] = BC_CONNECTED
    for t in range(2):
        trees["nbr_tree"][t] = 1 - t
        trees["nbr_face"][t] = [0, 1, 3, 2]
        trees["orient"][t] = [1, 1, 0, 0]
    return trees


def pillow_point(tree, xi, eta):
    """The two-tree sphere map: with x = 2 xi - 1, y = 2 eta - 1 and d =
    max(|x|, |y|), the point at polar angle d pi / 2 about the tree's pole
    along the direction (x, y); tree 1 negates the second and third
    components.  Shape (3,) + shape of xi."""
    x = 2.0 * np.asarray(xi, float) - 1.0
    y = 2.0 * np.asarray(eta, float) - 1.0
    d = np.maximum(np.abs(x), np.abs(y))
    rho = np.sqrt(x * x + y * y)
    safe = np.where(rho > 0, rho, 1.0)
    th = 0.5 * np.pi * d
    s = np.where(d >= 1.0, 1.0, np.sin(th))
    c = np.where(d >= 1.0, 0.0, np.cos(th))
    p = np.stack([s * x / safe, s * y / safe, c])
    if tree == 1:
        p[1] = -p[1]
        p[2] = -p[2]
    return p


def sphere_centres(leaves: np.ndarray, m: int, pillow: bool = False) -> np.ndarray:
    """Unit vectors of the mapped cell centres, shape (P, 3, m, m), on the
    cubed sphere or (pillow) the two-tree sphere."""
    xi, eta = cell_centres(leaves, m)
    out = np.empty((len(leaves), 3, m, m))
    for t in range(2 if pillow else 6):
        s = leaves["tree"] == t
        if s.any():
            f = pillow_point if pillow else sphere_point
            out[s] = np.moveaxis(f(t, xi[s], eta[s]), 0, 1)
    return out


def sphere_bumps(leaves, m, n=16, seed=0, amp=0.1, width=30.0):
    """h = 1 + sum of n bumps amp exp(-width d_k^2) around seeded centres
    drawn uniformly on the sphere (d_k the great-circle distance to centre
    k); fluid at rest.  Spreads resolvable gradients over much of the
    sphere, so that a criterion tags enough patches for a large adaptive
    mesh.  (P, 4, m, m)."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(n, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    r = sphere_centres(leaves, m)
    q = np.zeros((len(leaves), 4, m, m))
    q[:, 0] = 1.0
    for k in range(n):
        d = np.arccos(np.clip(np.einsum("pkij,k->pij", r, c[k]), -1.0, 1.0))
        q[:, 0] += amp * np.exp(-width * d * d)
    return q


def sphere_scalar(leaves, m, fn, pillow=False):
    """(P, 1, m, m) scalar state fn(r) at the cell centres, r of shape
    (P, 3, m, m) (unit vectors)."""
    return np.asarray(fn(sphere_centres(leaves, m, pillow)), dtype=np.float64)[:, None]


def sphere_halves(leaves, m, normal=(0.35, -0.5, 0.79), pillow=False):
    """q = 1 on the half of the sphere that `normal` points into, 0 on the
    other: a 0/1 state whose interface (a great circle) is not aligned with
    the trees' edges.  (P, 1, m, m)."""
    w = np.asarray(normal, float) / np.linalg.norm(normal)
    return sphere_scalar(leaves, m,
                         lambda r: (np.einsum("pkij,k->pij", r, w) > 0).astype(np.float64),
                         pillow)


def sphere_bump(leaves, m, lat=0.3, lon=0.5, amp=0.1, width=100.0):
    """h = 1 + amp exp(-width d^2), d the great-circle distance to the
    point (lat, lon); fluid at rest.  (P, 4, m, m): h, hu, hv, hw."""
    c = np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])
    r = sphere_centres(leaves, m)
    d = np.arccos(np.clip(np.einsum("pkij,k->pij", r, c), -1.0, 1.0))
    q = np.zeros((len(leaves), 4, m, m))
    q[:, 0] = 1.0 + amp * np.exp(-width * d * d)
    return q
