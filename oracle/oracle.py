"""ctypes front end of the CPU FP64 oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product path.  The C sources next
to this file state what is computed and where the paper says so.

State arrays handed to the oracle are "framed": (P, meqn, m+4, m+4) indexed
[p, k, j+1, i+1] for cells i, j in -1..m+2; the interior is
[..., 2:m+2, 2:m+2].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "liboracle.so")

LEAF_DTYPE = np.dtype([("tree", "<i4"), ("level", "<i4"), ("ix", "<i4"),
                       ("iy", "<i4")])
TREE_DTYPE = np.dtype([("nbr_tree", "<i4", (4,)), ("nbr_face", "<i4", (4,)),
                       ("orient", "<i4", (4,)), ("bc", "<i4", (4,))])

ADVECTION, SHALLOW, SPHERE, SWIRL, ROTATION = 0, 1, 2, 3, 4
S = 30
SIDE = 1 << S


class Params(C.Structure):
    _fields_ = [("m", C.c_int32), ("meqn", C.c_int32), ("physics", C.c_int32),
                ("limiter", C.c_int32), ("transverse", C.c_int32),
                ("pad", C.c_int32), ("g", C.c_double), ("ax", C.c_double),
                ("ay", C.c_double), ("period", C.c_double), ("time", C.c_double),
                ("axis", C.c_double * 3)]


def build(force: bool = False) -> str:
    """Compile the oracle with make (gcc)."""
    if force or not os.path.exists(LIB_PATH):
        subprocess.run(["make", "-B" if force else "-s", "-C", HERE],
                       check=True, capture_output=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.fco_sfc_sort.argtypes = [i64, vp]
        L.fco_mesh_new.argtypes = [i32, vp, i64, vp, i32, i32]
        L.fco_mesh_new.restype = vp
        L.fco_mesh_free.argtypes = [vp]
        L.fco_is_balanced.argtypes = [vp]
        L.fco_balance.argtypes = [i32, vp, i64, vp, i64, vp, vp]
        L.fco_locate_leaf.argtypes = [vp, i32, i64, i64, vp]
        L.fco_ghost_fill.argtypes = [vp, vp, vp, vp]
        L.fco_step.argtypes = [vp, vp, vp, vp, dp, i32, vp]
        L.fco_sums.argtypes = [vp, vp, vp, vp]
        L.fco_tags.argtypes = [vp, vp, vp, i32, dp, i32, i32, vp]
        L.fco_tag_values.argtypes = [vp, vp, vp, i32, vp, vp]
        L.fco_regrid.argtypes = [vp, vp, i32, i32, i64, vp, vp]
        L.fco_transfer.argtypes = [vp, vp, vp, vp, vp]
        L.fco_phi.argtypes = [i32, dp]
        L.fco_phi.restype = dp
        L.fco_swirl_psi.argtypes = [vp, dp, dp, dp]
        L.fco_swirl_psi.restype = dp
        L.fco_swirl_edge.argtypes = [vp, i32, dp, dp, dp, dp]
        L.fco_swirl_edge.restype = dp
        L.fco_riemann.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.fco_tsplit.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.fco_tsplit_sphere.argtypes = [vp, vp, vp, vp, vp, vp, i32]
        L.fco_features.argtypes = [vp, vp, vp, vp]
        L.fco_bf16.argtypes = [dp]
        L.fco_bf16.restype = dp
        L.fco_mlp.argtypes = [vp, vp, i64, vp, vp, vp, dp, i32, vp, vp]
        L.fco_mlp.restype = dp
        L.fco_adam.argtypes = [i64, vp, vp, vp, vp, i32, dp, dp, dp, dp]
        L.fco_learned_tags.argtypes = [i64, vp, vp, dp, vp]
        L.fco_dilate_tags.argtypes = [vp, vp, i32, vp]
        L.fco_sphere_kappa.argtypes = [vp, i64, i32, i32]
        L.fco_sphere_kappa.restype = dp
        L.fco_sphere_edge.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp]
        L.fco_sphere_centre.argtypes = [vp, i64, i32, i32, vp]
        L.fco_rotation_edge.argtypes = [vp, vp, i64, i32, i32, i32]
        L.fco_rotation_edge.restype = dp
        L.fco_rp_sphere.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.fco_step_subcycled.argtypes = [vp, vp, vp, vp, dp, vp]
        L.fco_ghost_fill_level.argtypes = [vp, vp, vp, vp, vp, i32]
        L.fco_set_threads.argtypes = [i32]
        L.fco_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    """Threads over whole patches in the ghost fill and the step's patch
    loop (results are the same for any count)."""
    lib().fco_set_threads(int(n))


def threads() -> int:
    return lib().fco_threads()


def params(m, physics=ADVECTION, limiter=4, transverse=2, g=1.0, ax=0.0,
           ay=0.0, period=1.0, time=0.0, axis=(0.0, 0.0, 1.0)):
    """SWIRL: the prescribed swirl flow of period `period`; `time` is the
    time of the state the next step starts from (the caller advances it).
    ROTATION: a rigid rotation of the sphere about `axis`, one turn per
    `period`."""
    meqn = {ADVECTION: 1, SHALLOW: 3, SPHERE: 4, SWIRL: 1, ROTATION: 1}[physics]
    return Params(m, meqn, physics, limiter, transverse, 0, g, ax, ay, period, time,
                  (C.c_double * 3)(*axis))


def sfc_sort(leaves: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE).copy()
    lib().fco_sfc_sort(len(a), _ptr(a))
    return a


def balance(trees, leaves) -> np.ndarray:
    trees = np.ascontiguousarray(trees, dtype=TREE_DTYPE)
    leaves = sfc_sort(leaves)
    cap = max(16, 64 * len(leaves))
    out = np.zeros(cap, dtype=LEAF_DTYPE)
    n = C.c_int64()
    rc = lib().fco_balance(len(trees), _ptr(trees), len(leaves), _ptr(leaves),
                           cap, _ptr(out), C.byref(n))
    if rc != 0:
        raise RuntimeError(f"fco_balance failed ({rc})")
    return out[: n.value].copy()


class Mesh:
    def __init__(self, trees, leaves, m, sphere=False):
        self.trees = np.ascontiguousarray(trees, dtype=TREE_DTYPE)
        self.leaves = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
        self.m = m
        self.sphere = sphere
        self.h = lib().fco_mesh_new(len(self.trees), _ptr(self.trees),
                                    len(self.leaves), _ptr(self.leaves), m,
                                    int(sphere))
        if not self.h:
            raise ValueError("invalid forest (unsorted, overlapping or bad "
                             "connectivity)")

    def __del__(self):
        if getattr(self, "h", None):
            lib().fco_mesh_free(self.h)
            self.h = None

    def __len__(self):
        return len(self.leaves)

    def balanced(self) -> bool:
        return bool(lib().fco_is_balanced(self.h))

    def locate(self, tree, x, y) -> int:
        out = C.c_int64()
        lib().fco_locate_leaf(self.h, tree, x, y, C.byref(out))
        return out.value


def framed(q: np.ndarray, m: int) -> np.ndarray:
    """(P, meqn, m, m) interior -> (P, meqn, m+4, m+4) with NaN ghosts."""
    P, meqn = q.shape[:2]
    f = np.full((P, meqn, m + 4, m + 4), np.nan)
    f[:, :, 2:m + 2, 2:m + 2] = q
    return f


def interior(f: np.ndarray, m: int) -> np.ndarray:
    return np.ascontiguousarray(f[:, :, 2:m + 2, 2:m + 2])


def ghost_fill(mesh: Mesh, par: Params, qf: np.ndarray) -> int:
    """Fill the ghost frame of qf in place; returns the interpolation
    nesting depth seen."""
    assert qf.dtype == np.float64 and qf.flags.c_contiguous
    depth = C.c_int32()
    rc = lib().fco_ghost_fill(mesh.h, C.byref(par), _ptr(qf), C.byref(depth))
    if rc != 0:
        raise RuntimeError(f"fco_ghost_fill failed ({rc})")
    return depth.value


def step(mesh: Mesh, par: Params, qf: np.ndarray, dt: float, reflux=True):
    """One step from a ghost-filled frame; returns (new frame, nu_max)."""
    qn = np.array(qf, copy=True)
    numax = C.c_double()
    rc = lib().fco_step(mesh.h, C.byref(par), _ptr(qf), _ptr(qn), dt,
                        int(reflux), C.byref(numax))
    if rc != 0:
        raise RuntimeError(f"fco_step failed ({rc})")
    return qn, numax.value


def step_subcycled(mesh: Mesh, par: Params, qf: np.ndarray, dt: float):
    """One sub-cycled step of the coarsest level (level l steps with
    dt 2^-l, dt the step of a level-0 patch) from a framed state (ghosts
    are filled inside); returns (new frame, largest Courant number)."""
    assert qf.dtype == np.float64 and qf.flags.c_contiguous
    qn = np.array(qf, copy=True)
    numax = C.c_double()
    rc = lib().fco_step_subcycled(mesh.h, C.byref(par), _ptr(qf), _ptr(qn), dt,
                                  C.byref(numax))
    if rc != 0:
        raise RuntimeError(f"fco_step_subcycled failed ({rc})")
    return qn, numax.value


def sums(mesh: Mesh, par: Params, qf: np.ndarray) -> np.ndarray:
    out = np.zeros(par.meqn)
    lib().fco_sums(mesh.h, C.byref(par), _ptr(qf), _ptr(out))
    return out


def tags(mesh, par, qf, criterion, threshold, lmin, lmax) -> np.ndarray:
    out = np.zeros(len(mesh), dtype=np.int8)
    rc = lib().fco_tags(mesh.h, C.byref(par), _ptr(qf), criterion, threshold,
                        lmin, lmax, _ptr(out))
    if rc != 0:
        raise RuntimeError(f"fco_tags failed ({rc})")
    return out


def tag_values(mesh, par, qf, criterion):
    """(refine, parent) criterion values per patch (see fco_tag_values)."""
    ref = np.zeros(len(mesh))
    parent = np.zeros(len(mesh))
    rc = lib().fco_tag_values(mesh.h, C.byref(par), _ptr(qf), criterion, _ptr(ref),
                              _ptr(parent))
    if rc != 0:
        raise RuntimeError(f"fco_tag_values failed ({rc})")
    return ref, parent


def regrid(mesh, tg, lmin, lmax) -> np.ndarray:
    tg = np.ascontiguousarray(tg, dtype=np.int8)
    cap = 64 * len(mesh) + 64
    out = np.zeros(cap, dtype=LEAF_DTYPE)
    n = C.c_int64()
    rc = lib().fco_regrid(mesh.h, _ptr(tg), lmin, lmax, cap, _ptr(out),
                          C.byref(n))
    if rc != 0:
        raise RuntimeError(f"fco_regrid failed ({rc})")
    return out[: n.value].copy()


def transfer(old: Mesh, new: Mesh, par, qf_old) -> np.ndarray:
    qn = np.full((len(new), par.meqn, new.m + 4, new.m + 4), np.nan)
    rc = lib().fco_transfer(old.h, new.h, C.byref(par), _ptr(qf_old), _ptr(qn))
    if rc != 0:
        raise RuntimeError(f"fco_transfer failed ({rc})")
    return qn


def phi(limiter: int, theta: float) -> float:
    return lib().fco_phi(limiter, theta)


def riemann(par, direction, ql, qr):
    ql = np.ascontiguousarray(ql, dtype=np.float64)
    qr = np.ascontiguousarray(qr, dtype=np.float64)
    W = np.zeros((3, par.meqn))
    s = np.zeros(3)
    am = np.zeros(par.meqn)
    ap = np.zeros(par.meqn)
    nw = lib().fco_riemann(C.byref(par), direction, _ptr(ql), _ptr(qr), _ptr(W),
                           _ptr(s), _ptr(am), _ptr(ap))
    if nw < 0:
        raise RuntimeError("riemann failed")
    return W[:nw], s[:nw], am, ap


def tsplit(par, direction, ql, qr, psi):
    """(B-psi, B+psi): the transverse split of a fluctuation psi from the
    edge of the given direction with states ql, qr."""
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (ql, qr, psi)]
    bm = np.zeros(par.meqn)
    bp = np.zeros(par.meqn)
    if lib().fco_tsplit(C.byref(par), direction, _ptr(a[0]), _ptr(a[1]), _ptr(a[2]),
                        _ptr(bm), _ptr(bp)) != 0:
        raise RuntimeError("tsplit failed")
    return bm, bp


def swirl_psi(par, x, y, t) -> float:
    """The swirl stream function (SWIRL) at tree coordinates (x, y), time t."""
    return lib().fco_swirl_psi(C.byref(par), x, y, t)


def swirl_edge(par, direction, a, b0, b1, t) -> float:
    """Normal velocity of the `direction` edge at coordinate a spanning
    [b0, b1] in the other coordinate (SWIRL)."""
    return lib().fco_swirl_edge(C.byref(par), direction, a, b0, b1, t)


# -------------------------------------------------------------------------
# a plain driver: ghost fill + step, fixed or CFL-controlled dt, regrid
# -------------------------------------------------------------------------
def advance(mesh, par, q, dt, reflux=True):
    """q: interior (P, meqn, m, m) -> (new interior, nu_max)."""
    f = framed(q, mesh.m)
    ghost_fill(mesh, par, f)
    fn, nu = step(mesh, par, f, dt, reflux)
    return interior(fn, mesh.m), nu


def advance_subcycled(mesh, par, q, dt):
    """q: interior -> (interior after one sub-cycled step of the coarsest
    level, level l stepping with dt 2^-l; nu_max over all its steps)."""
    fn, nu = step_subcycled(mesh, par, framed(q, mesh.m), dt)
    return interior(fn, mesh.m), nu


# -------------------------------------------------------------------------
# learned tagging (an extension of the paper's criterion tagging)
# -------------------------------------------------------------------------
MLP_IN, MLP_HID, MLP_OUT = 16, 64, 3
MLP_PARAMS = MLP_IN * MLP_HID + MLP_HID + MLP_HID * MLP_HID + MLP_HID + \
    MLP_HID * MLP_OUT + MLP_OUT


def features(mesh, par, qf) -> np.ndarray:
    """(P, 16) per-patch statistics from a ghost-filled frame."""
    out = np.zeros((len(mesh), MLP_IN))
    lib().fco_features(mesh.h, C.byref(par), _ptr(qf), _ptr(out))
    return out


def bf16(x) -> np.ndarray:
    f = lib().fco_bf16
    return np.vectorize(f, otypes=[np.float64])(np.asarray(x, np.float64))


def mlp(params, norm, x, y=None, cw=None, scale=1.0, round_bf16=True,
        want_grad=True):
    """Returns (loss, logits (M, 3), grad (5443,) or None)."""
    P = np.ascontiguousarray(params, np.float64)
    nm = np.ascontiguousarray(norm, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    M = len(x)
    assert P.size == MLP_PARAMS and nm.size == 2 * MLP_IN and x.shape[1] == MLP_IN
    logits = np.zeros((M, MLP_OUT))
    grad = np.zeros(MLP_PARAMS) if (want_grad and y is not None) else None
    yy = None if y is None else np.ascontiguousarray(y, np.int32)
    cw = np.ones(MLP_OUT) if cw is None else np.ascontiguousarray(cw, np.float64)
    loss = lib().fco_mlp(_ptr(P), _ptr(nm), M, _ptr(x),
                         None if yy is None else _ptr(yy), _ptr(cw), scale,
                         int(round_bf16), _ptr(logits),
                         None if grad is None else _ptr(grad))
    return loss, logits, grad


def adam(params, grad, m1, m2, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place on float64 arrays."""
    lib().fco_adam(params.size, _ptr(params), _ptr(np.ascontiguousarray(grad)),
                   _ptr(m1), _ptr(m2), t, lr, beta1, beta2, eps)


def learned_tags(logits, plain, confidence=0.6) -> np.ndarray:
    z = np.ascontiguousarray(logits, np.float64)
    pl = np.ascontiguousarray(plain, np.int8)
    out = np.zeros(len(pl), np.int8)
    lib().fco_learned_tags(len(pl), _ptr(z), _ptr(pl), confidence, _ptr(out))
    return out


def dilate_tags(mesh, tg, lmax) -> np.ndarray:
    tg = np.ascontiguousarray(tg, np.int8)
    out = np.zeros_like(tg)
    lib().fco_dilate_tags(mesh.h, _ptr(tg), lmax, _ptr(out))
    return out


# -------------------------------------------------------------------------
# cubed sphere geometry and solver pieces
# -------------------------------------------------------------------------
class EdgeGeom(C.Structure):
    _fields_ = [("gamma", C.c_double), ("n", C.c_double * 3), ("t", C.c_double * 3),
                ("vel", C.c_double)]


def sphere_kappa(mesh, p, i, j) -> float:
    return lib().fco_sphere_kappa(mesh.h, p, i, j)


def sphere_edge(mesh, p, direction, i, j):
    """(gamma, n, t) of the low-side edge of frame cell (i, j)."""
    g = C.c_double()
    n = np.zeros(3)
    t = np.zeros(3)
    lib().fco_sphere_edge(mesh.h, p, direction, i, j, C.byref(g), _ptr(n), _ptr(t))
    return g.value, n, t


def rotation_edge(mesh, par, p, direction, i, j) -> float:
    """ROTATION: flux of the rotation through the low-side edge of frame
    cell (i, j) over the computational cell size, towards higher index."""
    return lib().fco_rotation_edge(mesh.h, C.byref(par), p, direction, i, j)


def sphere_centre(mesh, p, i, j) -> np.ndarray:
    r = np.zeros(3)
    lib().fco_sphere_centre(mesh.h, p, i, j, _ptr(r))
    return r


def tsplit_sphere(par, gamma, n, t, ql, qr, psi, up):
    """Up-going (up = 1) or down-going (up = 0) part of the fluctuation psi
    split with the frame (gamma, n, t) of a transverse edge and the Roe
    averages of the normal edge's states ql, qr."""
    e = EdgeGeom(gamma, (C.c_double * 3)(*n), (C.c_double * 3)(*t))
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (ql, qr, psi)]
    out = np.zeros(4)
    if lib().fco_tsplit_sphere(C.byref(par), _ptr(a[0]), _ptr(a[1]), C.byref(e),
                               _ptr(a[2]), _ptr(out), int(up)) != 0:
        raise RuntimeError("tsplit failed")
    return out


def riemann_sphere(par, gamma, n, t, ql, qr):
    e = EdgeGeom(gamma, (C.c_double * 3)(*n), (C.c_double * 3)(*t))
    ql = np.ascontiguousarray(ql, dtype=np.float64)
    qr = np.ascontiguousarray(qr, dtype=np.float64)
    W = np.zeros((3, 4))
    s = np.zeros(3)
    am = np.zeros(4)
    ap = np.zeros(4)
    fl = C.c_double()
    nw = lib().fco_rp_sphere(C.byref(par), C.byref(e), _ptr(ql), _ptr(qr), _ptr(W),
                             _ptr(s), _ptr(am), _ptr(ap), C.byref(fl))
    if nw < 0:
        raise RuntimeError("riemann failed")
    return W, s, am, ap, fl.value
