"""Python binding of libfcx.so (include/fcx.h): argument marshalling only.

Every numerical step runs in the library's HIP kernels; this module only
checks shapes and dtypes, takes device pointers from torch tensors and the
current HIP stream, and translates error codes into exceptions.  It raises
if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libfcx.so")

LEAF_DTYPE = np.dtype([("tree", "<i4"), ("level", "<i4"), ("ix", "<i4"),
                       ("iy", "<i4")])
TREE_DTYPE = np.dtype([("nbr_tree", "<i4", (4,)), ("nbr_face", "<i4", (4,)),
                       ("orient", "<i4", (4,)), ("bc", "<i4", (4,))])

FCX_ADVECTION, FCX_SHALLOW, FCX_SPHERE, FCX_SWIRL, FCX_ROTATION = 0, 1, 2, 3, 4
GEO_FRAMES = 18          # geometry table frames per patch (fcx_sphere_geometry)
ERRORS = {-1: "FCX_EINVAL", -2: "FCX_EBALANCE", -3: "FCX_ENOMEM",
          -4: "FCX_EHIP", -5: "FCX_ECFL", -6: "FCX_ENEG", -7: "FCX_ESTATE"}

# the symbols include/fcx.h declares
EXPORTS = [
    "fcx_last_error", "fcx_version", "fcx_sfc_sort", "fcx_balance",
    "fcx_regrid_leaves",
    "fcx_create", "fcx_destroy", "fcx_upload_forest", "fcx_num_patches",
    "fcx_state_elems", "fcx_ghost_elems", "fcx_get_leaves", "fcx_patch_table",
    "fcx_ghost_fill",
    "fcx_patch_step", "fcx_fused_step", "fcx_reflux", "fcx_next_dt",
    "fcx_conservation_sums", "fcx_regrid_tags", "fcx_regrid_apply",
    "fcx_regrid_transfer", "fcx_batch_create", "fcx_batch_destroy",
    "fcx_batch_state_elems", "fcx_batch_state_offset", "fcx_batch_num_patches",
    "fcx_batch_set_tuning", "fcx_batch_step", "fcx_batch_capture",
    "fcx_batch_replay", "fcx_batch_sums", "fcx_features", "fcx_mlp_forward",
    "fcx_mlp_backward", "fcx_adam_step", "fcx_learned_tags", "fcx_dilate_tags",
    "fcx_sphere_geometry", "fcx_advance", "fcx_regrid", "fcx_run",
    "fcx_step_stats", "fcx_batch_step_stats", "fcx_conservation_sums_noalloc",
    "fcx_advance_subcycled", "fcx_sim_time", "fcx_batch_class_items",
]

MLP_INPUTS, MLP_HIDDEN, MLP_CLASSES, MLP_PARAMS = 16, 64, 3, 5443


class FcxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("m", C.c_int32), ("precision", C.c_int32),
                ("physics", C.c_int32), ("limiter", C.c_int32),
                ("transverse", C.c_int32), ("tile", C.c_int32),
                ("threads", C.c_int32), ("redo", C.c_int32),
                ("g", C.c_double), ("ax", C.c_double), ("ay", C.c_double),
                ("cfl_desired", C.c_double), ("cfl_max", C.c_double),
                ("period", C.c_double), ("axis", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1308_1472_amd.build` (there is no fallback)")
        # torch ships its own HIP runtime under the same soname; importing it
        # first makes the library bind to that one runtime instead of loading
        # a second copy from /opt/rocm into the process
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.fcx_last_error.restype = C.c_char_p
        L.fcx_version.restype = i32
        L.fcx_sfc_sort.argtypes = [i64, vp]
        L.fcx_balance.argtypes = [i32, vp, i64, vp, i64, vp, vp]
        L.fcx_regrid_leaves.argtypes = [i32, vp, i64, vp, vp, i32, i32, i64, vp, vp]
        L.fcx_create.argtypes = [vp, i32, vp, vp]
        L.fcx_destroy.argtypes = [vp]
        L.fcx_upload_forest.argtypes = [vp, i64, vp]
        for f in ("fcx_num_patches", "fcx_state_elems", "fcx_ghost_elems"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = i64
        L.fcx_get_leaves.argtypes = [vp, i64, vp]
        L.fcx_patch_table.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.fcx_ghost_fill.argtypes = [vp, vp, vp, vp]
        L.fcx_patch_step.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fcx_fused_step.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fcx_reflux.argtypes = [vp, vp, vp, vp, vp]
        L.fcx_next_dt.argtypes = [vp, vp, vp, vp, vp]
        L.fcx_conservation_sums.argtypes = [vp, vp, vp, vp]
        L.fcx_regrid_tags.argtypes = [vp, vp, vp, i32, dp, i32, i32, vp, vp]
        L.fcx_regrid_apply.argtypes = [vp, vp, i32, i32, vp, vp]
        L.fcx_regrid_transfer.argtypes = [vp, vp, vp, vp, vp]
        L.fcx_batch_create.argtypes = [i32, vp, vp]
        L.fcx_batch_destroy.argtypes = [vp]
        for f in ("fcx_batch_state_elems", "fcx_batch_num_patches"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = i64
        L.fcx_batch_state_offset.argtypes = [vp, i32]
        L.fcx_batch_state_offset.restype = i64
        L.fcx_batch_set_tuning.argtypes = [vp, i32, i32, i32, i32]
        L.fcx_batch_step.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fcx_batch_capture.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.fcx_batch_replay.argtypes = [vp, vp]
        L.fcx_batch_sums.argtypes = [vp, vp, vp, vp]
        fl = C.c_float
        L.fcx_features.argtypes = [vp, vp, vp, vp, vp]
        L.fcx_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
        L.fcx_mlp_backward.argtypes = [vp, vp, i64, vp, vp, vp, fl, vp, vp, vp]
        L.fcx_adam_step.argtypes = [i64, vp, vp, vp, vp, i32, fl, fl, fl, fl, vp]
        L.fcx_learned_tags.argtypes = [i64, vp, vp, fl, vp, vp]
        L.fcx_dilate_tags.argtypes = [vp, vp, i32, vp, vp]
        L.fcx_sphere_geometry.argtypes = [vp, vp, vp]
        L.fcx_advance.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fcx_regrid.argtypes = [vp, vp, vp, i32, dp, i32, i32, vp, vp, vp]
        L.fcx_step_stats.argtypes = [vp, vp]
        L.fcx_conservation_sums_noalloc.argtypes = [vp, vp, vp, vp]
        L.fcx_advance_subcycled.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.fcx_sim_time.argtypes = [vp, vp]
        L.fcx_batch_step_stats.argtypes = [vp, vp]
        L.fcx_batch_class_items.argtypes = [vp, vp, vp]
        L.fcx_run.argtypes = [vp, i32, vp, vp, i64, vp, i64, i32, i32, i32, i32, dp, i32,
                              i32, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise FcxError(rc, lib().fcx_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def sfc_sort(leaves) -> np.ndarray:
    a = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE).copy()
    _check(lib().fcx_sfc_sort(len(a), _np_ptr(a)))
    return a


def balance(trees, leaves) -> np.ndarray:
    trees = np.ascontiguousarray(trees, dtype=TREE_DTYPE)
    leaves = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
    n = C.c_int64()
    cap = 16 * len(leaves) + 64
    while True:
        out = np.zeros(cap, dtype=LEAF_DTYPE)
        rc = lib().fcx_balance(len(trees), _np_ptr(trees), len(leaves),
                               _np_ptr(leaves), cap, _np_ptr(out), C.byref(n))
        if rc == -1 and n.value > cap:
            cap = n.value
            continue
        _check(rc)
        return out[: n.value].copy()


def regrid_leaves(trees, leaves, tags, lmin, lmax) -> np.ndarray:
    trees = np.ascontiguousarray(trees, dtype=TREE_DTYPE)
    leaves = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
    tags = np.ascontiguousarray(tags, dtype=np.int8)
    if len(tags) != len(leaves):
        raise ValueError("one tag per leaf expected")
    n = C.c_int64()
    cap = 16 * len(leaves) + 64
    while True:
        out = np.zeros(cap, dtype=LEAF_DTYPE)
        rc = lib().fcx_regrid_leaves(len(trees), _np_ptr(trees), len(leaves),
                                     _np_ptr(leaves), _np_ptr(tags), lmin, lmax,
                                     cap, _np_ptr(out), C.byref(n))
        if rc == -1 and n.value > cap:
            cap = n.value
            continue
        _check(rc)
        return out[: n.value].copy()


def config(m, precision=64, physics=FCX_SHALLOW, limiter=4, transverse=2,
           tile=0, threads=0, g=1.0, ax=0.0, ay=0.0, cfl_desired=0.9,
           cfl_max=1.0, redo=1, period=1.0, axis=(0.0, 0.0, 1.0)):
    """period: FCX_SWIRL's flow period, FCX_ROTATION's time of one turn;
    axis: FCX_ROTATION's rotation axis."""
    return Config(m, precision, physics, limiter, transverse, tile, threads,
                  int(redo), g, ax, ay, cfl_desired, cfl_max, period,
                  (C.c_double * 3)(*axis))


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _dev(t, n, dtype):
    """Pointer of a contiguous device tensor of `dtype` with >= n elements."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype
            and t.is_contiguous() and t.numel() >= n):
        raise ValueError(f"expected a contiguous {dtype} device tensor of "
                         f">= {n} elements")
    return C.c_void_p(t.data_ptr())


# ---- learned tagging: context-free network calls ------------------------
def mlp_forward(params, norm, x, logits, stream=None):
    import torch
    rows = x.numel() // MLP_INPUTS
    f32 = torch.float32
    _check(lib().fcx_mlp_forward(_dev(params, MLP_PARAMS, f32), _dev(norm, 32, f32),
                                 rows, _dev(x, rows * MLP_INPUTS, f32),
                                 _dev(logits, rows * MLP_CLASSES, f32),
                                 _stream(stream)))


def mlp_backward(params, norm, x, labels, class_weight, scale, grad, loss,
                 stream=None):
    import torch
    rows = x.numel() // MLP_INPUTS
    f32 = torch.float32
    _check(lib().fcx_mlp_backward(_dev(params, MLP_PARAMS, f32), _dev(norm, 32, f32),
                                  rows, _dev(x, rows * MLP_INPUTS, f32),
                                  _dev(labels, rows, torch.int32),
                                  _dev(class_weight, MLP_CLASSES, f32), float(scale),
                                  _dev(grad, MLP_PARAMS, f32), _dev(loss, 1, f32),
                                  _stream(stream)))


def adam_step(params, grad, m1, m2, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              stream=None):
    import torch
    n = params.numel()
    f32 = torch.float32
    _check(lib().fcx_adam_step(n, _dev(params, n, f32), _dev(grad, n, f32),
                               _dev(m1, n, f32), _dev(m2, n, f32), int(t), lr, beta1,
                               beta2, eps, _stream(stream)))


def learned_tags(logits, plain, confidence, tags, stream=None):
    import torch
    rows = plain.numel()
    _check(lib().fcx_learned_tags(rows, _dev(logits, 3 * rows, torch.float32),
                                  _dev(plain, rows, torch.int8), float(confidence),
                                  _dev(tags, rows, torch.int8), _stream(stream)))


class Context:
    """One forest on the current HIP device (fcx_ctx)."""

    def __init__(self, cfg: Config, trees):
        self.cfg = cfg
        self.meqn = {FCX_ADVECTION: 1, FCX_SHALLOW: 3, FCX_SPHERE: 4, FCX_SWIRL: 1,
                     FCX_ROTATION: 1}[cfg.physics]
        self.trees = np.ascontiguousarray(trees, dtype=TREE_DTYPE)
        h = C.c_void_p()
        _check(lib().fcx_create(C.byref(cfg), len(self.trees),
                                _np_ptr(self.trees), C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().fcx_destroy(self.h)
            self.h = None

    # ---- forest -------------------------------------------------------
    def upload_forest(self, leaves):
        leaves = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
        _check(lib().fcx_upload_forest(self.h, len(leaves), _np_ptr(leaves)))

    def num_patches(self) -> int:
        return lib().fcx_num_patches(self.h)

    def state_elems(self) -> int:
        return lib().fcx_state_elems(self.h)

    def ghost_elems(self) -> int:
        return lib().fcx_ghost_elems(self.h)

    def leaves(self) -> np.ndarray:
        out = np.zeros(self.num_patches(), dtype=LEAF_DTYPE)
        _check(lib().fcx_get_leaves(self.h, len(out), _np_ptr(out)))
        return out

    def patch_table(self) -> dict:
        """Host copy of the patch tables: recs (P, 24), phislot, family,
        counts (slots, xi items, eta items), items (n, 8), aux (n, 6)."""
        P = self.num_patches()
        recs = np.zeros((P, 24), dtype=np.int32)
        phislot = np.zeros(P, dtype=np.int32)
        family = np.zeros(P, dtype=np.int32)
        counts = np.zeros(3, dtype=np.int32)
        _check(lib().fcx_patch_table(self.h, 0, _np_ptr(recs), _np_ptr(phislot),
                                     _np_ptr(family), _np_ptr(counts), None, None))
        n = int(counts[1]) + int(counts[2])
        items = np.zeros((n, 8), dtype=np.int32)
        aux = np.zeros((n, 6), dtype=np.int32)
        if n:
            _check(lib().fcx_patch_table(self.h, n, _np_ptr(recs), _np_ptr(phislot),
                                         _np_ptr(family), _np_ptr(counts), _np_ptr(items),
                                         _np_ptr(aux)))
        return {"recs": recs, "phislot": phislot, "family": family, "counts": counts,
                "items": items, "aux": aux}

    # ---- tensors ------------------------------------------------------
    def _dt(self):
        import torch
        return torch.float64 if self.cfg.precision == 64 else torch.float32

    def _state(self, t, n):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == self._dt()
                and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"expected a contiguous {self._dt()} device tensor "
                             f"of {n} elements")
        return C.c_void_p(t.data_ptr())

    def _q(self, t):
        return self._state(t, self.state_elems())

    def _g(self, t):
        return self._state(t, self.ghost_elems())

    @staticmethod
    def _d(t, n=1, dtype=None):
        import torch
        dtype = dtype or torch.float64
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype
                and t.numel() >= n):
            raise ValueError(f"expected a {dtype} device tensor")
        return C.c_void_p(t.data_ptr())

    # ---- the step -----------------------------------------------------
    def ghost_fill(self, q, ghost, stream=None):
        _check(lib().fcx_ghost_fill(self.h, self._q(q), self._g(ghost),
                                    _stream(stream)))

    def patch_step(self, q, ghost, q_new, dt, numax, stream=None):
        _check(lib().fcx_patch_step(self.h, self._q(q), self._g(ghost),
                                    self._q(q_new), self._d(dt), self._d(numax),
                                    _stream(stream)))

    def fused_step(self, q, q_new, dt, numax, stream=None):
        _check(lib().fcx_fused_step(self.h, self._q(q), self._q(q_new),
                                    self._d(dt), self._d(numax), _stream(stream)))

    def advance(self, q, q_new, dt, numax, status, stream=None):
        """Fused step + reflux + next dt in one call."""
        import torch
        _check(lib().fcx_advance(self.h, self._q(q), self._q(q_new), self._d(dt),
                                 self._d(numax), self._d(status, 1, torch.int32),
                                 _stream(stream)))

    def advance_subcycled(self, q, q_new, work, ghost, dt, numax, status, stream=None):
        """One sub-cycled step of the coarsest level (dt: a level-0 patch's
        step; level l steps with dt 2^-l)."""
        import torch
        _check(lib().fcx_advance_subcycled(self.h, self._q(q), self._q(q_new),
                                           self._q(work), self._g(ghost), self._d(dt),
                                           self._d(numax), self._d(status, 1, torch.int32),
                                           _stream(stream)))

    def reflux(self, q, q_new, dt, stream=None):
        _check(lib().fcx_reflux(self.h, self._q(q), self._q(q_new), self._d(dt),
                                _stream(stream)))

    def next_dt(self, numax, dt, status, stream=None):
        import torch
        _check(lib().fcx_next_dt(self.h, self._d(numax), self._d(dt),
                                 self._d(status, 1, torch.int32), _stream(stream)))

    def step_stats(self):
        """(accepted steps, rejected attempts, accepted cell updates)."""
        out = np.zeros(3, dtype=np.int64)
        _check(lib().fcx_step_stats(self.h, _np_ptr(out)))
        return tuple(int(v) for v in out)

    def sim_time(self) -> float:
        """Simulated time of the accepted steps since the context was made."""
        t = C.c_double()
        _check(lib().fcx_sim_time(self.h, C.byref(t)))
        return t.value

    def conservation_sums(self, q, sums, stream=None):
        _check(lib().fcx_conservation_sums(self.h, self._q(q),
                                           self._d(sums, self.meqn),
                                           _stream(stream)))

    def conservation_sums_noalloc(self, q, sums, stream=None):
        """As conservation_sums, with the library's fixed scratch array (the
        call allocates nothing)."""
        _check(lib().fcx_conservation_sums_noalloc(self.h, self._q(q),
                                                   self._d(sums, self.meqn),
                                                   _stream(stream)))

    # ---- regrid -------------------------------------------------------
    def regrid_tags(self, q, ghost, criterion, threshold, lmin, lmax, tags,
                    stream=None):
        import torch
        g = self._g(ghost) if ghost is not None else None
        _check(lib().fcx_regrid_tags(self.h, self._q(q), g, criterion, threshold,
                                     lmin, lmax,
                                     self._d(tags, self.num_patches(), torch.int8),
                                     _stream(stream)))

    def features(self, q, ghost, feats, stream=None):
        import torch
        _check(lib().fcx_features(self.h, self._q(q), self._g(ghost),
                                  _dev(feats, MLP_INPUTS * self.num_patches(),
                                       torch.float32), _stream(stream)))

    def dilate_tags(self, tags_in, lmax, tags_out, stream=None):
        import torch
        n = self.num_patches()
        _check(lib().fcx_dilate_tags(self.h, _dev(tags_in, n, torch.int8), lmax,
                                     _dev(tags_out, n, torch.int8), _stream(stream)))

    def sphere_geometry(self, out=None, stream=None):
        """(P, 18, m+4, m+4) geometry tables of a sphere context (device)."""
        import torch
        m = self.cfg.m
        n = self.num_patches() * GEO_FRAMES * (m + 4) ** 2
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(lib().fcx_sphere_geometry(self.h, _dev(out, n, torch.float64),
                                         _stream(stream)))
        return out.view(self.num_patches(), GEO_FRAMES, m + 4, m + 4)

    def regrid(self, q, ghost, criterion, threshold, lmin, lmax, stream=None,
               old_to_new=False):
        """Ghost fill, tags, and mesh change in one call; returns the new
        patch count (then allocate the new state and call regrid_transfer
        with q and ghost), and with old_to_new=True also the old-to-new map
        (see regrid_apply)."""
        n = C.c_int64()
        o2n = np.zeros(self.num_patches(), dtype=np.int64) if old_to_new else None
        _check(lib().fcx_regrid(self.h, self._q(q), self._g(ghost), criterion, threshold,
                                lmin, lmax, C.byref(n),
                                _np_ptr(o2n) if old_to_new else None, _stream(stream)))
        return (n.value, o2n) if old_to_new else n.value

    def run(self, q0, q1, ghost, steps, step0, regrid_every, criterion, threshold,
            lmin, lmax, dt, numax, status, fused=True, stream=None):
        """`steps` whole steps with periodic regrids on two capacity buffers
        (fused: True / 1 fused steps, False / 0 plain, 2 sub-cycled);
        returns (index of the buffer with the result, cell updates)."""
        import torch
        dtype = torch.float64 if self.cfg.precision == 64 else torch.float32
        for t in (q0, q1, ghost):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype
                    and t.is_contiguous()):
                raise ValueError("expected contiguous state tensors of the context's type")
        which = C.c_int32()
        cells = C.c_int64()
        _check(lib().fcx_run(self.h, int(fused), C.c_void_p(q0.data_ptr()),
                             C.c_void_p(q1.data_ptr()),
                             min(q0.numel(), q1.numel()), C.c_void_p(ghost.data_ptr()),
                             ghost.numel(), steps, step0, regrid_every, criterion,
                             threshold, lmin, lmax, self._d(dt), self._d(numax),
                             self._d(status, 1, torch.int32), C.byref(which),
                             C.byref(cells), _stream(stream)))
        return which.value, cells.value

    def regrid_apply(self, tags_host, lmin, lmax, old_to_new=False):
        """Applies host tags; returns the new patch count, and with
        old_to_new=True also the map of every old patch: >= 0 kept at that
        index, -2 - k refined into k .. k+3, -1 merged into a parent."""
        t = np.ascontiguousarray(tags_host, dtype=np.int8)
        if len(t) != self.num_patches():
            raise ValueError("one tag per patch expected")
        n = C.c_int64()
        o2n = np.zeros(len(t), dtype=np.int64) if old_to_new else None
        _check(lib().fcx_regrid_apply(self.h, _np_ptr(t), lmin, lmax, C.byref(n),
                                      _np_ptr(o2n) if old_to_new else None))
        return (n.value, o2n) if old_to_new else n.value

    def regrid_transfer(self, q_old, ghost_old, q_new, stream=None):
        # q_old / ghost_old are laid out on the previous forest
        _check(lib().fcx_regrid_transfer(self.h, C.c_void_p(q_old.data_ptr()),
                                         C.c_void_p(ghost_old.data_ptr()),
                                         self._q(q_new), _stream(stream)))


class Batch:
    """Independent forests advanced together (fcx_batch).  The contexts
    must outlive the batch; the binding keeps references to them."""

    def __init__(self, contexts):
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = C.c_void_p()
        _check(lib().fcx_batch_create(len(self.contexts), arr, C.byref(h)))
        self.h = h
        self.n = len(self.contexts)
        self.precision = self.contexts[0].cfg.precision

    def __del__(self):
        if getattr(self, "h", None):
            lib().fcx_batch_destroy(self.h)
            self.h = None

    def state_elems(self) -> int:
        return lib().fcx_batch_state_elems(self.h)

    def state_offset(self, f) -> int:
        return lib().fcx_batch_state_offset(self.h, f)

    def num_patches(self) -> int:
        return lib().fcx_batch_num_patches(self.h)

    def set_tuning(self, tile_big=16, threads8=64, threads16=256, persistent=0):
        _check(lib().fcx_batch_set_tuning(self.h, tile_big, threads8, threads16,
                                          persistent))

    def _q(self, t):
        import torch
        dt = torch.float64 if self.precision == 64 else torch.float32
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt
                and t.is_contiguous() and t.numel() == self.state_elems()):
            raise ValueError("expected the batch state tensor")
        return C.c_void_p(t.data_ptr())

    def _per_forest(self, t, dtype):
        return Context._d(t, self.n, dtype)

    def step(self, q, q_new, dt, numax, status, stream=None):
        import torch
        _check(lib().fcx_batch_step(self.h, self._q(q), self._q(q_new),
                                    self._per_forest(dt, torch.float64),
                                    self._per_forest(numax, torch.float64),
                                    self._per_forest(status, torch.int32),
                                    _stream(stream)))

    def capture(self, steps, q_a, q_b, dt, numax, status):
        import torch
        _check(lib().fcx_batch_capture(self.h, steps, self._q(q_a), self._q(q_b),
                                       self._per_forest(dt, torch.float64),
                                       self._per_forest(numax, torch.float64),
                                       self._per_forest(status, torch.int32)))

    def replay(self, stream=None):
        _check(lib().fcx_batch_replay(self.h, _stream(stream)))

    def step_stats(self):
        """(n, 3): per forest accepted steps, rejected attempts, accepted
        cell updates."""
        out = np.zeros((self.n, 3), dtype=np.int64)
        _check(lib().fcx_batch_step_stats(self.h, _np_ptr(out)))
        return out

    def class_items(self):
        """(items, simple): per tile class (advection 8x8, shallow water
        8x8, advection with the tuned tile, shallow water with it) the work
        items of the current tuning and those with a strip-copy halo."""
        items = np.zeros(4, dtype=np.int32)
        simple = np.zeros(4, dtype=np.int32)
        _check(lib().fcx_batch_class_items(self.h, _np_ptr(items), _np_ptr(simple)))
        return items.tolist(), simple.tolist()

    def sums(self, q, out, stream=None):
        import torch
        _check(lib().fcx_batch_sums(self.h, self._q(q),
                                    Context._d(out, 4 * self.n, torch.float64),
                                    _stream(stream)))
