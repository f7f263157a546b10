#!/usr/bin/env python
"""Benchmark of one time step of the leaf-patch AMR hot path on one MI355X.

Workload (the headline configuration): 2D shallow water (h, hu, hv), g = 1,
Roe solver with transverse waves and the MC limiter, unit square with
reflecting walls, radial dam break (h = 2 for r < 0.25, else 1, at rest);
2:1-balanced adaptive forest on levels 3..6 with m = 16, refined where
|grad h| > 0.1 and regridded every 4 steps; CFL 0.9.  Inputs are seeded
synthetic data built on the host, then resident in HBM.

A step = regrid (every 4th step: tags on the GPU, host refine/coarsen/
balance, transfer on the GPU) + ghost fill + wave-propagation update +
coarse-fine reflux + next dt, all through libfcx.so.  Two variants are
timed: FP32 state in one fused ghost-gather + update launch per step (the
reported value) and the FP64 plain path (separate ghost-fill and step
launches).  A large uniform variant (level 8, 65,536 patches, 16.8 M cells)
gives the HBM roofline of the same kernels at a size far beyond the
on-chip caches.

Prints one JSON line.  `python bench.py --gpus N` with N > 1 exits: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed math (256 CUs x 64 lanes x 2.4 GHz, one
# operation per lane per clock; an FMA counts once)
VALU_PEAK_GOPS = 256 * 64 * 2.4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--large-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp32", "fp64", "large", "batch", "sphere",
                                       "mlp", "copy", "cpu", "subcycle", "meshing", "swirl",
                                       "rotation", "all"],
                    default="all")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--sphere-steps", type=int, default=1000)
    ap.add_argument("--sphere64-steps", type=int, default=48)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("step.hpp", "advect.hpp", "batch.hpp", "device.hpp"):
        with open(os.path.join(ROOT, "paper_1308_1472_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_profile(name, key):
    """A figure of a committed rocprofv3 summary under profiles/, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*(\w+)", text)
    b = re.search(key + r":\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def stored_traffic(name):
    """HBM bytes per launch (memory counters scaled by a plain copy)."""
    return stored_profile(name, "hbm_bytes_per_launch")


STATUS_BITS = {1: "cfl_kept", 2: "negative_depth", 4: "nested_interpolation",
               8: "rejected_and_redone"}
# bits that mark a timed step as wrong (a redone attempt is the CFL rule
# working, not a fault)
BAD_BITS = 1 | 2 | 4


def status_bits(words):
    """Per status bit, the number of status words (forests) that carry it."""
    words = [int(w) for w in words]
    return {name: sum(1 for w in words if w & bit) for bit, name in STATUS_BITS.items()}


class Workload:
    """Adaptive dam break driven entirely through the library: the timed
    steps run in the library's own run loop (fcx_run) on two state buffers
    sized for the finest forest the run can reach."""

    LMIN, LMAX, M, THR, REGRID = 3, 6, 16, 0.1, 4

    def __init__(self, precision, fused, uniform_level=None, tile=0, threads=0):
        import torch
        from paper_1308_1472_amd import fcx
        from paper_1308_1472_amd import inputs as I
        self.torch, self.fcx, self.I = torch, fcx, I
        self.trees, self.pl = I.walled_square()
        self.fused = fused
        self.uniform = uniform_level is not None
        self.cfg = fcx.config(self.M, precision, fcx.FCX_SHALLOW, cfl_desired=0.9,
                              cfl_max=1.0, tile=tile, threads=threads)
        self.ctx = fcx.Context(self.cfg, self.trees)
        self.dtype = torch.float32 if precision == 32 else torch.float64
        fn = lambda x, y: I.dam_break(x, y)
        if self.uniform:
            leaves = fcx.sfc_sort(I.uniform_leaves(1, uniform_level))
        else:
            leaves = fcx.sfc_sort(I.uniform_leaves(1, self.LMIN))
            # initial mesh: tag the initial data, refine, re-evaluate, until
            # nothing changes
            for _ in range(2 * (self.LMAX - self.LMIN) + 2):
                self.ctx.upload_forest(leaves)
                q = self._tensor(I.state_from(leaves, self.M, fn, self.pl))
                g = torch.empty(self.ctx.ghost_elems(), dtype=self.dtype, device="cuda")
                self.ctx.regrid(q, g, 1, self.THR, self.LMIN, self.LMAX)
                new = self.ctx.leaves()
                if len(new) == len(leaves) and (new == leaves).all():
                    break
                leaves = new
        self.ctx.upload_forest(leaves)
        # capacity: every patch at the finest level the run can reach
        finest = uniform_level if self.uniform else self.LMAX
        pmax = 1 << (2 * finest)
        meqn = self.ctx.meqn
        cap = pmax * meqn * self.M * self.M
        self.buf = [torch.empty(cap, dtype=self.dtype, device="cuda") for _ in range(2)]
        self.ghost = torch.empty(pmax * meqn * (8 * self.M + 16), dtype=self.dtype,
                                 device="cuda")
        q0 = self._tensor(I.state_from(leaves, self.M, fn, self.pl))
        self.buf[0][:q0.numel()].copy_(q0)
        self.cur = 0
        dev = "cuda"
        hmin = 1.0 / (self.M << int(leaves["level"].max()))
        # start at half the target Courant number: the first steps of a dam
        # break raise the largest wave speed
        dt0 = 0.45 * hmin / 2.0 ** 0.5
        if fused == 2:                    # sub-cycled: the step of a level-0 patch
            dt0 *= float(1 << int(leaves["level"].max()))
        self.dt = torch.full((1,), dt0, dtype=torch.float64, device=dev)
        self.numax = torch.zeros(1, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.n = 0

    def _tensor(self, q):
        return self.torch.from_numpy(q.ravel()).to(self.dtype).cuda()

    def state(self):
        """(current state, the other buffer) as tensors of the forest's size."""
        n = self.ctx.state_elems()
        return self.buf[self.cur][:n], self.buf[1 - self.cur][:n]

    def advance(self, steps, every=None):
        """`steps` steps in the library's run loop; returns cell updates."""
        every = self.REGRID if every is None else every
        which, cells = self.ctx.run(
            self.buf[self.cur], self.buf[1 - self.cur], self.ghost, steps, self.n,
            0 if self.uniform else every, 1, self.THR, self.LMIN, self.LMAX,
            self.dt, self.numax, self.status, fused=self.fused)
        if which == 1:
            self.cur = 1 - self.cur
        self.n += steps
        return cells


TUNE = {"tile": 0, "threads": 0}


def run(precision, fused, steps, warmup, uniform_level=None):
    """Warm-up attempts, then `steps` timed attempts in the library's run
    loop (reject-and-redo on: only accepted steps count as cell updates)."""
    import torch
    w = Workload(precision, fused, uniform_level, TUNE["tile"], TUNE["threads"])
    if warmup:
        w.advance(warmup)
    torch.cuda.synchronize()
    w.status.zero_()                      # flags of the timed attempts only
    before = w.ctx.step_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cells = float(w.advance(steps))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    after = w.ctx.step_stats()
    status = int(w.status.item())
    # the step kernel alone: nk back-to-back launches on the current mesh
    # between two HIP events on the launch stream (the launch is idempotent:
    # it reads q and writes q_new)
    nk = 20
    q, qn = w.state()
    g = w.ghost[:w.ctx.ghost_elems()]
    if not w.fused:
        w.ctx.ghost_fill(q, g)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(nk):
        if w.fused:
            w.ctx.fused_step(q, qn, w.dt, w.numax)
        else:
            w.ctx.patch_step(q, g, qn, w.dt, w.numax)
    b.record()
    torch.cuda.synchronize()
    w.numax.zero_()
    out = {
        "seconds": el, "cells": cells, "rate": cells / el,
        "attempts": steps, "accepted": after[0] - before[0],
        "rejected": after[1] - before[1],
        "kernel_ms_mean": a.elapsed_time(b) / nk,
        "kernel_cells_mean": float(w.ctx.num_patches() * w.M * w.M),
        "patches_last": w.ctx.num_patches(),
        "status": status, "status_bits": status_bits([status]),
    }
    if uniform_level is not None:
        out["_state"] = q                 # for the FP32-vs-FP64 comparison
    return out


def run_time_stepping(coarse_steps=24, precision=32):
    """The meshing-strategy comparison of the paper on one GPU: the adaptive
    dam break advanced with one global dt (fused and plain steps, regrid
    every 4 steps) and sub-cycled (level l steps with its own dt, regrid
    every 4 and every 1 coarsest-level steps), each from t = 0 for about the
    same simulated time; reports simulated time per second of wall clock
    (time to solution) and cell updates per second."""
    import torch
    out = {}
    variants = (("global_fused_regrid4", True, 4, 8 * coarse_steps),
                ("global_plain_regrid4", False, 4, 8 * coarse_steps),
                ("subcycled_regrid4", 2, 4, coarse_steps),
                ("subcycled_regrid1", 2, 1, coarse_steps))
    for name, mode, every, steps in variants:
        Workload(precision, mode).advance(4, every)          # warm-up
        torch.cuda.synchronize()
        w = Workload(precision, mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cells = float(w.advance(steps, every))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        acc, rej, _ = w.ctx.step_stats()
        sim = w.ctx.sim_time()
        status = int(w.status.item())
        out[name] = {"attempts": steps, "accepted": acc, "rejected": rej,
                     "regrid_every": every, "seconds": el, "sim_time": sim,
                     "sim_time_per_s": sim / el, "cell_updates": cells,
                     "rate": cells / el, "patches_last": w.ctx.num_patches(),
                     "status": status, "status_bits": status_bits([status])}
    base = out["global_fused_regrid4"]["sim_time_per_s"]
    for name in out:
        out[name]["time_to_solution_speedup_vs_global_fused"] = out[name]["sim_time_per_s"] / base
    return out


def run_meshing(precision=32, m=8, lmin=3, lmax=8, T=0.25, thr=0.5):
    """The meshing strategies of the paper's advection example (its wall-clock
    table: uniform or adaptive mesh, remesh every step or every 4, global or
    sub-cycled time steps) on one GPU.  Stand-in flow: the paper's swirl
    velocity field is not given, so the 0/1 disk (radius 1/4, centre (1/2,
    1/2)) is carried by the constant velocity a = (1, 1/2) on the periodic
    unit square, m = 8, levels 3-8 (uniform: level 8), refined where
    max - min of q over a patch exceeds 1/2 (coarsened below), CFL 0.9, to
    t = T.  Reports wall clock to T, cell updates, and the L1 error against
    the translated disk."""
    import math
    import numpy as np
    import torch
    from paper_1308_1472_amd import fcx
    from paper_1308_1472_amd import inputs as I
    trees, pl = I.periodic_square()
    ax, ay = 1.0, 0.5
    cx, cy = 0.5, 0.5
    disk = lambda x, y: np.where((x - cx) ** 2 + (y - cy) ** 2 < 0.0625, 1.0, 0.0)
    dtype = torch.float32 if precision == 32 else torch.float64

    def make(mode, uniform):
        cfg = fcx.config(m, precision, fcx.FCX_ADVECTION, ax=ax, ay=ay)
        ctx = fcx.Context(cfg, trees)
        if uniform:
            leaves = fcx.sfc_sort(I.uniform_leaves(1, lmax))
        else:
            leaves = fcx.sfc_sort(I.uniform_leaves(1, lmin))
            for _ in range(2 * (lmax - lmin) + 2):
                ctx.upload_forest(leaves)
                q = torch.from_numpy(I.state_from(leaves, m, disk, pl).ravel()).to(dtype).cuda()
                g = torch.empty(ctx.ghost_elems(), dtype=dtype, device="cuda")
                ctx.regrid(q, g, 0, thr, lmin, lmax)
                new = ctx.leaves()
                if len(new) == len(leaves) and (new == leaves).all():
                    break
                leaves = new
        ctx.upload_forest(leaves)
        pmax = 1 << (2 * lmax)
        bufs = [torch.empty(pmax * m * m, dtype=dtype, device="cuda") for _ in range(2)]
        ghost = torch.empty(pmax * (8 * m + 16), dtype=dtype, device="cuda")
        q0 = I.state_from(leaves, m, disk, pl)
        bufs[0][:q0.size].copy_(torch.from_numpy(q0.ravel()))
        # CFL 0.9 with |a| = 1 on the finest cells (sub-cycled: a level-0
        # patch's step, each level scaled by its own size)
        dt = 0.9 / m if mode == 2 else 0.9 / (m << lmax)
        return ctx, bufs, ghost, torch.full((1,), dt, dtype=torch.float64, device="cuda")

    def exact_l1(ctx, q):
        lv = ctx.leaves()
        want = I.state_from(lv, m, lambda x, y: disk((x - ax * T) % 1.0, (y - ay * T) % 1.0),
                            pl)
        got = q.double().cpu().numpy().reshape(want.shape)
        h = np.ldexp(1.0, -lv["level"].astype(int)) / m
        return float(np.sum(np.abs(got - want)[:, 0] * (h ** 2)[:, None, None]))

    strategies = (("uniform", 1, 0, True), ("amr_every_step_global", 1, 1, False),
                  ("amr_every_4_global", 1, 4, False), ("amr_every_step_subcycle", 2, 1, False),
                  ("amr_every_4_subcycle", 2, 4, False))
    out = {}
    for name, mode, every, uniform in strategies:
        for rep in range(2):                      # the first run warms up
            ctx, bufs, ghost, dt = make(mode, uniform)
            nu = torch.zeros_like(dt)
            st = torch.zeros(1, dtype=torch.int32, device="cuda")
            span = dt.item() * (math.ldexp(1.0, -lmin) if mode == 2 else 1.0)
            steps = int(math.ceil(T / span - 1e-9))
            sums = torch.zeros(1, dtype=torch.float64, device="cuda")
            ctx.conservation_sums(bufs[0][:ctx.state_elems()], sums)
            m0 = sums.item()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            which, cells = ctx.run(bufs[0], bufs[1], ghost, steps, 0, every, 0, thr, lmin,
                                   lmax, dt, nu, st, fused=mode)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        qf = bufs[which][:ctx.state_elems()]
        ctx.conservation_sums(qf, sums)
        status = int(st.item())
        out[name] = {"seconds": el, "steps": steps, "sim_time": ctx.sim_time(),
                     "cell_updates": cells, "rate": cells / el,
                     "patches_last": ctx.num_patches(), "l1_error": exact_l1(ctx, qf),
                     "mass_rel_change": sums.item() / m0 - 1.0, "status": status,
                     "status_bits": status_bits([status])}
    base = out["uniform"]["seconds"]
    for name in out:
        out[name]["speedup_vs_uniform"] = base / out[name]["seconds"]
    return out


def run_swirl(precision=32, m=8, lmin=3, lmax=6, T=2.0, thr=0.2):
    """The paper's advection example (Sec. 5, Example 1): q = 1 on the left
    half of the unit square and 0 on the right, carried by a twisting flow
    that the paper does not give.  Stand-in flow (FCX_SWIRL): the swirl
    stream function sin^2(pi x) sin^2(pi y) cos(pi t / T) / pi, which
    reverses at T / 2, so the exact state after one period T is the initial
    one.  Walled square, m = 8, levels 3-6 (the paper's 64^2 to 512^2),
    refined where max - min of q over a patch exceeds 0.2 (the front smears
    as it winds up), CFL 0.9 with the redo rule; uniform level 6 for
    comparison.  Runs fcx_run in chunks, each sized from the remaining time
    over the current dt, until the simulated time reaches T (it ends at most
    one step past T); reports wall clock, cell updates, rate and the L1 error
    against the initial state."""
    import numpy as np
    import torch
    from paper_1308_1472_amd import fcx
    from paper_1308_1472_amd import inputs as I
    trees, pl = I.walled_square()
    halves = lambda x, y: np.where(x < 0.5, 1.0, 0.0) + 0.0 * y
    dtype = torch.float32 if precision == 32 else torch.float64

    def make(uniform):
        cfg = fcx.config(m, precision, fcx.FCX_SWIRL, period=T)
        ctx = fcx.Context(cfg, trees)
        if uniform:
            leaves = fcx.sfc_sort(I.uniform_leaves(1, lmax))
        else:
            leaves = fcx.sfc_sort(I.uniform_leaves(1, lmin))
            for _ in range(2 * (lmax - lmin) + 2):
                ctx.upload_forest(leaves)
                q = torch.from_numpy(I.state_from(leaves, m, halves, pl).ravel()).to(dtype).cuda()
                g = torch.empty(ctx.ghost_elems(), dtype=dtype, device="cuda")
                ctx.regrid(q, g, 0, thr, lmin, lmax)
                new = ctx.leaves()
                if len(new) == len(leaves) and (new == leaves).all():
                    break
                leaves = new
        ctx.upload_forest(leaves)
        pmax = 1 << (2 * lmax)
        bufs = [torch.empty(pmax * m * m, dtype=dtype, device="cuda") for _ in range(2)]
        ghost = torch.empty(pmax * (8 * m + 16), dtype=dtype, device="cuda")
        q0 = I.state_from(leaves, m, halves, pl)
        bufs[0][:q0.size].copy_(torch.from_numpy(q0.ravel()))
        return ctx, bufs, ghost, torch.full((1,), 0.9 / (m << lmax), dtype=torch.float64,
                                           device="cuda")

    out = {}
    for name, every, uniform in (("uniform_level6", 0, True), ("amr_every_4", 4, False),
                                 ("amr_every_step", 1, False)):
        for rep in range(2):                      # the first run warms up
            ctx, bufs, ghost, dt = make(uniform)
            nu = torch.zeros_like(dt)
            st = torch.zeros(1, dtype=torch.int32, device="cuda")
            attempts, cells, which, k = 0, 0, 0, 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while True:
                left = T - ctx.sim_time()
                if left <= 0:
                    break
                chunk = max(1, min(256, int(left / dt.item())))
                a, b = bufs[which], bufs[1 - which]
                w, c = ctx.run(a, b, ghost, chunk, k, every, 0, thr, lmin, lmax, dt, nu, st,
                               fused=1)
                which = which if w == 0 else 1 - which
                attempts, cells, k = attempts + chunk, cells + c, k + chunk
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        lv = ctx.leaves()
        want = I.state_from(lv, m, halves, pl)
        got = bufs[which][:ctx.state_elems()].double().cpu().numpy().reshape(want.shape)
        h = np.ldexp(1.0, -lv["level"].astype(int)) / m
        l1 = float(np.sum(np.abs(got - want)[:, 0] * (h ** 2)[:, None, None]))
        acc, rej, _ = ctx.step_stats()
        status = int(st.item())
        out[name] = {"seconds": el, "attempts": attempts, "accepted": acc, "rejected": rej,
                     "sim_time": ctx.sim_time(), "cell_updates": cells, "rate": cells / el,
                     "patches_last": ctx.num_patches(), "l1_error_vs_initial": l1,
                     "status": status, "status_bits": status_bits([status])}
    base = out["uniform_level6"]["seconds"]
    for name in out:
        out[name]["speedup_vs_uniform"] = base / out[name]["seconds"]
    return out


def run_rotation(precision=32, m=8, lmin=3, lmax=6, T=1.0, thr=0.2,
                 axis=(0.3, -0.4, 0.866)):
    """The paper's sphere example (Sec. 5, Example 2): q = 1 on one half of
    the sphere and 0 on the other, the halves split by a great circle that
    follows no tree edge, carried by a rigid rotation (FCX_ROTATION) once
    around a tilted axis, so the exact state after the period T is the
    initial one.  On the two-tree (pillow) sphere of the example, one tree
    per hemisphere, m = 8, levels 3-6 (64^2 to 512^2 cells per hemisphere),
    refined where max - min of q over a patch exceeds 0.2, CFL 0.9 with the
    redo rule, plain steps; uniform level 6 for comparison.  Runs fcx_run in
    chunks until the simulated time reaches T (at most one step past it);
    reports wall clock, cell updates, rate and the L1 error (area weighted)
    against the initial state."""
    import numpy as np
    import torch
    from paper_1308_1472_amd import fcx
    from paper_1308_1472_amd import inputs as I
    trees = I.pillow_sphere()
    nt = len(trees)
    dtype = torch.float32 if precision == 32 else torch.float64

    def make(uniform):
        cfg = fcx.config(m, precision, fcx.FCX_ROTATION, period=T, axis=axis)
        ctx = fcx.Context(cfg, trees)
        if uniform:
            leaves = fcx.sfc_sort(I.uniform_leaves(nt, lmax))
        else:
            leaves = fcx.sfc_sort(I.uniform_leaves(nt, lmin))
            for _ in range(2 * (lmax - lmin) + 2):
                ctx.upload_forest(leaves)
                q = torch.from_numpy(I.sphere_halves(leaves, m, pillow=True).ravel()).to(
                    dtype).cuda()
                g = torch.empty(ctx.ghost_elems(), dtype=dtype, device="cuda")
                ctx.regrid(q, g, 0, thr, lmin, lmax)
                new = ctx.leaves()
                if len(new) == len(leaves) and (new == leaves).all():
                    break
                leaves = new
        ctx.upload_forest(leaves)
        pmax = nt << (2 * lmax)
        bufs = [torch.empty(pmax * m * m, dtype=dtype, device="cuda") for _ in range(2)]
        ghost = torch.empty(pmax * (8 * m + 16), dtype=dtype, device="cuda")
        q0 = I.sphere_halves(leaves, m, pillow=True)
        bufs[0][:q0.size].copy_(torch.from_numpy(q0.ravel()))
        dt0 = 0.5 * (np.pi / 2) / (m << lmax) * T / (2 * np.pi)
        return ctx, bufs, ghost, torch.full((1,), dt0, dtype=torch.float64, device="cuda")

    out = {}
    for name, every, uniform in (("uniform_level6", 0, True), ("amr_every_4", 4, False),
                                 ("amr_every_step", 1, False)):
        for rep in range(2):                      # the first run warms up
            ctx, bufs, ghost, dt = make(uniform)
            nu = torch.zeros_like(dt)
            st = torch.zeros(1, dtype=torch.int32, device="cuda")
            attempts, cells, which, k = 0, 0, 0, 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while True:
                left = T - ctx.sim_time()
                if left <= 0:
                    break
                chunk = max(1, min(256, int(left / dt.item())))
                a, b = bufs[which], bufs[1 - which]
                w, c = ctx.run(a, b, ghost, chunk, k, every, 0, thr, lmin, lmax, dt, nu, st,
                               fused=0)
                which = which if w == 0 else 1 - which
                attempts, cells, k = attempts + chunk, cells + c, k + chunk
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        lv = ctx.leaves()
        want = I.sphere_halves(lv, m, pillow=True)
        got = bufs[which][:ctx.state_elems()].double().cpu().numpy().reshape(want.shape)
        geo = ctx.sphere_geometry().cpu().numpy()
        kap = geo[:, 0].reshape(len(lv), m + 4, m + 4)[:, 2:m + 2, 2:m + 2]
        h = np.ldexp(1.0, -lv["level"].astype(int)) / m
        l1 = float(np.sum(np.abs(got - want)[:, 0] * kap * (h ** 2)[:, None, None]))
        acc, rej, _ = ctx.step_stats()
        status = int(st.item())
        out[name] = {"seconds": el, "attempts": attempts, "accepted": acc, "rejected": rej,
                     "sim_time": ctx.sim_time(), "cell_updates": cells, "rate": cells / el,
                     "patches_last": ctx.num_patches(), "l1_error_vs_initial": l1,
                     "status": status, "status_bits": status_bits([status])}
    base = out["uniform_level6"]["seconds"]
    for name in out:
        out[name]["speedup_vs_uniform"] = base / out[name]["seconds"]
    return out


def rel_l1(a, b, meqn, cells):
    """Largest relative L1 difference over the components of two states of
    one forest (compact layout: patch, component, cells), a against b."""
    a = a.double().view(-1, meqn, cells)
    b = b.double().view(-1, meqn, cells)
    worst = 0.0
    for k in range(meqn):
        den = b[:, k].abs().sum().item()
        if den > 0:
            worst = max(worst, (a[:, k] - b[:, k]).abs().sum().item() / den)
    return worst


def _batch_forests(precision, nforests=64):
    """The seeded forests of the batch: contexts and initial states."""
    from paper_1308_1472_amd import fcx
    from paper_1308_1472_amd import inputs as I
    ctxs, states = [], []
    for seed in range(nforests):
        spec, trees, pl, raw, fn = I.batch_forest(seed)
        lv = fcx.balance(trees, raw)
        phys = fcx.FCX_ADVECTION if spec["physics"] == "advection" else fcx.FCX_SHALLOW
        cfg = fcx.config(spec["m"], precision, phys, ax=spec.get("ax", 0.0),
                         ay=spec.get("ay", 0.0))
        ctx = fcx.Context(cfg, trees)
        ctx.upload_forest(lv)
        ctxs.append(ctx)
        states.append(I.state_from(lv, spec["m"], fn, pl))
    return ctxs, states


def _probe_dt(n):
    """A dt far below every forest's stable one: the first step's next-dt
    rule then sets dt = cfl_desired / (largest wave speed / cell size) per
    forest, from the forest's own waves."""
    import torch
    return torch.full((n,), 1e-7, dtype=torch.float64, device="cuda")


def run_batch(steps, warmup, nforests=64, graph_steps=10):
    """The 64-forest batch: seeded forests (advection or shallow water by
    seed parity, m in {8, 16, 32}, patch counts log-uniform in 16..16384,
    levels 2..8), FP32, one launch per tile class (a workgroup per tile or
    persistent workgroups), captured in a graph of `graph_steps` steps,
    tunables from the autotuner.  dt per forest from its own first step
    (probe), then the CFL rule with reject-and-redo; the rate counts the
    accepted cell updates of the timed replays."""
    import torch
    from paper_1308_1472_amd import autotune, fcx
    ctxs, states = _batch_forests(32, nforests)
    batch = fcx.Batch(ctxs)
    q = torch.empty(batch.state_elems(), dtype=torch.float32, device="cuda")
    for f, st in enumerate(states):
        o = batch.state_offset(f)
        q[o:o + st.size].copy_(torch.from_numpy(st.ravel()))
    cells = float(sum(st.size // c.meqn for st, c in zip(states, ctxs)))
    # algorithmic bytes: read and write every state value once (FP32)
    step_bytes = float(sum(st.size * 4 * 2 for st in states))
    adv_bytes = float(sum(st.size * 4 * 2 for st, c in zip(states, ctxs) if c.meqn == 1))
    best, timings = autotune.tune(batch, q, steps=2, reps=2)
    qa, qb = q.clone(), torch.empty_like(q)
    n = batch.n
    dt = _probe_dt(n)
    nu = torch.zeros(n, dtype=torch.float64, device="cuda")
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    batch.step(qa, qb, dt, nu, status)          # the probe step
    qa, qb = qb, qa
    batch.capture(graph_steps, qa, qb, dt, nu, status)
    for _ in range(max(1, warmup // graph_steps)):
        batch.replay()
    torch.cuda.synchronize()
    status.zero_()
    before = batch.step_stats()
    reps = max(1, steps // graph_steps)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record()
    for _ in range(reps):
        batch.replay()
    b.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = a.elapsed_time(b)
    after = batch.step_stats()
    items, simple = batch.class_items()
    d = after - before
    acc_cells = float(d[:, 2].sum())
    nst = reps * graph_steps
    words = status.cpu().tolist()
    return {"forests": n, "patches": batch.num_patches(), "cells": cells,
            "steps": nst, "seconds": el, "rate": acc_cells / el,
            "accepted_cell_updates": acc_cells,
            "attempts": int(n * nst), "rejected": int(d[:, 1].sum()),
            "ms_per_step": ms / nst, "tuning": best,
            "autotune_ms_per_step": {k: round(v, 4) for k, v in sorted(timings.items())},
            "status_words_nonzero": int(sum(1 for w in words if w)),
            "status_bits": status_bits(words), "status_bad": int(
                sum(1 for w in words if w & BAD_BITS)),
            "bytes_per_step": step_bytes, "advection_bytes_per_step": adv_bytes,
            "class_items": items, "class_items_simple_halo": simple}


def run_batch_fp64_plain(steps=10, nforests=64):
    """The same 64 forests on the plain FP64 path, forest after forest:
    ghost fill, step, reflux, next dt (the library's single calls, no
    batching, no graph), from the same probe dt: the like-for-like
    reference of the batched FP32 rate."""
    import torch
    ctxs, states = _batch_forests(64, nforests)
    runs = []
    for c, st in zip(ctxs, states):
        q = torch.from_numpy(st.ravel().copy()).cuda()
        runs.append({"c": c, "q": q, "qn": torch.empty_like(q),
                     "g": torch.empty(c.ghost_elems(), dtype=torch.float64, device="cuda"),
                     "dt": torch.full((1,), 1e-7, dtype=torch.float64, device="cuda"),
                     "nu": torch.zeros(1, dtype=torch.float64, device="cuda"),
                     "st": torch.zeros(1, dtype=torch.int32, device="cuda")})

    def one_step():
        for r in runs:
            c = r["c"]
            c.ghost_fill(r["q"], r["g"])
            c.patch_step(r["q"], r["g"], r["qn"], r["dt"], r["nu"])
            c.reflux(r["q"], r["qn"], r["dt"])
            c.next_dt(r["nu"], r["dt"], r["st"])
            r["q"], r["qn"] = r["qn"], r["q"]

    one_step()                                   # the probe step
    for _ in range(3):
        one_step()
    torch.cuda.synchronize()
    for r in runs:
        r["st"].zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cells = float(sum(st.size // c.meqn for st, c in zip(states, ctxs)))
    words = [int(r["st"].item()) for r in runs]
    return {"steps": steps, "seconds": el, "rate": cells * steps / el,
            "ms_per_step": el / steps * 1e3, "status_bits": status_bits(words)}


def run_sphere(steps, precision=32, m=32, lmin=4, lmax=7, every=8, target=50000,
               kernel_timing=True, threshold=None):
    """Shallow water on the cubed sphere, adaptive: 6 trees, levels lmin..lmax,
    m x m patches, a seeded sum of Gaussian height bumps on h = 1 at rest.
    The initial mesh refines uniform level lmin by lmax - lmin regrids (|grad h|
    criterion, data carried by the regrid transfer); the threshold is set by
    bisection so that this mesh has target patches within 20 %.  Timed: the
    library's run loop with plain steps (ghost fill, step, reflux with
    cube-edge mass sync, next dt) and a regrid every `every` steps."""
    import math
    import numpy as np
    import torch
    from paper_1308_1472_amd import fcx
    from paper_1308_1472_amd import inputs as I
    trees = I.cubed_sphere()
    lv0 = fcx.sfc_sort(I.uniform_leaves(6, lmin))
    cfg = fcx.config(m, precision, fcx.FCX_SPHERE, cfl_desired=0.8, cfl_max=1.0)
    dtype = torch.float32 if precision == 32 else torch.float64
    q0 = torch.from_numpy(I.sphere_bumps(lv0, m).ravel()).to(dtype).cuda()
    maxp = 6 << (2 * lmax)
    cap = maxp * 4 * m * m
    bufs = [torch.empty(cap, dtype=dtype, device="cuda") for _ in range(2)]
    ghost = torch.empty(maxp * 4 * (8 * m + 16), dtype=dtype, device="cuda")

    def initial(thr):
        ctx = fcx.Context(cfg, trees)
        ctx.upload_forest(lv0)
        bufs[0][:q0.numel()].copy_(q0)
        cur = 0
        for _ in range(lmax - lmin):
            n = ctx.state_elems()
            ctx.regrid(bufs[cur][:n], ghost[:ctx.ghost_elems()], 1, thr, lmin, lmax)
            ctx.regrid_transfer(bufs[cur][:n], ghost, bufs[1 - cur][:ctx.state_elems()])
            cur = 1 - cur
        torch.cuda.synchronize()
        return ctx, cur

    lo, hi = math.log(1e-4), math.log(10.0)
    best = None
    for _ in range(0 if threshold is not None else 24):
        mid = 0.5 * (lo + hi)
        ctx, cur = initial(math.exp(mid))
        P = ctx.num_patches()
        if best is None or abs(P - target) < abs(best[1] - target):
            best = (math.exp(mid), P)
        if abs(P - target) <= 0.05 * target:
            break
        if P > target:
            lo = mid          # too many patches: raise the threshold
        else:
            hi = mid
    thr = threshold if threshold is not None else best[0]
    ctx, cur = initial(thr)
    P0 = ctx.num_patches()
    dt = torch.full((1,), 0.3 * (math.pi / 2) / (m << lmax), dtype=torch.float64,
                    device="cuda")
    nu = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    sums = torch.zeros(4, dtype=torch.float64, device="cuda")
    ctx.conservation_sums(bufs[cur][:ctx.state_elems()], sums)
    m0 = sums[0].item()
    q_a, q_b = bufs[cur], bufs[1 - cur]
    # warm-up: a few steps and one regrid, outside the timed region
    which, _ = ctx.run(q_a, q_b, ghost, every + 1, 0, every, 1, thr, lmin, lmax, dt, nu,
                       st, fused=False)
    if which == 1:
        q_a, q_b = q_b, q_a
    st.zero_()
    before = ctx.step_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    which, cells = ctx.run(q_a, q_b, ghost, steps, every + 1, every, 1, thr, lmin, lmax,
                           dt, nu, st, fused=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    after = ctx.step_stats()
    q_end = (q_b if which == 1 else q_a)[:ctx.state_elems()]
    ctx.conservation_sums(q_end, sums)
    mass = sums[0].item() / m0 - 1.0
    if not kernel_timing:
        status = int(st.item())
        return {"precision": precision, "patches_initial": P0,
                "patches_last": ctx.num_patches(), "steps": steps, "regrid_every": every,
                "cells": cells, "accepted": after[0] - before[0],
                "rejected": after[1] - before[1], "rate": cells / el,
                "mass_rel_change": mass, "status": status,
                "status_bits": status_bits([status])}
    # the step kernel alone: back-to-back launches on the final forest,
    # timed with events on the launch stream
    n = ctx.state_elems()
    g = ghost[:ctx.ghost_elems()]
    q_tmp = (q_a if which == 1 else q_b)[:n]
    ctx.ghost_fill(q_end, g)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(10):
        ctx.patch_step(q_end, g, q_tmp, dt, nu)
    ev[1].record()
    torch.cuda.synchronize()
    kms = ev[0].elapsed_time(ev[1]) / 10
    kcells = ctx.num_patches() * m * m
    # algorithmic bytes per cell: the state read and written (32 B in FP32)
    # and the geometry the step reads for the cell: the FP64 capacity (8 B),
    # two edge frames and the centre (in FP32 for FP32 state: 56 + 12 B)
    bpc = 32.0 + 8.0 + 68.0 if precision == 32 else 64.0 + 8.0 + 136.0
    alg = kcells * bpc
    status = int(st.item())
    return {"precision": precision, "threshold": thr, "patches_initial": P0,
            "patches_last": ctx.num_patches(),
            "steps": steps, "regrid_every": every, "cells": cells,
            "accepted": after[0] - before[0], "rejected": after[1] - before[1],
            "rate": cells / el, "ms_per_step": el / steps * 1e3,
            "mass_rel_change": mass, "status": status,
            "status_bits": status_bits([status]), "dt": dt.item(),
            "step_kernel": {"kernel": "k_sphere_step", "cells": kcells, "kernel_ms": kms,
                            "rate": kcells / (kms * 1e-3),
                            "roofline": {"bound": "hbm", "unit": "GB/s",
                                         "achieved": alg / (kms * 1e-3) / 1e9,
                                         "peak": HBM_PEAK_GBS,
                                         "frac": alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                         "bytes_per_cell": bpc}}}


def run_mlp(rows=50000, reps=50):
    """Tag network: forward (inference) and forward + backward + Adam
    (training step) throughput on seeded inputs, bfloat16 MFMA kernels."""
    import numpy as np
    import torch
    from paper_1308_1472_amd import fcx
    rng = np.random.default_rng(0)
    P = torch.from_numpy(rng.normal(0, 0.2, fcx.MLP_PARAMS).astype(np.float32)).cuda()
    norm = torch.cat([torch.zeros(16), torch.ones(16)]).cuda()
    x = torch.from_numpy(rng.normal(size=(rows, 16)).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.integers(0, 3, rows).astype(np.int32)).cuda()
    cw = torch.ones(3, device="cuda")
    z = torch.empty(rows, 3, device="cuda")
    g = torch.empty(fcx.MLP_PARAMS, device="cuda")
    loss = torch.empty(1, device="cuda")
    m1, m2 = torch.zeros_like(g), torch.zeros_like(g)
    out = {}
    for name in ("forward", "train_step"):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        for k in range(reps + 3):
            if k == 3:
                ev[0].record()
            if name == "forward":
                fcx.mlp_forward(P, norm, x, z)
            else:
                fcx.mlp_backward(P, norm, x, y, cw, 1.0 / rows, g, loss)
                fcx.adam_step(P, g, m1, m2, k + 1)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        # matrix products: 16x64 + 64x64 + 64x3 MACs per row forward; the
        # backward forms the same products twice more (weights and inputs)
        macs = 16 * 64 + 64 * 64 + 64 * 3
        flops = 2 * macs * rows * (1 if name == "forward" else 3)
        out[name] = {"rows": rows, "ms": ms, "rows_per_s": rows / (ms * 1e-3),
                     "tflops_bf16": flops / (ms * 1e-3) / 1e12}
    return out


def copy_calibration():
    """A plain device copy of known size (1 GiB, three times), whose memory
    counters scale the counters of the step kernels."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each": n * 4, "copies": 3}), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads():
    """Threads available to this process: the CPU affinity mask, capped by
    OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(warmup, steps, budget_s=6.0, reps=3):
    """The CPU FP64 oracle on the same attempts as the GPU's timed window of
    the headline workload (same initial mesh, dt rule with reject-and-redo,
    regrid every 4): the first `warmup` attempts untimed, then up to `steps`
    attempts timed, single-threaded and on every host thread, median of
    `reps` runs each.  A window longer than `budget_s` of one-thread work is
    cut to the attempts that fit, and both thread counts time that same cut
    window (same cell updates)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1308_1472_amd import inputs as I
    trees, pl = I.walled_square()
    m, lmin, lmax = Workload.M, Workload.LMIN, Workload.LMAX
    fn = lambda x, y: I.dam_break(x, y)
    par = O.params(m, O.SHALLOW)
    nthreads = _host_threads()
    O.set_threads(nthreads)
    lv = O.sfc_sort(I.uniform_leaves(1, lmin))
    for _ in range(2 * (lmax - lmin) + 2):
        mesh = O.Mesh(trees, lv, m)
        f = O.framed(I.state_from(lv, m, fn, pl), m)
        O.ghost_fill(mesh, par, f)
        lv2 = O.regrid(mesh, O.tags(mesh, par, f, 1, Workload.THR, lmin, lmax),
                       lmin, lmax)
        if np.array_equal(lv2, lv):
            break
        lv = lv2
    mesh = O.Mesh(trees, lv, m)
    q = I.state_from(lv, m, fn, pl)
    # the bench's first dt: 0.45 of the finest cell over sqrt(2)
    dt = 0.45 / (m << int(lv["level"].max())) / 2.0 ** 0.5

    def attempt(n, mesh, q, dt):
        if n > 0 and n % Workload.REGRID == 0:
            f = O.framed(q, m)
            O.ghost_fill(mesh, par, f)
            tg = O.tags(mesh, par, f, 1, Workload.THR, lmin, lmax)
            mesh2 = O.Mesh(trees, O.regrid(mesh, tg, lmin, lmax), m)
            q = O.interior(O.transfer(mesh, mesh2, par, f), m)
            mesh = mesh2
        qn, nu = O.advance(mesh, par, q, dt)
        ok = not nu > 1.0
        return mesh, (qn if ok else q), dt * 0.9 / nu, (len(mesh) * m * m if ok else 0)

    for n in range(warmup):
        mesh, q, dt, _ = attempt(n, mesh, q, dt)
    start = (mesh, q, dt)

    def window(limit, budget):
        mesh, q, dt = start
        cells, k = 0, 0
        t0 = time.perf_counter()
        while k < limit and (budget is None or time.perf_counter() - t0 < budget):
            mesh, q, dt, c = attempt(warmup + k, mesh, q, dt)
            cells += c
            k += 1
        return time.perf_counter() - t0, cells, k

    # the window that fits the budget on one thread, then the timed runs
    O.set_threads(1)
    _, cells, k = window(steps, budget_s)
    out = {}
    for name, t in (("single_thread", 1), ("all_threads", nthreads)):
        O.set_threads(t)
        times = sorted(window(k, None)[0] for _ in range(reps))
        out[name] = {"threads": t, "seconds_median": times[reps // 2],
                     "rate": cells / times[reps // 2]}
    O.set_threads(1)
    return {"value": out["all_threads"]["rate"], "unit": "cell-updates/s",
            "cores": nthreads, "kind": "oracle",
            "sample": f"attempts {warmup}..{warmup + k - 1} of the same adaptive dam break "
                      f"(levels 3-6, m = 16, regrid every 4, dt rule with reject-and-redo), "
                      f"{cells} cell updates, FP64, the ghost fill and the step's patch "
                      f"loop split over {nthreads} threads, median of {reps}",
            "single_thread": out["single_thread"]["rate"],
            "all_threads": out["all_threads"]["rate"],
            "seconds_median": {"single_thread": out["single_thread"]["seconds_median"],
                               "all_threads": out["all_threads"]["seconds_median"]},
            "cell_updates": cells, "attempts": k,
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def main():
    args = parse()
    TUNE["tile"], TUNE["threads"] = args.tile, args.threads
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path "
              "has no multi-GPU layout built", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.only == "copy":
        copy_calibration()
        return
    if args.only == "cpu":
        print(json.dumps({"cpu_baseline": cpu_baseline(args.warmup, args.steps)}), flush=True)
        return
    res = {}
    if args.only in ("fp32", "all"):
        res["fp32"] = run(32, True, args.steps, args.warmup)
        print(f"# fp32 fused: {res['fp32']}", file=sys.stderr, flush=True)
    if args.only in ("fp64", "all"):
        res["fp64"] = run(64, False, args.steps, args.warmup)
        print(f"# fp64 plain: {res['fp64']}", file=sys.stderr, flush=True)
    if args.only in ("large", "all"):
        res["large32"] = run(32, True, args.large_steps, 3, uniform_level=8)
        s32 = res["large32"].pop("_state")
        print(f"# large fp32: {res['large32']}", file=sys.stderr, flush=True)
        res["large64"] = run(64, False, args.large_steps, 3, uniform_level=8)
        s64 = res["large64"].pop("_state")
        # the same dam break, steps and dt rule in both precisions
        res["large32"]["rel_l1_vs_fp64"] = rel_l1(s32, s64, 3, 16 * 16)
        del s32, s64
        print(f"# large fp64: {res['large64']}; fp32 vs fp64 rel L1 "
              f"{res['large32']['rel_l1_vs_fp64']:.3e}", file=sys.stderr, flush=True)
    if args.only in ("batch", "all"):
        res["batch"] = run_batch(args.batch_steps, 30)
        print(f"# batch fp32: {res['batch']}", file=sys.stderr, flush=True)
        res["batch64"] = run_batch_fp64_plain()
        print(f"# batch fp64 plain: {res['batch64']}", file=sys.stderr, flush=True)
    if args.only in ("sphere", "all"):
        res["sphere"] = run_sphere(args.sphere_steps)
        print(f"# sphere fp32: {res['sphere']}", file=sys.stderr, flush=True)
        res["sphere64"] = run_sphere(args.sphere64_steps, precision=64, kernel_timing=False,
                                     threshold=res["sphere"]["threshold"])
        print(f"# sphere fp64: {res['sphere64']}", file=sys.stderr, flush=True)
    if args.only in ("subcycle", "all"):
        res["subcycle"] = run_time_stepping()
        print(f"# time stepping: {res['subcycle']}", file=sys.stderr, flush=True)
    if args.only in ("meshing", "all"):
        res["meshing"] = run_meshing()
        print(f"# meshing strategies: {res['meshing']}", file=sys.stderr, flush=True)
    if args.only in ("swirl", "all"):
        res["swirl"] = run_swirl()
        print(f"# example 1 (stand-in swirl): {res['swirl']}", file=sys.stderr, flush=True)
    if args.only in ("rotation", "all"):
        res["rotation"] = run_rotation()
        print(f"# example 2 (sphere rotation): {res['rotation']}", file=sys.stderr, flush=True)
    if args.only in ("mlp", "all"):
        res["mlp"] = run_mlp()
        print(f"# mlp: {res['mlp']}", file=sys.stderr, flush=True)
    # timed legs whose status words carry a bit that marks a wrong step
    bad = {k: r.get("status_bits") for k, r in res.items()
           if isinstance(r, dict) and (int(r.get("status", 0)) & BAD_BITS or r.get("status_bad"))}
    for leg in ("subcycle", "meshing", "swirl", "rotation"):
        for k, r in res.get(leg, {}).items():
            if r["status"] & BAD_BITS:
                bad[leg + "/" + k] = r["status_bits"]
    head = res.get("fp32") or res.get("fp64") or res.get("large32")
    if head is None:
        print(json.dumps({k: res.get(k) for k in ("batch", "batch64", "sphere", "sphere64",
                                                  "subcycle", "meshing", "swirl", "rotation",
                                                  "mlp")
                          if k in res}),
              flush=True)
        sys.exit(3 if bad else 0)
    steps = args.steps if "fp32" in res or "fp64" in res else args.large_steps
    bytes_per_cell = 24.0 if head is not res.get("fp64") else 48.0
    ADAPTIVE = ("shallow-water radial dam break, walled unit square, adaptive levels 3-6, "
                "m=16, regrid every 4 steps")
    LEVEL8 = ("the same dam break on the uniform level-8 forest (65,536 patches of 16x16, "
              "16.8 M cells, far beyond the 256 MB last-level cache)")

    def roof(r, bpc, profile, workload):
        """HBM roofline of the step kernel: algorithmic bytes (read and write
        every state value once) per launch over the launch time measured
        with HIP events on the launch stream."""
        alg = r["kernel_cells_mean"] * bpc
        ach = alg / (r["kernel_ms_mean"] * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
               "traffic": stored_traffic(profile) if profile else None,
               "workload": workload,
               "kernel": "k_step", "kernel_ms": r["kernel_ms_mean"],
               "bytes_per_launch": alg,
               "profile": "profiles/" + profile if profile else None}
        if profile is None:
            return out
        frac = stored_profile(profile, "valu_issue_frac")
        if frac is not None:
            out["valu_issue_frac"] = frac
            out["valu_lane_ops_per_cell"] = stored_profile(profile, "valu_lane_ops_per_cell")
        return out

    out = {
        "metric": "cell-updates/s + HBM GB/s % peak, FP32 batched vs FP64 plain, "
                  "shallow water m=16",
        "value": head["rate"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": head["seconds"] / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head is res.get("fp32") else "f64",
        "data": "synthetic",
        "config": {
            "workload": ADAPTIVE,
            "m": 16, "levels": [3, 6], "regrid_every": 4,
            "cells_per_step_mean": head["kernel_cells_mean"],
            "patches_at_end": head["patches_last"],
            "attempts": head["attempts"], "accepted": head["accepted"],
            "rejected": head["rejected"],
            "path": "fused ghost-gather + update, FP32 state, FP64 dt/CFL/sums, "
                    "reject-and-redo CFL rule; value counts accepted cell updates",
        },
        # the adaptive state (about 8 MB in FP32) lives in the 256 MB
        # last-level cache, so the HBM roofline is quoted on the same kernel
        # at uniform level 8 (16.8 M cells, 0.4 GB per step) when it ran
        "roofline": (roof(res["large32"], 24.0, "k_step_fused_sw_fp32_level8.txt", LEVEL8)
                     if "large32" in res else
                     roof(head, bytes_per_cell, "k_step_fused_sw_fp32_adaptive.txt", ADAPTIVE)),
        "roofline_adaptive": roof(head, bytes_per_cell, "k_step_fused_sw_fp32_adaptive.txt",
                                  ADAPTIVE),
        "status_bits": {k: r["status_bits"] for k, r in res.items()
                        if isinstance(r, dict) and "status_bits" in r},
    }
    if "fp64" in res:
        out["fp64_plain"] = {"value": res["fp64"]["rate"],
                             "ms_per_step": res["fp64"]["seconds"] / args.steps * 1e3,
                             "kernel_ms": res["fp64"]["kernel_ms_mean"],
                             "rejected": res["fp64"]["rejected"],
                             "roofline": roof(res["fp64"], 48.0, None, ADAPTIVE)}
        if "fp32" in res:
            out["speedup_fp32_fused_vs_fp64_plain"] = res["fp32"]["rate"] / res["fp64"]["rate"]
    if "large32" in res:
        out["large_uniform_level8"] = {
            "cells": res["large32"]["kernel_cells_mean"],
            "steps": args.large_steps,
            "fp32_fused_rate": res["large32"]["rate"],
            "fp64_plain_rate": res["large64"]["rate"],
            "speedup_fp32_fused_vs_fp64_plain": res["large32"]["rate"] / res["large64"]["rate"],
            "fp32_rel_l1_vs_fp64": res["large32"]["rel_l1_vs_fp64"],
            "fp32_roofline": roof(res["large32"], 24.0, "k_step_fused_sw_fp32_level8.txt",
                                  LEVEL8),
            "fp64_roofline": roof(res["large64"], 48.0, "k_step_plain_sw_fp64_level8.txt",
                                  LEVEL8),
        }
    if "batch" in res:
        rb = res["batch"]
        ach = rb["bytes_per_step"] / (rb["ms_per_step"] * 1e-3) / 1e9
        out["batched_64_forests"] = {
            "workload": "64 seeded forests, advection or shallow water, m in "
                        "{8,16,32}, 16..16384 patches each, levels 2-8, FP32, "
                        "one launch per tile class (a workgroup per tile, or persistent "
                        "workgroups, as the autotuner picks) in a HIP graph",
            "patches": rb["patches"], "cells": rb["cells"], "rate": rb["rate"],
            "steps": rb["steps"], "attempts": rb["attempts"], "rejected": rb["rejected"],
            "ms_per_step": rb["ms_per_step"], "tuning": rb["tuning"],
            "autotune_ms_per_step": rb["autotune_ms_per_step"],
            "hbm_GBps_algorithmic_whole_step": ach,
            "hbm_frac_whole_step": ach / HBM_PEAK_GBS,
            "status_words_nonzero": rb["status_words_nonzero"],
            "status_bits": rb["status_bits"],
        }
        prof = "k_batch_adv_fp32_16.txt"
        if stored_profile(prof, "class_us") is not None:
            # from the committed rocprofv3 summary (kernel times inside the
            # graph replays are not visible to events on the stream)
            us = stored_profile(prof, "class_us")
            out["batched_64_forests"]["advection_16x16_class"] = {
                "kernels": "k_batch_adv (simple halos) + k_batch_adv (general halos)",
                "cells": stored_profile(prof, "class_cells"), "kernel_us": us,
                "bytes_per_cell": 8.0, "hbm_frac": stored_profile(prof, "class_hbm_frac"),
                "valu_lane_ops_per_cell": stored_profile(prof, "valu_lane_ops_per_cell"),
                "source": "profiles/" + prof}
        if "batch64" in res:
            out["batched_64_forests"]["fp64_plain_same_forests"] = res["batch64"]
            out["batched_64_forests"]["speedup_vs_fp64_plain_same_forests"] = (
                rb["rate"] / res["batch64"]["rate"])
    if "sphere" in res:
        out["cubed_sphere"] = dict(res["sphere"], workload=(
            "shallow water on the cubed sphere, 6 trees, adaptive levels 4-7, m=32, "
            "seeded Gaussian height bumps, threshold set for ~50k initial patches, "
            "regrid every 8 steps (|grad h| criterion), FP32 state, FP64 geometry "
            "and sums, plain path with reflux, the library's run loop"))
        if "sphere64" in res:
            out["cubed_sphere"]["fp64_state_run"] = res["sphere64"]
    if "subcycle" in res:
        out["time_stepping"] = dict(res["subcycle"], workload=(
            ADAPTIVE + ", FP32; global dt (fused or plain steps) against per-level dt "
            "(sub-cycled, plain launches), each from t = 0"))
    if "meshing" in res:
        out["meshing_strategies"] = dict(res["meshing"], workload=(
            "the paper's advection example on one GPU with a stand-in flow (its swirl "
            "field is not given): 0/1 disk carried by a = (1, 1/2) on the periodic unit "
            "square, m = 8, levels 3-8 (uniform: level 8), max - min > 1/2 refines, "
            "CFL 0.9, FP32, to t = 0.25"))
    if "swirl" in res:
        out["example1_swirl"] = dict(res["swirl"], workload=(
            "the paper's advection example 1 with a stand-in twisting flow (the swirl "
            "stream function, reversing at T/2 = 1): 0/1 halves on the walled unit square, "
            "m = 8, levels 3-6 (uniform: level 6), max - min > 0.2 refines, CFL 0.9 with "
            "redo, FP32, over one period T = 2 (exact state: the initial one)"))
    if "rotation" in res:
        out["example2_rotation"] = dict(res["rotation"], workload=(
            "the paper's sphere example 2: 0/1 halves (split by a great circle off the tree "
            "edges) carried once around the tilted axis (0.3, -0.4, 0.866) by a rigid "
            "rotation, on the two-tree (pillow) sphere, one tree per hemisphere, m = 8, "
            "levels 3-6 (uniform: level 6), max - min > 0.2 refines, CFL 0.9 with redo, "
            "FP32, plain steps, over one turn T = 1 (exact state: the initial one)"))
    if "mlp" in res:
        out["learned_tagging_mlp"] = res["mlp"]
    if not args.no_cpu_baseline and "fp32" in res:
        out["cpu_baseline"] = cpu_baseline(args.warmup, args.steps)
    if bad:
        out["flagged_timed_legs"] = bad
    print(json.dumps(out), flush=True)
    if bad:
        print(f"timed steps carry error bits: {bad}", file=sys.stderr, flush=True)
        sys.exit(3)


if __name__ == "__main__":
    main()
