"""Adaptive shallow-water runs driven entirely through libfcx.so.

A run is the radial dam break in the walled unit square (reflecting walls,
g = 1, fluid at rest, h = h_in inside a disc, 1 outside) on a 2:1-balanced
forest between two levels, with patches tagged by the |grad h| criterion
(Sec. 5 tags a patch when its criterion passes a threshold; here the
criterion is the largest central-difference gradient of h).  Every kernel
of a step and of a regrid runs in the library; this module only sequences
the calls and owns the device buffers (torch tensors).

Tagging modes at a regrid step:
  "plain"   -- the criterion tags;
  "learned" -- the network's tags with the criterion as fallback;
both optionally followed by the one-patch refinement buffer, for tags that
stay in use for several steps.
"""
from __future__ import annotations

import numpy as np

from . import fcx
from . import inputs as I


class DamBreak:
    """One adaptive (or uniform) dam break on the current HIP device."""

    def __init__(self, precision=64, m=16, lmin=3, lmax=6, threshold=0.1,
                 centre=(0.5, 0.5), radius=0.25, h_in=2.0, uniform_level=None,
                 fused=True):
        import torch
        self.torch = torch
        self.m, self.lmin, self.lmax, self.thr = m, lmin, lmax, threshold
        self.fused = fused
        self.trees, self.pl = I.walled_square()
        self.cfg = fcx.config(m, precision, fcx.FCX_SHALLOW, cfl_desired=0.9,
                              cfl_max=1.0)
        self.ctx = fcx.Context(self.cfg, self.trees)
        self.dtype = torch.float64 if precision == 64 else torch.float32
        cx, cy = centre
        self.fn = lambda x, y: I.dam_break(x, y, cx, cy, radius, h_in)
        if uniform_level is not None:
            leaves = fcx.sfc_sort(I.uniform_leaves(1, uniform_level))
        else:
            # initial mesh: tag the initial data, refine, evaluate again on
            # the new leaves, until nothing changes
            leaves = fcx.sfc_sort(I.uniform_leaves(1, lmin))
            for _ in range(2 * (lmax - lmin) + 2):
                self.ctx.upload_forest(leaves)
                self._alloc()
                self._set(I.state_from(leaves, m, self.fn, self.pl))
                self.ctx.regrid_apply(self.plain_tags().cpu().numpy(), lmin, lmax)
                new = self.ctx.leaves()
                if len(new) == len(leaves) and (new == leaves).all():
                    break
                leaves = new
        self.ctx.upload_forest(leaves)
        self._alloc()
        self._set(I.state_from(leaves, m, self.fn, self.pl))
        dev = "cuda"
        self.dt = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dt_probe = torch.zeros(1, dtype=torch.float64, device=dev)
        self.numax = torch.zeros(1, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.steps = 0
        self.regrids = 0
        self.patch_steps = 0

    # ---- buffers --------------------------------------------------------
    def _alloc(self):
        t = self.torch
        P = self.ctx.num_patches()
        self.q = t.empty(self.ctx.state_elems(), dtype=self.dtype, device="cuda")
        self.qn = t.empty_like(self.q)
        self.ghost = t.empty(self.ctx.ghost_elems(), dtype=self.dtype, device="cuda")
        self.tags = t.empty(P, dtype=t.int8, device="cuda")
        self.tags2 = t.empty(P, dtype=t.int8, device="cuda")
        self.feats = t.empty(P * fcx.MLP_INPUTS, dtype=t.float32, device="cuda")
        self.logits = t.empty(P * fcx.MLP_CLASSES, dtype=t.float32, device="cuda")

    def _set(self, q):
        self.q.copy_(self.torch.from_numpy(np.ascontiguousarray(q).ravel()).to(self.dtype))

    def num_patches(self):
        return self.ctx.num_patches()

    def leaves(self):
        return self.ctx.leaves()

    def state(self):
        P = self.num_patches()
        return self.q.double().cpu().numpy().reshape(P, 3, self.m, self.m)

    # ---- tags -----------------------------------------------------------
    def plain_tags(self):
        """Criterion tags of the current state (device int8; also leaves a
        ghost fill of q in self.ghost)."""
        self.ctx.ghost_fill(self.q, self.ghost)
        self.ctx.regrid_tags(self.q, self.ghost, 1, self.thr, self.lmin, self.lmax,
                             self.tags)
        return self.tags

    def features(self):
        """(P, 16) per-patch statistics of the current state (device)."""
        self.ctx.ghost_fill(self.q, self.ghost)
        self.ctx.features(self.q, self.ghost, self.feats)
        return self.feats.view(-1, fcx.MLP_INPUTS)

    def learned_tags(self, net, confidence=0.6):
        """Network tags with the criterion as fallback (device int8)."""
        plain = self.plain_tags()
        self.ctx.features(self.q, self.ghost, self.feats)
        fcx.mlp_forward(net.params, net.norm, self.feats, self.logits)
        fcx.learned_tags(self.logits, plain, confidence, self.tags2)
        self.tags, self.tags2 = self.tags2, self.tags
        return self.tags

    def dilate(self, tags):
        out = self.tags2 if tags.data_ptr() == self.tags.data_ptr() else self.tags
        self.ctx.dilate_tags(tags, self.lmax, out)
        return out

    def regrid(self, tags_dev):
        """Refine / coarsen / balance from device tags, then transfer."""
        tags_host = tags_dev.cpu().numpy()
        self.ctx.ghost_fill(self.q, self.ghost)
        q_old, g_old = self.q, self.ghost
        self.ctx.regrid_apply(tags_host, self.lmin, self.lmax)
        self._alloc()
        self.ctx.regrid_transfer(q_old, g_old, self.q)
        self.regrids += 1

    # ---- time stepping --------------------------------------------------
    def set_dt(self, dt):
        self.dt.fill_(dt)

    def step(self):
        """One step with the fixed dt: ghost fill + update (fused or not),
        coarse-fine reflux; the CFL check goes into self.status."""
        if self.fused:
            self.ctx.fused_step(self.q, self.qn, self.dt, self.numax)
        else:
            self.ctx.ghost_fill(self.q, self.ghost)
            self.ctx.patch_step(self.q, self.ghost, self.qn, self.dt, self.numax)
        self.ctx.reflux(self.q, self.qn, self.dt)
        # the probe dt absorbs the adaptive update; only the flags matter
        self.ctx.next_dt(self.numax, self.dt_probe, self.status)
        self.q, self.qn = self.qn, self.q
        self.steps += 1
        self.patch_steps += self.ctx.num_patches()


def run(sim: DamBreak, dt: float, nsteps: int, every: int, mode="plain",
        net=None, dilate=False, confidence=0.6, on_regrid=None):
    """Advance nsteps with a regrid every `every` steps (none at step 0)."""
    sim.set_dt(dt)
    for n in range(nsteps):
        if n > 0 and n % every == 0:
            if on_regrid is not None:
                on_regrid(sim, n)
            tags = sim.plain_tags() if mode == "plain" else sim.learned_tags(net, confidence)
            if dilate:
                tags = sim.dilate(tags)
            sim.regrid(tags)
        sim.step()
    return sim


def project_uniform(ref_state, ref_level, leaves, m):
    """Conservative average of a uniform-level solution (P_ref, meqn, m, m in
    SFC order of one tree) onto the cells of an adaptive forest."""
    n = (1 << ref_level) * m
    P, meqn = ref_state.shape[:2]
    ref_leaves = fcx.sfc_sort(I.uniform_leaves(1, ref_level))
    img = np.empty((meqn, n, n))
    for p, a in enumerate(ref_leaves):
        img[:, a["iy"] * m:(a["iy"] + 1) * m, a["ix"] * m:(a["ix"] + 1) * m] = ref_state[p]
    out = np.empty((len(leaves), meqn, m, m))
    for p, a in enumerate(leaves):
        r = 1 << (ref_level - int(a["level"]))          # ref cells per cell side
        x0, y0 = a["ix"] * m * r, a["iy"] * m * r
        blk = img[:, y0:y0 + m * r, x0:x0 + m * r]
        out[p] = blk.reshape(meqn, m, r, m, r).mean(axis=(2, 4))
    return out


def l1_error(state, leaves, m, ref_proj, comp=0):
    """sum |q - q_ref| * cell area over the forest, component comp."""
    area = np.ldexp(1.0, -2 * leaves["level"].astype(np.int64)) / (m * m)
    d = np.abs(state[:, comp] - ref_proj[:, comp]).sum(axis=(1, 2))
    return float((d * area).sum())
