"""Learned tagging: data from seeded adaptive dam-break runs, training of the
tag network on the GPU with the library's own bfloat16 MFMA kernels, and
the comparison of regridding policies.

Data.  Each seed gives a dam break (inputs.dam_break_spec) on levels 3..6
with m = 16, tagged by |grad h| > 0.1.  In a run that regrids every E steps
with the criterion, the mesh is fixed from a regrid at step n until step
n + E; the features of every patch right after the regrid at n are paired
with the criterion's tag of the same patch at n + h (h = 4: "n+4" labels),
or with the union of the tags at n + 4, 8, 12, 16 (E = 16: "or16" labels:
refine if any is +1, coarsen if all are -1, else keep).  Classes: 0 refine,
1 keep, 2 coarsen.

Training.  Inputs are standardised with the training set's mean and
standard deviation (kept with the weights).  Weighted softmax
cross-entropy with inverse-frequency class weights, Adam (lr 1e-3,
betas 0.9 / 0.999), fixed seeds; forward, backward and Adam are library
kernels (fcx_mlp_backward, fcx_adam_step).

Policies compared on held-out seeds (same fixed dt for all):
  (i)   criterion every 4 steps;
  (ii)  criterion every 16 steps, with the one-patch refinement buffer;
  (iii) network every 16 steps with the criterion as fallback, with the
        buffer.
Error: L1 of h against a uniform level-7 FP64 run (dt / 2, twice the
steps) averaged conservatively onto each adaptive mesh.

`python -m paper_1308_1472_amd.learned train` writes the weights file;
`... evaluate` prints the comparison as JSON.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import amr, fcx
from . import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "tagger.npz")

M, LMIN, LMAX, THR = 16, 3, 6, 0.1
C_EST = 2.5          # bound on |u| + sqrt(g h) for h_in <= 3 (fixed dt rule)
NSTEPS = 320
TRAIN_SEEDS = range(0, 180)
TEST_SEEDS = range(180, 200)


def fixed_dt(level=LMAX):
    """dt with Courant number <= 0.8 on the finest level for any seed."""
    return 0.8 / (M << level) / C_EST


class Net:
    """Parameters and normalisation on the device (FP32)."""

    def __init__(self, params, norm):
        import torch
        self.params = torch.as_tensor(np.asarray(params, np.float32)).cuda().contiguous()
        self.norm = torch.as_tensor(np.asarray(norm, np.float32)).cuda().contiguous()

    @staticmethod
    def init(seed, norm):
        """He-style random initialisation."""
        rng = np.random.default_rng(seed)
        ni, nh, no = fcx.MLP_INPUTS, fcx.MLP_HIDDEN, fcx.MLP_CLASSES
        P = np.concatenate([
            rng.normal(0, np.sqrt(2 / ni), ni * nh), np.zeros(nh),
            rng.normal(0, np.sqrt(2 / nh), nh * nh), np.zeros(nh),
            rng.normal(0, np.sqrt(1 / nh), nh * no), np.zeros(no)])
        return Net(P, norm)

    def save(self, path, meta):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        np.savez(path, params=self.params.cpu().numpy(), norm=self.norm.cpu().numpy(),
                 meta=np.array(json.dumps(meta)))

    @staticmethod
    def load(path=WEIGHTS):
        z = np.load(path, allow_pickle=False)
        return Net(z["params"], z["norm"]), json.loads(str(z["meta"]))


def _sim(seed, precision=64):
    s = I.dam_break_spec(seed)
    return amr.DamBreak(precision, M, LMIN, LMAX, THR, s["centre"], s["radius"], s["h_in"])


def collect(seed, labels="n+4", nsteps=NSTEPS, keep_every=4):
    """(features (R, 16) float32, classes (R,) int32) of one seed; keeps the
    samples of every `keep_every`-th regrid point."""
    import torch
    every, hs = (4, (4,)) if labels == "n+4" else (16, (4, 8, 12, 16))
    sim = _sim(seed)
    sim.set_dt(fixed_dt())
    feats, ys = [], []
    pend = None                     # (features, tags so far) on the current mesh
    point = 0
    for n in range(nsteps + 1):
        if pend is not None and (n - pend[2]) in hs:
            pend[1].append(sim.plain_tags().clone())
            if len(pend[1]) == len(hs):
                t = torch.stack(pend[1]).to(torch.int32)
                if len(hs) == 1:
                    tag = t[0]
                else:
                    tag = torch.where((t == 1).any(0), 1,
                                      torch.where((t == -1).all(0), -1, 0))
                feats.append(pend[0])
                ys.append((1 - tag).to(torch.int32))
                pend = None
        if n == nsteps:
            break
        if n % every == 0:
            if n > 0:
                sim.regrid(sim.plain_tags())
            if point % keep_every == 0:
                pend = (sim.features().clone(), [], n)
            point += 1
        sim.step()
    if not feats:
        return np.zeros((0, 16), np.float32), np.zeros(0, np.int32)
    return (torch.cat(feats).cpu().numpy(), torch.cat(ys).cpu().numpy())


def train(X, Y, epochs=32, batch=8192, lr=1e-3, seed=0, log=None):
    """Trains a fresh network on (X, Y) with the library kernels."""
    import torch
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 1e-12, sd, 1.0)
    net = Net.init(seed, np.concatenate([mu, sd]))
    counts = np.bincount(Y, minlength=3).astype(np.float64)
    cw = np.where(counts > 0, counts.sum() / (3 * np.maximum(counts, 1)), 0.0)
    cw_d = torch.tensor(cw, dtype=torch.float32, device="cuda")
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    Yd = torch.from_numpy(np.ascontiguousarray(Y, np.int32)).cuda()
    n = len(X)
    grad = torch.zeros(fcx.MLP_PARAMS, device="cuda")
    loss = torch.zeros(1, device="cuda")
    m1, m2 = torch.zeros_like(grad), torch.zeros_like(grad)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    t = 0
    hist = [evaluate_loss(net, Xd, Yd, cw_d)]
    batch = min(batch, n)
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb, yb = Xd[idx].contiguous(), Yd[idx].contiguous()
            fcx.mlp_backward(net.params, net.norm, xb, yb, cw_d, 1.0 / batch, grad, loss)
            t += 1
            fcx.adam_step(net.params, grad, m1, m2, t, lr=lr)
        hist.append(evaluate_loss(net, Xd, Yd, cw_d))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return net, {"class_weight": cw.tolist(), "loss_per_epoch": hist, "steps": t,
                 "rows": int(n)}


def evaluate_loss(net, Xd, Yd, cw_d):
    import torch
    grad = torch.zeros(fcx.MLP_PARAMS, device="cuda")
    loss = torch.zeros(1, device="cuda")
    fcx.mlp_backward(net.params, net.norm, Xd, Yd, cw_d, 1.0 / len(Xd), grad, loss)
    return float(loss.item())


def predict(net, X):
    import torch
    Xd = torch.as_tensor(np.ascontiguousarray(X, np.float32)).cuda()
    z = torch.empty(len(X), 3, dtype=torch.float32, device="cuda")
    fcx.mlp_forward(net.params, net.norm, Xd, z)
    return z.cpu().numpy()


def compare(seed, net, nsteps=NSTEPS, confidence=0.6, ref_cache=None):
    """Errors, regrid counts and times of the three policies for one seed."""
    import torch
    s = I.dam_break_spec(seed)
    dt = fixed_dt()
    ref = ref_cache.get(seed) if ref_cache is not None else None
    if ref is None:
        r = amr.DamBreak(64, M, LMIN, LMAX + 1, THR, s["centre"], s["radius"], s["h_in"],
                         uniform_level=LMAX + 1)
        amr.run(r, dt / 2, 2 * nsteps, every=1 << 30)
        ref = r.state()
        if ref_cache is not None:
            ref_cache[seed] = ref
    out = {}
    for name, every, mode, dil in (("plain4", 4, "plain", False),
                                   ("plain16", 16, "plain", True),
                                   ("learned16", 16, "learned", True)):
        sim = _sim(seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        amr.run(sim, dt, nsteps, every, mode, net, dil, confidence)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        lv = sim.leaves()
        proj = amr.project_uniform(ref, LMAX + 1, lv, M)
        out[name] = {"l1_h": amr.l1_error(sim.state(), lv, M, proj),
                     "regrids": sim.regrids, "seconds": el,
                     "patch_steps": sim.patch_steps,
                     "patches_end": int(len(lv)), "status": int(sim.status.item())}
    return out


def mismatch(net, X, Y):
    """Fraction of patches whose most likely class differs from the label."""
    z = predict(net, X)
    return float((z.argmax(axis=1) != Y).mean())


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1308_1472_amd.learned")
    ap.add_argument("cmd", choices=["train", "evaluate"])
    ap.add_argument("--labels", choices=["n+4", "or16"], default="n+4")
    ap.add_argument("--train-seeds", type=int, default=len(TRAIN_SEEDS))
    ap.add_argument("--test-seeds", type=int, default=len(TEST_SEEDS))
    ap.add_argument("--epochs", type=int, default=32)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args(argv)
    say = lambda *x: print(*x, file=sys.stderr, flush=True)
    if a.cmd == "train":
        t0 = time.perf_counter()
        Xs, Ys = [], []
        for k, s in enumerate(list(TRAIN_SEEDS)[:a.train_seeds]):
            x, y = collect(s, a.labels)
            Xs.append(x)
            Ys.append(y)
            if k % 20 == 0:
                say(f"seed {s}: {len(x)} rows")
        X, Y = np.concatenate(Xs), np.concatenate(Ys)
        t1 = time.perf_counter()
        net, info = train(X, Y, epochs=a.epochs, log=say)
        t2 = time.perf_counter()
        Xt, Yt = [], []
        for s in list(TEST_SEEDS)[:a.test_seeds]:
            x, y = collect(s, a.labels)
            Xt.append(x)
            Yt.append(y)
        Xt, Yt = np.concatenate(Xt), np.concatenate(Yt)
        info.update({"labels": a.labels, "train_seeds": a.train_seeds,
                     "collect_s": t1 - t0, "train_s": t2 - t1,
                     "class_counts": np.bincount(Y, minlength=3).tolist(),
                     "test_mismatch": mismatch(net, Xt, Yt),
                     "test_rows": int(len(Xt))})
        net.save(a.out, info)
        print(json.dumps(info))
    else:
        net, meta = Net.load(a.out)
        rows = []
        for s in list(TEST_SEEDS)[:a.test_seeds]:
            r = compare(s, net)
            rows.append(r)
            say(json.dumps({"seed": s, **{k: v["l1_h"] for k, v in r.items()}}))
        agg = {k: {f: float(np.mean([r[k][f] for r in rows]))
                   for f in ("l1_h", "regrids", "seconds", "patch_steps")}
               for k in rows[0]}
        print(json.dumps({"labels": meta.get("labels"), "seeds": len(rows), **agg}))


if __name__ == "__main__":
    main()
