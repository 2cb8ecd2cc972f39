"""Offline training of the footprint network (Algorithm 1 of the paper).

Algorithm 1 draws directions uniformly on the sphere and offsets uniformly in
the part of the plane perpendicular to the direction that lies within the
maximal footprint radius, labels them with the true contribution, and fits
the MLP with Adam on the squared error until a validation error falls below
a tolerance.  This script follows those steps with these choices:

* labels: exact FP64 footprints (``footprint_net.exact_footprint``) instead
  of a projector applied to a finely sampled basis;
* offsets: uniform in the disk of radius h*sqrt(3) (circumradius of the
  support cube) of the plane, keeping the samples whose line meets the
  support -- the kernel gates the network by that same test, so samples
  outside never matter;
* directions: 70% uniform on the sphere, 30% within 15 degrees of the
  x1-x2 plane (circular and cone-beam trajectories live there);
* inputs folded into 0 <= w1 <= w2 <= w3 (fold convention 1);
* Adam, cosine learning-rate decay, fresh samples each step from a
  regenerated pool, then a short quantisation-aware phase that rounds the
  hidden weights and the activations entering them to BF16;
* stopping: a fixed step budget; the reached validation relative L2 error
  (FP32 and BF16-quantised) is written into the blob header.

Usage:  python -m paper_2511_11078_amd.train_footprint --degree 3 --out weights/mlp_n3.bin

The shipped degree-3 and degree-2 weights used --steps 80000 --qat-steps 8000
--batch 32768 --lr 2e-3 --threads 6 --pool 2000000 (about 60-70 minutes each
on 6 host cores).
"""
from __future__ import annotations

import argparse
import math
import os
import time

import numpy as np

from . import footprint_net as fn


def sample_pairs(n: int, count: int, rng) -> tuple[np.ndarray, np.ndarray]:
    """Directions and offsets (lines meeting the support), FP64."""
    h = 0.5 * (n + 1)
    r_s = h * math.sqrt(3.0)
    ws, xs = [], []
    have = 0
    while have < count:
        m = 2 * (count - have) + 1024
        w = rng.standard_normal((m, 3))
        low = rng.random(m) < 0.3
        w[low, 2] = np.tan(np.deg2rad(rng.uniform(-15.0, 15.0, low.sum()))) * np.linalg.norm(w[low, :2], axis=1)
        w /= np.linalg.norm(w, axis=1, keepdims=True)
        # uniform point of the disk of radius r_s in w's perpendicular plane
        a = rng.standard_normal((m, 3))
        a -= (a * w).sum(1, keepdims=True) * w
        a /= np.linalg.norm(a, axis=1, keepdims=True)
        rad = r_s * np.sqrt(rng.random(m))
        x = a * rad[:, None]
        keep = fn.chord_nonempty(n, w, x)
        ws.append(w[keep])
        xs.append(x[keep])
        have += int(keep.sum())
    return np.concatenate(ws)[:count], np.concatenate(xs)[:count]


def make_dataset(n: int, count: int, seed: int):
    rng = np.random.default_rng(seed)
    w, x = sample_pairs(n, count, rng)
    y = fn.exact_footprint(n, w, x)
    f = fn.fold_features(w, x)
    return f.astype(np.float32), y.astype(np.float32)


def rel_l2(model, f, y, quant: bool, chunk: int = 1 << 16) -> float:
    import torch

    model.quant = quant
    num = den = 0.0
    with torch.no_grad():
        for s in range(0, f.shape[0], chunk):
            p = model(torch.from_numpy(f[s:s + chunk])).double().numpy()
            t = y[s:s + chunk].astype(np.float64)
            num += ((p - t) ** 2).sum()
            den += (t ** 2).sum()
    model.quant = False
    return math.sqrt(num / den)


def train(n: int, steps: int, qat_steps: int, batch: int, lr: float, seed: int, out: str,
          threads: int, pool: int, log=print):
    import torch

    torch.set_num_threads(threads)
    torch.manual_seed(seed)
    model = fn.make_torch_model(n)
    fval, yval = make_dataset(n, 200_000, seed + 1000)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    total = steps + qat_steps
    t0 = time.time()
    fpool = ypool = None
    for step in range(total):
        if step % 2000 == 0:
            fpool, ypool = make_dataset(n, pool, seed + step)
            fpool_t = torch.from_numpy(fpool)
            ypool_t = torch.from_numpy(ypool)
        if step < steps:
            cur = lr * (0.01 + 0.99 * 0.5 * (1 + math.cos(math.pi * step / steps)))
        else:
            model.quant = True
            cur = lr * 0.02 * (1 - (step - steps) / max(qat_steps, 1)) + 1e-6
        for g in opt.param_groups:
            g["lr"] = cur
        idx = torch.randint(0, fpool.shape[0], (batch,))
        pred = model(fpool_t[idx])
        loss = torch.mean((pred - ypool_t[idx]) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        if step % 1000 == 0 or step == total - 1:
            r32 = rel_l2(model, fval, yval, False)
            rq = rel_l2(model, fval, yval, True)
            model.quant = step >= steps
            log(f"step {step:6d} lr {cur:.2e} loss {loss.item():.3e} val_rel_fp32 {r32:.3e} "
                f"val_rel_bf16 {rq:.3e} t {time.time() - t0:.0f}s")
    model.quant = False
    r32 = rel_l2(model, fval, yval, False)
    rq = rel_l2(model, fval, yval, True)
    blob = fn.model_to_blob(model, n, seed, r32, rq)
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "wb") as fh:
        fh.write(blob)
    log(f"wrote {out}: val rel-L2 fp32 {r32:.3e} bf16 {rq:.3e}")
    return model


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--qat-steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--pool", type=int, default=1_000_000)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    train(a.degree, a.steps, a.qat_steps, a.batch, a.lr, a.seed, a.out, a.threads, a.pool,
          log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
