"""Offline training of the footprint network (Algorithm 1 of the paper).

Algorithm 1 draws directions uniformly on the sphere and offsets uniformly in
the part of the plane perpendicular to the direction that lies within the
maximal footprint radius, labels them with the true contribution, and fits
the MLP with Adam on the squared error until a validation error falls below
a tolerance.  This script follows those steps with these choices:

* labels: exact FP64 footprints (``footprint_net.exact_footprint``) instead
  of a projector applied to a finely sampled basis, drawn afresh for every
  few hundred steps (on the GPU when one is given, where they cost far less
  than the step itself);
* offsets: uniform in the disk of radius h*sqrt(3) (circumradius of the
  support cube) of the plane, keeping the samples whose line meets the
  support -- the kernel gates the network by that same test, so samples
  outside never matter;
* directions: 70% uniform on the sphere, 30% within 15 degrees of the
  x1-x2 plane (circular and cone-beam trajectories live there);
* inputs folded into 0 <= w1 <= w2 <= w3 (fold convention 1);
* phase 1: Adam with a short warm-up and cosine decay of the learning rate,
  FP32 arithmetic;
* phase 2: the kernel's arithmetic (hidden weights rounded to BF16 with a
  straight-through gradient, activations carried as two BF16 numbers), Adam
  at a small, decaying learning rate;
* phase 3: the hidden weights frozen at their BF16 values, the FP32
  parameters (layer 1, every bias, the output layer) refitted by L-BFGS on a
  large fixed sample;
* stopping: a fixed step budget; the reached validation relative L2 error
  (FP32, and in the kernel's arithmetic) is written into the blob header.

A run can be cut into pieces (``--time-limit`` seconds each): the state is
kept in ``--ckpt`` and the next call with the same arguments resumes it.

Several degrees train side by side, one network each, in batched products.

Usage:  python -m paper_2511_11078_amd.train_footprint --degrees 3,2,1 --device cuda \\
            --ckpt train.pt --out-dir paper_2511_11078_amd/weights
"""
from __future__ import annotations

import argparse
import math
import os
import time

import numpy as np

from . import footprint_net as fn


def sample_pairs_t(n: int, count: int, gen, device="cpu"):
    """Directions and offsets (lines meeting the support), FP64 torch
    tensors on ``device``, drawn with the torch generator ``gen``."""
    import torch

    h = 0.5 * (n + 1)
    r_s = h * math.sqrt(3.0)
    f64 = dict(dtype=torch.float64, device=device)
    ws, xs = [], []
    have = 0
    while have < count:
        m = 2 * (count - have) + 1024
        w = torch.randn(m, 3, generator=gen, **f64)
        low = torch.rand(m, generator=gen, **f64) < 0.3
        ang = torch.deg2rad((torch.rand(m, generator=gen, **f64) * 2.0 - 1.0) * 15.0)
        w[:, 2] = torch.where(low, torch.tan(ang) * torch.linalg.norm(w[:, :2], dim=1), w[:, 2])
        w = w / torch.linalg.norm(w, dim=1, keepdim=True)
        # uniform point of the disk of radius r_s in w's perpendicular plane
        a = torch.randn(m, 3, generator=gen, **f64)
        a = a - (a * w).sum(1, keepdim=True) * w
        a = a / torch.linalg.norm(a, dim=1, keepdim=True)
        rad = r_s * torch.sqrt(torch.rand(m, generator=gen, **f64))
        x = a * rad[:, None]
        keep = fn.chord_nonempty(n, w, x)
        ws.append(w[keep])
        xs.append(x[keep])
        have += int(keep.sum())
    return torch.cat(ws)[:count], torch.cat(xs)[:count]


def sample_pairs(n: int, count: int, rng) -> tuple[np.ndarray, np.ndarray]:
    """numpy form of ``sample_pairs_t`` on the host, seeded from ``rng``."""
    import torch

    gen = torch.Generator(device="cpu")
    gen.manual_seed(int(rng.integers(0, 2 ** 62)))
    w, x = sample_pairs_t(n, count, gen)
    return w.numpy(), x.numpy()


def make_dataset(n: int, count: int, seed: int, device="cpu"):
    """FP32 features and FP32 labels (FP64 exact footprints rounded once)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    w, x = sample_pairs_t(n, count, gen, device)
    y = fn.exact_footprint(n, w, x, chunk=1 << 20)
    f = fn.fold_features(w, x)
    return f.to(torch.float32), y.to(torch.float32)


def make_group_dataset(degrees, count: int, seed: int, device="cpu"):
    """Stacked datasets of several degrees: features [G, count, 5], labels [G, count]."""
    import torch

    fs, ys = [], []
    for g, n in enumerate(degrees):
        f, y = make_dataset(n, count, seed + 104729 * g, device)
        fs.append(f)
        ys.append(y)
    return torch.stack(fs), torch.stack(ys)


def rel_l2(model, f, y, quant: str, chunk: int = 1 << 18):
    """Validation relative L2 error of each network of the model."""
    import torch

    prev = model.quant
    model.quant = quant
    G = f.shape[0]
    num = torch.zeros(G, dtype=torch.float64, device=f.device)
    den = torch.zeros(G, dtype=torch.float64, device=f.device)
    with torch.no_grad():
        for s in range(0, f.shape[1], chunk):
            p = model(f[:, s:s + chunk]).double()
            t = y[:, s:s + chunk].double()
            num += ((p - t) ** 2).sum(1)
            den += (t ** 2).sum(1)
    model.quant = prev
    return [float(v) for v in torch.sqrt(num / den).cpu()]


def lr_at(step: int, steps: int, qat_steps: int, lr: float, warmup: int = 2000) -> float:
    if step < steps:
        if step < warmup:
            return lr * (step + 1) / warmup
        p = (step - warmup) / max(steps - warmup, 1)
        return 1e-7 + (lr - 1e-7) * 0.5 * (1 + math.cos(math.pi * p))
    p = (step - steps) / max(qat_steps, 1)
    return 1e-8 + (0.03 * lr) * 0.5 * (1 + math.cos(math.pi * p))


def _loss(model, f, y, inv_ms):
    """Sum over the networks of their mean squared error relative to the mean
    squared label (each network weighs the same)."""
    p = model(f)
    return (((p - y) ** 2).mean(1) * inv_ms).sum()


def refit_fp32_params(model, f, y, inv_ms, iters: int, log):
    """Freeze the hidden weights at their BF16 values and refit the FP32
    parameters (layer 1, biases, output layer) by full-batch L-BFGS in the
    kernel's arithmetic."""
    import torch

    with torch.no_grad():
        for W in model.wh:
            W.copy_(W.to(torch.bfloat16).to(torch.float32))
            W.requires_grad_(False)
    params = [model.w1, model.b1, model.wo, model.bo] + list(model.bh)
    model.quant = "split"
    opt = torch.optim.LBFGS(params, lr=1.0, max_iter=iters, history_size=50, tolerance_grad=0.0,
                            tolerance_change=0.0, line_search_fn="strong_wolfe")
    chunk = 1 << 19
    nchunks = (f.shape[1] + chunk - 1) // chunk

    def closure():
        opt.zero_grad(set_to_none=True)
        total = 0.0
        for s in range(0, f.shape[1], chunk):
            loss = _loss(model, f[:, s:s + chunk], y[:, s:s + chunk], inv_ms) / nchunks
            loss.backward()
            total += float(loss.detach())
        return torch.tensor(total)

    loss = opt.step(closure)
    log(f"refit: {iters} L-BFGS iterations, relative loss {float(loss):.3e}")
    for W in model.wh:
        W.requires_grad_(True)


def train(degrees, steps: int, qat_steps: int, batch: int, lr: float, seed: int, out_dir: str, threads: int,
          pool: int, device: str, ckpt: str | None, time_limit: float, refit_iters: int, refit_samples: int,
          log=print):
    """Train one network per degree, side by side; write mlp_n<degree>.bin
    into out_dir when the step budget is reached (None before that)."""
    import torch

    torch.set_num_threads(threads)
    torch.manual_seed(seed)
    dev = torch.device(device)
    degrees = [int(d) for d in degrees]
    model = fn.make_torch_model(degrees).to(dev)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    start = 0
    if ckpt and os.path.exists(ckpt):
        st = torch.load(ckpt, map_location=dev, weights_only=True)
        model.load_state_dict(st["model"])
        opt.load_state_dict(st["opt"])
        start = int(st["step"])
        log(f"resumed from {ckpt} at step {start}")
    fval, yval = make_group_dataset(degrees, 1_000_000, seed + 1000, dev)
    inv_ms = 1.0 / (yval.double() ** 2).mean(1).float()
    total = steps + qat_steps
    t0 = time.time()
    last_log = -1e9
    pool_every = max(1, pool // batch)
    gen = torch.Generator(device=dev)
    step = start
    fpool = ypool = None

    def fmt(v):
        return " ".join(f"n{d}:{e:.3e}" for d, e in zip(degrees, v))

    while step < total:
        if fpool is None or (step - start) % pool_every == 0:
            fpool, ypool = make_group_dataset(degrees, pool, seed + 7919 * step + 1, dev)
            gen.manual_seed(seed + step)
        model.quant = "split" if step >= steps else "fp32"
        cur = lr_at(step, steps, qat_steps, lr)
        for g in opt.param_groups:
            g["lr"] = cur
        idx = torch.randint(0, fpool.shape[1], (batch,), generator=gen, device=dev)
        loss = _loss(model, fpool[:, idx], ypool[:, idx], inv_ms)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        step += 1
        now = time.time() - t0
        if step % 20000 == 0 or step == total or now - last_log > 30.0:
            last_log = now
            log(f"step {step:7d}/{total} lr {cur:.2e} loss {loss.item():.3e} "
                f"val fp32 [{fmt(rel_l2(model, fval, yval, 'fp32'))}] "
                f"kernel [{fmt(rel_l2(model, fval, yval, 'split'))}] t {now:.0f}s")
        if ckpt and (now > time_limit or step == total):
            torch.save({"model": model.state_dict(), "opt": opt.state_dict(), "step": step}, ckpt)
            if step < total:
                log(f"time limit: state saved to {ckpt} at step {step}")
                return None
    if refit_iters > 0:
        fr, yr = make_group_dataset(degrees, refit_samples, seed + 2000, dev)
        before = rel_l2(model, fval, yval, "split")
        saved = {k: v.clone() for k, v in model.state_dict().items()}
        refit_fp32_params(model, fr, yr, inv_ms, refit_iters, log)
        after = rel_l2(model, fval, yval, "split")
        log(f"refit: validation rel-L2 in the kernel's arithmetic [{fmt(before)}] -> [{fmt(after)}]")
        if not sum(a * a for a in after) < sum(b * b for b in before):
            model.load_state_dict(saved)
            log("refit: not kept")
    model.quant = "fp32"
    r32 = rel_l2(model, fval, yval, "fp32")
    rq = rel_l2(model, fval, yval, "split")
    r1 = rel_l2(model, fval, yval, "bf16")
    os.makedirs(out_dir, exist_ok=True)
    for g, n in enumerate(degrees):
        blob = fn.model_to_blob(model, n, seed, r32[g], rq[g], g=g)
        path = os.path.join(out_dir, f"mlp_n{n}.bin")
        with open(path, "wb") as fh:
            fh.write(blob)
        log(f"wrote {path}: val rel-L2 fp32 {r32[g]:.3e}, kernel arithmetic {rq[g]:.3e} "
            f"(activations rounded once to BF16: {r1[g]:.3e})")
    return model


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--degrees", default="3", help="comma-separated degrees, trained side by side")
    ap.add_argument("--steps", type=int, default=300000)
    ap.add_argument("--qat-steps", type=int, default=30000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=1.5e-3)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--pool", type=int, default=4_000_000)
    ap.add_argument("--device", default="cpu")
    ap.add_argument("--ckpt", default=None, help="state file for runs cut into pieces")
    ap.add_argument("--time-limit", type=float, default=float("inf"), help="seconds before saving and stopping")
    ap.add_argument("--refit-iters", type=int, default=300)
    ap.add_argument("--refit-samples", type=int, default=2_000_000)
    ap.add_argument("--out-dir", required=True, help="where mlp_n<degree>.bin are written")
    a = ap.parse_args()
    train([int(d) for d in a.degrees.split(",")], a.steps, a.qat_steps, a.batch, a.lr, a.seed, a.out_dir,
          a.threads, a.pool, a.device, a.ckpt, a.time_limit, a.refit_iters, a.refit_samples,
          log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
