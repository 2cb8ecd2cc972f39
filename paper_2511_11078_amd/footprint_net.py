"""The learned footprint f_theta of Sec. 2.2 (Algorithm 1) -- model, inputs, blob.

The paper replaces the closed-form contribution P phi(w, s) of one basis to
one line by a shallow MLP taking the direction w and the in-plane offset s.
Here the network is 5 -> 64 -> 64 -> 64 -> 64 -> 1 with SiLU after each of
the four hidden layers (12,929 parameters).

Inputs (fold convention 1).  phi is invariant under the 48 signed
permutations Q of the axes, so P phi(Q w, Q x) = P phi(w, x).  Every (w, x)
is first mapped by the Q that sorts |w| ascending and makes it non-negative,
giving 0 <= w1 <= w2 <= w3.  In that region e1 is never close to w, so the
in-plane frame u = normalise(e1 - w1 w), v = u x w (the frame of the paper's
projection algorithm, u perpendicular to w, v = u x w) is continuous.  The
five features are (w1, w2, w3, u.x, v.x); x is any point of the line relative
to the basis centre.

Precision split used by the GPU kernel: fold, frame and layer 1 in FP32; the
three 64x64 layers take BF16 operands with FP32 accumulation; SiLU in FP32;
the output layer in FP32.  The kernel multiplies the network output by the
indicator that the line meets the basis support (an exact slab test), so the
network is only ever used where the true footprint can be non-zero.

Training labels come from ``exact_footprint`` below: an FP64 vectorised
piecewise Gauss-Legendre integral (exact for B-splines, see the module
docstring of ``train_footprint``), written for training only.
"""
from __future__ import annotations

import struct

import numpy as np

MAGIC = b"SSMLP\x00\x00\x01"
VERSION = 1
FOLD_ID = 1
ACT_SILU = 1
IN_DIM, HIDDEN, DEPTH = 5, 64, 4
HEADER_FMT = "<8sIIIIIIIIff"   # magic, version, degree, in, hidden, depth, act, fold, seed, rel_fp32, rel_bf16
HEADER_BYTES = struct.calcsize(HEADER_FMT)


def blob_bytes() -> int:
    body = 4 * (HIDDEN * IN_DIM + HIDDEN)                  # layer 1, FP32
    body += (DEPTH - 1) * (2 * HIDDEN * HIDDEN + 4 * HIDDEN)  # hidden, BF16 W + FP32 b
    body += 4 * (HIDDEN + 1)                                 # output, FP32
    return HEADER_BYTES + body


# --------------------------------------------------------------------------
# folding and features (numpy, FP64 -- for training data)
# --------------------------------------------------------------------------
def fold_features(w: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(w, x) [B, 3] -> features [B, 5] of fold convention 1."""
    w = np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    aw = np.abs(w)
    perm = np.argsort(aw, axis=1, kind="stable")          # ascending |w|
    rows = np.arange(w.shape[0])[:, None]
    sgn = np.where(w[rows, perm] < 0, -1.0, 1.0)
    wf = aw[rows, perm]
    xf = x[rows, perm] * sgn
    u = -wf[:, 0:1] * wf
    u[:, 0] += 1.0
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(u, wf)
    return np.concatenate([wf, (u * xf).sum(1, keepdims=True), (v * xf).sum(1, keepdims=True)], axis=1)


def chord_nonempty(n: int, w: np.ndarray, x: np.ndarray) -> np.ndarray:
    h = 0.5 * (n + 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = (-h - x) / w
        tb = (h - x) / w
    lo = np.where(w == 0, np.where(np.abs(x) < h, -np.inf, np.inf), np.minimum(ta, tb))
    hi = np.where(w == 0, np.where(np.abs(x) < h, np.inf, -np.inf), np.maximum(ta, tb))
    return lo.max(1) < hi.min(1)


# --------------------------------------------------------------------------
# FP64 training labels
# --------------------------------------------------------------------------
def _bspline(n: int, x: np.ndarray) -> np.ndarray:
    a = np.abs(x)
    if n == 0:
        return (a < 0.5).astype(np.float64)
    if n == 1:
        return np.maximum(1.0 - a, 0.0)
    if n == 2:
        return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))
    if n == 3:
        return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3, np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))
    raise ValueError(n)


def exact_footprint(n: int, w: np.ndarray, x: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
    """int phi(x + t w) dt for unit w, in FP64: clip to the support cube, cut
    at the interior knot planes, Gauss-Legendre of order ceil((3n+1)/2) on
    each piece (exact, the integrand being a polynomial of degree 3n there)."""
    w = np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(w.shape[0])
    h = 0.5 * (n + 1)
    m = max(1, (3 * n + 2) // 2)
    gx, gw = np.polynomial.legendre.leggauss(m)
    knots = -h + np.arange(1, n + 1, dtype=np.float64)
    for s in range(0, w.shape[0], chunk):
        W = w[s:s + chunk]
        X = x[s:s + chunk]
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (-h - X) / W
            tb = (h - X) / W
            lo = np.where(W == 0, np.where(np.abs(X) < h, -np.inf, np.inf), np.minimum(ta, tb))
            hi = np.where(W == 0, np.where(np.abs(X) < h, np.inf, -np.inf), np.maximum(ta, tb))
            t0 = lo.max(1)
            t1 = hi.min(1)
            valid = t0 < t1
            t0 = np.where(valid, t0, 0.0)
            t1 = np.where(valid, t1, 0.0)
            T = (knots[None, None, :] - X[:, :, None]) / W[:, :, None]
        T = np.where(np.isfinite(T), T, t0[:, None, None])
        T = np.clip(T, t0[:, None, None], t1[:, None, None]).reshape(W.shape[0], -1)
        T = np.sort(np.concatenate([t0[:, None], T, t1[:, None]], axis=1), axis=1)
        mid = 0.5 * (T[:, 1:] + T[:, :-1])
        half = 0.5 * (T[:, 1:] - T[:, :-1])
        t = mid[..., None] + half[..., None] * gx                       # [B, S, m]
        pos = X[:, None, None, :] + t[..., None] * W[:, None, None, :]  # [B, S, m, 3]
        val = _bspline(n, pos).prod(-1)
        seg = (val * gw).sum(-1) * half
        out[s:s + chunk] = np.where(valid, seg.sum(-1), 0.0)
    return out


# --------------------------------------------------------------------------
# torch model (training and FP32 reference evaluation)
# --------------------------------------------------------------------------
def feature_scale(n: int):
    """Fixed affine map of the raw features to roughly [-1, 1]."""
    h = 0.5 * (n + 1)
    r = h * np.sqrt(3.0)
    lo = np.array([0.0, 0.0, 1.0 / np.sqrt(3.0), -r, -r])
    hi = np.array([1.0 / np.sqrt(3.0), 1.0 / np.sqrt(2.0), 1.0, r, r])
    scale = 2.0 / (hi - lo)
    shift = -1.0 - lo * scale
    return scale, shift


def make_torch_model(n: int):
    import torch
    from torch import nn

    class FootprintMLP(nn.Module):
        def __init__(self):
            super().__init__()
            sc, sh = feature_scale(n)
            self.register_buffer("in_scale", torch.tensor(sc, dtype=torch.float32))
            self.register_buffer("in_shift", torch.tensor(sh, dtype=torch.float32))
            self.l1 = nn.Linear(IN_DIM, HIDDEN)
            self.hidden = nn.ModuleList([nn.Linear(HIDDEN, HIDDEN) for _ in range(DEPTH - 1)])
            self.out = nn.Linear(HIDDEN, 1)
            self.out_scale = 0.5
            self.quant = False

        @staticmethod
        def _bf16(t):
            # straight-through rounding to BF16 (round to nearest even)
            return t + (t.to(torch.bfloat16).to(t.dtype) - t).detach()

        def forward(self, f):
            z = f * self.in_scale + self.in_shift
            a = torch.nn.functional.silu(self.l1(z))
            for lin in self.hidden:
                if self.quant:
                    a = torch.nn.functional.linear(self._bf16(a), self._bf16(lin.weight), lin.bias)
                else:
                    a = lin(a)
                a = torch.nn.functional.silu(a)
            return self.out(a).squeeze(-1) * self.out_scale

    return FootprintMLP()


def model_to_blob(model, n: int, seed: int, rel_fp32: float, rel_bf16: float) -> bytes:
    """Fold the input normalisation into layer 1 and the output scale into the
    output layer, round the hidden weights to BF16 (RNE) and serialise."""
    import torch

    with torch.no_grad():
        sc = model.in_scale.double().numpy()
        sh = model.in_shift.double().numpy()
        W1 = model.l1.weight.double().numpy()
        b1 = model.l1.bias.double().numpy()
        W1f = (W1 * sc[None, :]).astype(np.float32)
        b1f = (b1 + W1 @ sh).astype(np.float32)
        parts = [W1f.tobytes(), b1f.tobytes()]
        for lin in model.hidden:
            wb = lin.weight.detach().float().to(torch.bfloat16).view(torch.int16).numpy().astype(np.int16)
            parts.append(wb.tobytes())
            parts.append(lin.bias.detach().float().numpy().astype(np.float32).tobytes())
        wo = (model.out.weight.double().numpy().reshape(-1) * model.out_scale).astype(np.float32)
        bo = np.array([model.out.bias.double().item() * model.out_scale], dtype=np.float32)
        parts += [wo.tobytes(), bo.tobytes()]
    header = struct.pack(HEADER_FMT, MAGIC, VERSION, n, IN_DIM, HIDDEN, DEPTH, ACT_SILU, FOLD_ID, seed,
                         float(rel_fp32), float(rel_bf16))
    blob = header + b"".join(parts)
    assert len(blob) == blob_bytes()
    return blob


def parse_blob(blob: bytes) -> dict:
    """Header fields and FP32/BF16 arrays of a weight blob."""
    if len(blob) != blob_bytes():
        raise ValueError("weight blob has the wrong size")
    hdr = struct.unpack_from(HEADER_FMT, blob, 0)
    if hdr[0] != MAGIC or hdr[1] != VERSION:
        raise ValueError("not a footprint-MLP blob of this version")
    off = HEADER_BYTES

    def take(dtype, count):
        nonlocal off
        a = np.frombuffer(blob, dtype=dtype, count=count, offset=off)
        off += a.nbytes
        return a

    d = {"degree": hdr[2], "in": hdr[3], "hidden": hdr[4], "depth": hdr[5], "act": hdr[6],
         "fold": hdr[7], "seed": hdr[8], "rel_fp32": hdr[9], "rel_bf16": hdr[10]}
    d["W1"] = take(np.float32, HIDDEN * IN_DIM).reshape(HIDDEN, IN_DIM)
    d["b1"] = take(np.float32, HIDDEN)
    d["Wh"], d["bh"] = [], []
    for _ in range(DEPTH - 1):
        bits = take(np.uint16, HIDDEN * HIDDEN).astype(np.uint32) << 16
        d["Wh"].append(bits.view(np.float32).reshape(HIDDEN, HIDDEN))
        d["bh"].append(take(np.float32, HIDDEN))
    d["Wo"] = take(np.float32, HIDDEN)
    d["bo"] = take(np.float32, 1)[0]
    return d


def blob_forward(blob: dict, feats: np.ndarray, bf16_activations: bool = True) -> np.ndarray:
    """Evaluate a parsed blob on [B, 5] FP32 features with the kernel's
    precision split (numpy; activations entering the BF16 layers are rounded
    to BF16 with round-to-nearest-even when ``bf16_activations``)."""
    def silu(z):
        return z / (1.0 + np.exp(-z))

    def to_bf16(a):
        b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
        rnd = ((b >> 16) & 1) + 0x7FFF
        return ((b + rnd) & 0xFFFF0000).astype(np.uint32).view(np.float32)

    f = np.asarray(feats, dtype=np.float32)
    a = silu(f @ blob["W1"].T + blob["b1"]).astype(np.float32)
    for W, b in zip(blob["Wh"], blob["bh"]):
        inp = to_bf16(a) if bf16_activations else a
        a = silu(inp.astype(np.float64) @ W.T.astype(np.float64) + b).astype(np.float32)
    return (a.astype(np.float64) @ blob["Wo"] + blob["bo"]).astype(np.float32)
