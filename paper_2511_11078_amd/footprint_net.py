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
three 64x64 layers take BF16 operands with FP32 accumulation -- the weights
are BF16 numbers, and each FP32 activation entering such a layer is carried
as the sum of two BF16 numbers (its rounding and the rounding of what that
leaves), so the layer is two BF16 products into one FP32 accumulator and
the activations lose about 16 bits instead of 8; SiLU in FP32; the output
layer in FP32.  The kernel multiplies the network output by the
indicator that the line meets the basis support (an exact slab test), so the
network is only ever used where the true footprint can be non-zero.

Training labels come from ``exact_footprint`` below: an FP64 vectorised
piecewise Gauss-Legendre integral (exact for B-splines, see the module
docstring of ``train_footprint``), written for training only; it runs on
the host or, during training, on the GPU.
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
# folding, features and FP64 training labels.  Each is written once with
# torch operations, so that it runs on the host (numpy in, numpy out) and on
# a GPU during training (torch tensors in, torch tensors out).
# --------------------------------------------------------------------------
def _as_torch(a):
    import torch

    if isinstance(a, torch.Tensor):
        return a.to(torch.float64), False
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)), True


def fold_features(w, x):
    """(w, x) [B, 3] -> features [B, 5] of fold convention 1: sort |w|
    ascending (stable: lower axis first on ties), apply the same signed
    permutation to x, frame u = normalise(e1 - w1 w), v = u x w."""
    import torch

    w, to_np = _as_torch(w)
    x, _ = _as_torch(x)
    aw = w.abs()
    perm = torch.argsort(aw, dim=1, stable=True)
    wsel = torch.gather(w, 1, perm)
    sgn = torch.where(wsel < 0, -1.0, 1.0).to(w.dtype)
    wf = torch.gather(aw, 1, perm)
    xf = torch.gather(x, 1, perm) * sgn
    u = -wf[:, 0:1] * wf
    u[:, 0] += 1.0
    u = u / torch.linalg.norm(u, dim=1, keepdim=True)
    v = torch.linalg.cross(u, wf, dim=1)
    out = torch.cat([wf, (u * xf).sum(1, keepdim=True), (v * xf).sum(1, keepdim=True)], dim=1)
    return out.numpy() if to_np else out


def _chord(n: int, w, x):
    """Parameter interval (t0, t1) of the line x + t w inside the open
    support cube (-h, h)^3, and whether it is non-empty."""
    import torch

    h = 0.5 * (n + 1)
    inside = x.abs() < h
    ta = (-h - x) / w
    tb = (h - x) / w
    inf = torch.full_like(x, float("inf"))
    lo = torch.where(w == 0, torch.where(inside, -inf, inf), torch.minimum(ta, tb))
    hi = torch.where(w == 0, torch.where(inside, inf, -inf), torch.maximum(ta, tb))
    t0 = lo.max(1).values
    t1 = hi.min(1).values
    return t0, t1, t0 < t1


def chord_nonempty(n: int, w, x):
    w, to_np = _as_torch(w)
    x, _ = _as_torch(x)
    ok = _chord(n, w, x)[2]
    return ok.numpy() if to_np else ok


def _bspline(n: int, x):
    import torch

    a = x.abs()
    if n == 0:
        return (a < 0.5).to(x.dtype)
    if n == 1:
        return torch.clamp(1.0 - a, min=0.0)
    if n == 2:
        return torch.where(a < 0.5, 0.75 - a * a, torch.where(a < 1.5, 0.5 * (1.5 - a) ** 2, torch.zeros_like(a)))
    if n == 3:
        return torch.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                           torch.where(a < 2.0, (2.0 - a) ** 3 / 6.0, torch.zeros_like(a)))
    raise ValueError(n)


def exact_footprint(n: int, w, x, chunk: int = 1 << 16):
    """int phi(x + t w) dt for unit w, in FP64: clip to the support cube, cut
    at the interior knot planes, Gauss-Legendre of order ceil((3n+1)/2) on
    each piece (exact, the integrand being a polynomial of degree 3n there).
    numpy arrays in -> numpy out (host); torch tensors in -> torch out on
    their device."""
    import torch

    w, to_np = _as_torch(w)
    x, _ = _as_torch(x)
    dev = w.device
    out = torch.empty(w.shape[0], dtype=torch.float64, device=dev)
    h = 0.5 * (n + 1)
    m = max(1, (3 * n + 2) // 2)
    gx_np, gw_np = np.polynomial.legendre.leggauss(m)
    gx = torch.from_numpy(gx_np).to(dev)
    gw = torch.from_numpy(gw_np).to(dev)
    knots = (-h + torch.arange(1, n + 1, dtype=torch.float64)).to(dev)
    for s in range(0, w.shape[0], chunk):
        W = w[s:s + chunk]
        X = x[s:s + chunk]
        t0, t1, valid = _chord(n, W, X)
        t0 = torch.where(valid, t0, torch.zeros_like(t0))
        t1 = torch.where(valid, t1, torch.zeros_like(t1))
        T = (knots[None, None, :] - X[:, :, None]) / W[:, :, None]
        T = torch.where(torch.isfinite(T), T, t0[:, None, None])
        T = torch.minimum(torch.maximum(T, t0[:, None, None]), t1[:, None, None]).reshape(W.shape[0], -1)
        T = torch.sort(torch.cat([t0[:, None], T, t1[:, None]], dim=1), dim=1).values
        mid = 0.5 * (T[:, 1:] + T[:, :-1])
        half = 0.5 * (T[:, 1:] - T[:, :-1])
        t = mid[..., None] + half[..., None] * gx                       # [B, S, m]
        pos = X[:, None, None, :] + t[..., None] * W[:, None, None, :]  # [B, S, m, 3]
        val = _bspline(n, pos).prod(-1)
        seg = (val * gw).sum(-1) * half
        out[s:s + chunk] = torch.where(valid, seg.sum(-1), torch.zeros_like(t0))
    return out.numpy() if to_np else out


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


def make_torch_model(degrees):
    """G independent networks, one per entry of ``degrees``, evaluated side by
    side with batched products: inputs [G, B, 5] -> outputs [G, B].  A single
    degree may be given as an int (G = 1)."""
    import torch
    from torch import nn

    degs = [int(degrees)] if np.isscalar(degrees) else [int(d) for d in degrees]
    G = len(degs)

    def uniform(shape, fan_in):
        bound = 1.0 / np.sqrt(fan_in)
        return nn.Parameter(torch.empty(shape).uniform_(-bound, bound))

    class FootprintMLP(nn.Module):
        """``quant`` selects the arithmetic of the hidden layers: "fp32";
        "split" -- the kernel's: weights rounded to BF16, each activation
        entering a BF16 layer carried as the sum of two BF16 numbers (its
        rounding and the rounding of the remainder); "bf16" -- weights and
        activations each rounded once to BF16.  Rounding is round to nearest
        even with a straight-through gradient.  Weights are stored [G, in,
        out] so that every product is a plain batched product."""

        def __init__(self):
            super().__init__()
            self.degrees = degs
            sc = np.stack([feature_scale(d)[0] for d in degs])
            sh = np.stack([feature_scale(d)[1] for d in degs])
            self.register_buffer("in_scale", torch.tensor(sc, dtype=torch.float32)[:, None, :])
            self.register_buffer("in_shift", torch.tensor(sh, dtype=torch.float32)[:, None, :])
            self.w1 = uniform((G, IN_DIM, HIDDEN), IN_DIM)
            self.b1 = uniform((G, 1, HIDDEN), IN_DIM)
            self.wh = nn.ParameterList([uniform((G, HIDDEN, HIDDEN), HIDDEN) for _ in range(DEPTH - 1)])
            self.bh = nn.ParameterList([uniform((G, 1, HIDDEN), HIDDEN) for _ in range(DEPTH - 1)])
            self.wo = uniform((G, HIDDEN, 1), HIDDEN)
            self.bo = uniform((G, 1, 1), HIDDEN)
            self.out_scale = 0.5
            self.quant = "fp32"

        @staticmethod
        def _bf16(t):
            return t + (t.to(torch.bfloat16).to(t.dtype) - t).detach()

        def _act(self, a):
            if self.quant == "bf16":
                return self._bf16(a)
            if self.quant == "split":
                hi = a.to(torch.bfloat16).to(a.dtype)
                lo = (a - hi).to(torch.bfloat16).to(a.dtype)
                return a + (hi + lo - a).detach()
            return a

        def forward(self, f):
            if f.dim() == 2:
                f = f[None]
            z = f * self.in_scale + self.in_shift
            a = torch.nn.functional.silu(torch.baddbmm(self.b1, z, self.w1))
            for W, b in zip(self.wh, self.bh):
                if self.quant != "fp32":
                    a = torch.baddbmm(b, self._act(a), self._bf16(W))
                else:
                    a = torch.baddbmm(b, a, W)
                a = torch.nn.functional.silu(a)
            return torch.baddbmm(self.bo, a, self.wo).squeeze(-1) * self.out_scale

    return FootprintMLP()


def model_to_blob(model, n: int, seed: int, rel_fp32: float, rel_bf16: float, g: int = None) -> bytes:
    """Network g (default: the one of degree n) of a model: fold the input
    normalisation into layer 1 and the output scale into the output layer,
    round the hidden weights to BF16 (RNE) and serialise ([out][in] rows)."""
    import torch

    if g is None:
        g = model.degrees.index(n)
    with torch.no_grad():
        sc = model.in_scale[g, 0].detach().cpu().double().numpy()
        sh = model.in_shift[g, 0].detach().cpu().double().numpy()
        W1 = model.w1[g].detach().cpu().double().numpy().T          # [out][in]
        b1 = model.b1[g, 0].detach().cpu().double().numpy()
        W1f = (W1 * sc[None, :]).astype(np.float32)
        b1f = (b1 + W1 @ sh).astype(np.float32)
        parts = [W1f.tobytes(), b1f.tobytes()]
        for W, b in zip(model.wh, model.bh):
            wt = W[g].detach().cpu().float().t().contiguous()
            wb = wt.to(torch.bfloat16).view(torch.int16).numpy().astype(np.int16)
            parts.append(wb.tobytes())
            parts.append(b[g, 0].detach().cpu().float().numpy().astype(np.float32).tobytes())
        wo = (model.wo[g, :, 0].detach().cpu().double().numpy() * model.out_scale).astype(np.float32)
        bo = np.array([model.bo[g, 0, 0].detach().cpu().double().item() * model.out_scale], dtype=np.float32)
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


def to_bf16(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to BF16 (round to nearest even), returned as FP32."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    rnd = ((b >> 16) & 1) + 0x7FFF
    return ((b + rnd) & 0xFFFF0000).astype(np.uint32).view(np.float32)


def blob_forward(blob: dict, feats: np.ndarray, activations: str = "split") -> np.ndarray:
    """Evaluate a parsed blob on [B, 5] FP32 features (numpy).  The hidden
    weights are the blob's BF16 values; ``activations`` is how the inputs of
    the three BF16 layers are carried: "split" (the kernel's: the sum of two
    BF16 numbers, the rounding of the FP32 value and the rounding of the
    remainder), "bf16" (one rounding) or "fp32"."""
    def silu(z):
        return z / (1.0 + np.exp(-z))

    f = np.asarray(feats, dtype=np.float32)
    a = silu(f @ blob["W1"].T + blob["b1"]).astype(np.float32)
    for W, b in zip(blob["Wh"], blob["bh"]):
        if activations == "split":
            hi = to_bf16(a)
            lo = to_bf16((a - hi).astype(np.float32))
            inp = hi.astype(np.float64) + lo.astype(np.float64)
        elif activations == "bf16":
            inp = to_bf16(a).astype(np.float64)
        else:
            inp = a.astype(np.float64)
        a = silu(inp @ W.T.astype(np.float64) + b).astype(np.float32)
    return (a.astype(np.float64) @ blob["Wo"] + blob["bo"]).astype(np.float32)
