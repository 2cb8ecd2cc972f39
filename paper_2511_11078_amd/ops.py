"""User-facing operators on top of the C ABI.

* ``Context``   -- one ss_ctx (device, basis degree, footprint form).
* ``Projector`` -- forward model P_phi of eq. (7) for fixed volume size and
  geometry, and its transpose.
* ``Project``   -- torch.autograd.Function: forward = ss_project, backward =
  ss_backproject (the adjoint is the gradient of c -> P c).
* ``cgls``      -- least-squares reconstruction of Sec. 3, eq. (6): CGLS from
  x = 0, FP32 vectors, FP64 scalars computed on the device.

All arithmetic runs in the HIP library; this module only passes device
pointers and torch's current stream.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import _lib

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def default_weights(degree: int) -> str:
    return os.path.join(WEIGHTS_DIR, f"mlp_n{degree}.bin")


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype, device, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (ROCm) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{device}")
    return ctypes.c_void_p(t.data_ptr())


def _check_shape(t, shape, name: str):
    """The library receives raw pointers only: every buffer must have exactly
    the shape the call reads or writes (a smaller one would be overrun)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if tuple(t.shape) != tuple(int(s) for s in shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(int(s) for s in shape)}")


class Context:
    """An ss_ctx: degree n in 0..3, form 'quad' (exact FP32, knot-cell walk),
    'mlp' (BF16 network) or 'pair' (exact FP32 per (line, basis) pair on the
    network form's walk)."""

    def __init__(self, degree: int = 3, form: str = "quad", device: int = 0, weights=None):
        lib = _lib.load()
        self.degree, self.form, self.device = int(degree), form, int(device)
        blob = None
        if form == "mlp":
            path = weights or default_weights(degree)
            with open(path, "rb") as fh:
                blob = fh.read()
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob)) if blob else None
        _lib.check(lib.ss_create(ctypes.byref(h), self.device, self.degree, _lib.FORMS[form],
                                 buf, len(blob) if blob else 0))
        self._h = h
        self._lib = lib

    def set_scratch_limit(self, nbytes: int):
        """Largest knot-cell table the quadrature adjoint may allocate; larger
        tables are processed in z-chunks (ss_set_scratch_limit)."""
        _lib.check(self._lib.ss_set_scratch_limit(self._h, int(nbytes)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ss_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- transforms ---------------------------------------------------------
    def project(self, c: torch.Tensor, geom, out: torch.Tensor | None = None) -> torch.Tensor:
        """Sinogram [V, R, C] of coefficients c [N3, N2, N1] (eq. (7))."""
        if c.dim() != 3:
            raise ValueError("coefficients must be [N3, N2, N1]")
        dims = (c.shape[2], c.shape[1], c.shape[0])
        shape = (geom.n_views, geom.det_rows, geom.det_cols)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=c.device)
        _check_shape(out, shape, "out")
        g = _lib.GeometryArg(geom)
        _lib.check(self._lib.ss_project(self._h, _dev_ptr(c, torch.float32, self.device, "c"), _lib.dims_arg(dims),
                                        g.ref(), _dev_ptr(out, torch.float32, self.device, "out"),
                                        _stream(self.device)))
        return out

    def backproject(self, y: torch.Tensor, geom, dims, out: torch.Tensor | None = None) -> torch.Tensor:
        """Transpose of ``project``: coefficients [N3, N2, N1] from y [V, R, C]."""
        shape = (dims[2], dims[1], dims[0])
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=y.device)
        _check_shape(y, (geom.n_views, geom.det_rows, geom.det_cols), "y")
        _check_shape(out, shape, "out")
        g = _lib.GeometryArg(geom)
        _lib.check(self._lib.ss_backproject(self._h, _dev_ptr(y, torch.float32, self.device, "y"), g.ref(),
                                            _lib.dims_arg(dims), _dev_ptr(out, torch.float32, self.device, "out"),
                                            _stream(self.device)))
        return out

    def footprint(self, dirs: torch.Tensor, offsets: torch.Tensor) -> torch.Tensor:
        """P phi(w, x) for pairs (dirs [K, 3] unit, offsets [K, 3])."""
        if dirs.dim() != 2 or dirs.shape[1] != 3:
            raise ValueError("dirs must be [K, 3]")
        k = dirs.shape[0]
        _check_shape(offsets, (k, 3), "offsets")
        out = torch.empty(k, dtype=torch.float32, device=dirs.device)
        _lib.check(self._lib.ss_footprint(self._h, _dev_ptr(dirs, torch.float32, self.device, "dirs"),
                                          _dev_ptr(offsets, torch.float32, self.device, "offsets"), k,
                                          _dev_ptr(out, torch.float32, self.device, "out"), _stream(self.device)))
        return out

    # -- FP64 scalars / FP32 vector updates ---------------------------------
    def dot_f64(self, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((), dtype=torch.float64, device=a.device)
        if a.numel() != b.numel():
            raise ValueError("dot of vectors of different lengths")
        if out.numel() != 1:
            raise ValueError("out must hold one FP64 value")
        _lib.check(self._lib.ss_dot_f64(self._h, _dev_ptr(a, torch.float32, self.device, "a"),
                                        _dev_ptr(b, torch.float32, self.device, "b"), a.numel(),
                                        _dev_ptr(out, torch.float64, self.device, "out"), _stream(self.device)))
        return out

    def ratio(self, num: torch.Tensor, den: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        for t, name in ((num, "num"), (den, "den"), (out, "out")):
            if t.numel() != 1:
                raise ValueError(f"{name} must hold one FP64 value")
        _lib.check(self._lib.ss_cgls_scalars(self._h, _dev_ptr(num, torch.float64, self.device, "num"),
                                             _dev_ptr(den, torch.float64, self.device, "den"),
                                             _dev_ptr(out, torch.float64, self.device, "out"), _stream(self.device)))
        return out

    def axpy(self, alpha: torch.Tensor, sign: int, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        if x.numel() != y.numel():
            raise ValueError("axpy of vectors of different lengths")
        if alpha.numel() != 1:
            raise ValueError("alpha must hold one FP64 value")
        _lib.check(self._lib.ss_axpy(self._h, _dev_ptr(alpha, torch.float64, self.device, "alpha"), int(sign),
                                     _dev_ptr(x, torch.float32, self.device, "x"),
                                     _dev_ptr(y, torch.float32, self.device, "y"), x.numel(), _stream(self.device)))
        return y

    def xpay(self, beta: torch.Tensor, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        if x.numel() != y.numel():
            raise ValueError("xpay of vectors of different lengths")
        if beta.numel() != 1:
            raise ValueError("beta must hold one FP64 value")
        _lib.check(self._lib.ss_xpay(self._h, _dev_ptr(beta, torch.float64, self.device, "beta"),
                                     _dev_ptr(x, torch.float32, self.device, "x"),
                                     _dev_ptr(y, torch.float32, self.device, "y"), x.numel(), _stream(self.device)))
        return y


def project_noalloc(c: torch.Tensor, geom, degree: int = 3, out: torch.Tensor | None = None) -> torch.Tensor:
    """ss_project_noalloc: the quadrature-form forward of ``Context.project``
    without a context and without any allocation by the library (its
    scratch is a static device array per GPU; calls on one GPU must not
    overlap in time).  ``out`` [V, R, C] is allocated here when not given."""
    lib = _lib.load()
    if c.dim() != 3:
        raise ValueError("coefficients must be [N3, N2, N1]")
    dims = (c.shape[2], c.shape[1], c.shape[0])
    shape = (geom.n_views, geom.det_rows, geom.det_cols)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=c.device)
    _check_shape(out, shape, "out")
    device = c.device.index if c.device.index is not None else 0
    g = _lib.GeometryArg(geom)
    _lib.check(lib.ss_project_noalloc(device, int(degree), _dev_ptr(c, torch.float32, device, "c"),
                                      _lib.dims_arg(dims), g.ref(), _dev_ptr(out, torch.float32, device, "out"),
                                      _stream(device)))
    return out


class Projector:
    """P_phi of eq. (7) for coefficient volumes of size ``dims`` = (N1, N2, N3)
    and a fixed acquisition geometry."""

    def __init__(self, dims, geom, degree: int = 3, form: str = "quad", device: int = 0, weights=None,
                 context: Context | None = None):
        self.dims = tuple(int(d) for d in dims)
        self.geom = geom
        _lib.validate_problem(self.dims, geom)
        self.ctx = context or Context(degree, form, device, weights)
        self.device = self.ctx.device

    @property
    def sino_shape(self):
        return (self.geom.n_views, self.geom.det_rows, self.geom.det_cols)

    @property
    def vol_shape(self):
        return (self.dims[2], self.dims[1], self.dims[0])

    def forward(self, c: torch.Tensor, out=None) -> torch.Tensor:
        return self.ctx.project(c, self.geom, out)

    def adjoint(self, y: torch.Tensor, out=None) -> torch.Tensor:
        return self.ctx.backproject(y, self.geom, self.dims, out)

    __call__ = forward


class Project(torch.autograd.Function):
    """y = P c with dL/dc = P^T dL/dy (the matched adjoint)."""

    @staticmethod
    def forward(ctx, c: torch.Tensor, projector: Projector):
        ctx.projector = projector
        return projector.forward(c.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.projector.adjoint(g.contiguous()), None


class Backproject(torch.autograd.Function):
    """c = P^T y with dL/dy = P dL/dc."""

    @staticmethod
    def forward(ctx, y: torch.Tensor, projector: Projector):
        ctx.projector = projector
        return projector.adjoint(y.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.projector.forward(g.contiguous()), None


def project(c: torch.Tensor, projector: Projector) -> torch.Tensor:
    return Project.apply(c, projector)


def cgls(projector: Projector, y: torch.Tensor, iters: int = 50, x0=None, callback=None,
         residuals: bool = False):
    """CGLS for min ||P x - y||^2 (eq. (6)), x_0 = 0 unless given.

    Vectors stay FP32 on the device; the inner products are accumulated in
    FP64 and the step length alpha and ratio beta are formed in FP64 on the
    device, so the loop never synchronises with the host.  Returns
    (x, history) with history the device FP64 tensor of ||A^T r_k||^2; with
    ``residuals`` also the device FP64 tensor of ||r_k||^2 (one more inner
    product per iteration)."""
    ctx = projector.ctx
    dev = y.device
    f64 = dict(dtype=torch.float64, device=dev)
    x = torch.zeros(projector.vol_shape, dtype=torch.float32, device=dev) if x0 is None else x0.clone()
    r = y.clone()
    if x0 is not None:
        r -= projector.forward(x)
    s = projector.adjoint(r)
    p = s.clone()
    q = torch.empty_like(y)
    gamma = torch.empty((), **f64)
    gamma_new = torch.empty((), **f64)
    qq = torch.empty((), **f64)
    alpha = torch.empty((), **f64)
    beta = torch.empty((), **f64)
    hist = torch.empty(iters + 1, **f64)
    rhist = torch.empty(iters + 1, **f64) if residuals else None
    ctx.dot_f64(s, s, gamma)
    hist[0] = gamma
    if residuals:
        ctx.dot_f64(r, r, rhist[0])
    for k in range(iters):
        projector.forward(p, q)
        ctx.dot_f64(q, q, qq)
        ctx.ratio(gamma, qq, alpha)
        ctx.axpy(alpha, +1, p, x)
        ctx.axpy(alpha, -1, q, r)
        projector.adjoint(r, s)
        ctx.dot_f64(s, s, gamma_new)
        ctx.ratio(gamma_new, gamma, beta)
        ctx.xpay(beta, s, p)
        gamma, gamma_new = gamma_new, gamma
        hist[k + 1] = gamma
        if residuals:
            ctx.dot_f64(r, r, rhist[k + 1])
        if callback is not None:
            callback(k, x, r)
    if residuals:
        return x, hist, rhist
    return x, hist
