"""Seeded synthetic inputs: acquisition geometries and coefficient volumes.

This module only *generates inputs*; it holds none of the transform's
arithmetic (no ray set-up, traversal or footprint), so both the HIP path and
the FP64 checker may consume what it produces.

Geometry convention (one 12-float vector per view, world unit = coefficient
spacing, coefficient k at x_k = k - (N - 1)/2 per axis):

* parallel: ``(w, d0, du, dv)`` -- ray direction, detector centre, and the
  detector's column / row steps.  Pixel (row j, col i) is the line through
  d0 + (i - (C-1)/2) du + (j - (R-1)/2) dv with direction w.
* cone: ``(src, d0, du, dv)`` -- source position, detector centre and steps.
  Pixel (j, i) is the line through src and that pixel centre.

In both cases the whole line is integrated (the x-ray transform of eq. (2)
of the paper is an integral over all t).

Stand-ins: the paper evaluates on BrainWeb volumes with ASTRA-simulated
cone-beam data (Sec. 3), neither of which is available here.  The ellipsoid
phantoms, noise and smoothed random fields below are synthetic substitutes
of the same kind (a normalised volume of a few smooth structures).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Geometry:
    kind: str              # 'parallel' | 'cone'
    n_views: int
    det_rows: int
    det_cols: int
    vecs: np.ndarray       # float32 [n_views, 12]

    @property
    def n_rays(self) -> int:
        return self.n_views * self.det_rows * self.det_cols

    def subset_views(self, v0: int, v1: int) -> "Geometry":
        return Geometry(self.kind, v1 - v0, self.det_rows, self.det_cols,
                        np.ascontiguousarray(self.vecs[v0:v1]))


# --------------------------------------------------------------------------
# directions and frames
# --------------------------------------------------------------------------
def fibonacci_directions(n: int) -> np.ndarray:
    """Spherical Fibonacci points: z_i = 1 - (2i+1)/n, azimuth i*pi*(3 - sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = i * np.pi * (3.0 - np.sqrt(5.0))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def uniform_directions(n: int, seed: int) -> np.ndarray:
    """Directions uniform on the unit sphere (normalised Gaussian vectors)."""
    g = np.random.default_rng(seed).standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def great_circle_plus_tilts(n_circle: int = 180, n_tilt: int = 60, seed: int = 2) -> np.ndarray:
    """n_circle directions (cos t, sin t, 0), t = i*pi/n_circle, then n_tilt
    uniform random directions (lines are unoriented, so half a circle covers
    every in-plane direction)."""
    t = np.arange(n_circle, dtype=np.float64) * np.pi / n_circle
    circ = np.stack([np.cos(t), np.sin(t), np.zeros_like(t)], axis=1)
    return np.concatenate([circ, uniform_directions(n_tilt, seed)], axis=0)


def detector_frame(w: np.ndarray):
    """An orthonormal (u, v) with u, v perpendicular to w and v = u x w.

    u = normalise(e_a - w_a w) for the axis a of smallest |w_a| (lowest index
    on ties); in-plane great-circle directions get u = (-sin t, cos t, 0) and
    v = e3 by the same rule up to sign, which we fix explicitly."""
    w = np.asarray(w, dtype=np.float64)
    if abs(w[2]) < 1e-12:
        u = np.array([-w[1], w[0], 0.0])
        u /= np.linalg.norm(u)
        v = np.array([0.0, 0.0, 1.0])
        return u, v
    a = int(np.argmin(np.abs(w)))
    e = np.zeros(3)
    e[a] = 1.0
    u = e - w[a] * w
    u /= np.linalg.norm(u)
    v = np.cross(u, w)
    return u, v


def parallel_geometry(dirs: np.ndarray, det_rows: int, det_cols: int, pitch: float = 1.0,
                      centre=(0.0, 0.0, 0.0)) -> Geometry:
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    vecs = np.zeros((dirs.shape[0], 12), dtype=np.float64)
    for k, w in enumerate(dirs):
        w = w / np.linalg.norm(w)
        u, v = detector_frame(w)
        vecs[k, 0:3] = w
        vecs[k, 3:6] = centre
        vecs[k, 6:9] = pitch * u
        vecs[k, 9:12] = pitch * v
    return Geometry("parallel", dirs.shape[0], det_rows, det_cols, vecs.astype(np.float32))


def cone_circular_geometry(n_views: int, det_rows: int, det_cols: int, src_radius: float,
                           src_det: float, pitch: float = 1.0, angle0: float = 0.0) -> Geometry:
    """Source on the circle of radius ``src_radius`` in the plane x3 = 0 at
    angles 2*pi*i/n_views; flat detector perpendicular to the central ray at
    distance ``src_det`` from the source, columns along the circle's tangent,
    rows along e3."""
    th = angle0 + 2.0 * np.pi * np.arange(n_views, dtype=np.float64) / n_views
    c, s = np.cos(th), np.sin(th)
    vecs = np.zeros((n_views, 12), dtype=np.float64)
    vecs[:, 0] = src_radius * c
    vecs[:, 1] = src_radius * s
    vecs[:, 3] = (src_radius - src_det) * c
    vecs[:, 4] = (src_radius - src_det) * s
    vecs[:, 6] = -pitch * s
    vecs[:, 7] = pitch * c
    vecs[:, 11] = pitch
    return Geometry("cone", n_views, det_rows, det_cols, vecs.astype(np.float32))


# --------------------------------------------------------------------------
# coefficient volumes, float32 [N3, N2, N1] (x fastest)
# --------------------------------------------------------------------------
def _random_rotation(rng) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_params(n_ell: int = 6, seed: int = 0, centre_radius: float = 0.5, max_axis: float = 0.5):
    """Random ellipsoids in normalised coordinates [-1, 1]^3: centre uniform in
    the ball of radius 0.5, semi-axes U(0.1, 0.5), uniform random rotation,
    density U(0, 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_ell):
        while True:
            cen = rng.uniform(-centre_radius, centre_radius, 3)
            if np.linalg.norm(cen) <= centre_radius:
                break
        axes = rng.uniform(0.1, max_axis, 3)
        rot = _random_rotation(rng)
        rho = rng.uniform(0.0, 1.0)
        out.append((cen, axes, rot, rho))
    return out


def ellipsoid_phantom(dims, n_ell: int = 6, seed: int = 0, params=None) -> np.ndarray:
    """c_k = sum_e rho_e [xi_k in E_e], xi = x / ((N - 1)/2) per axis; the same
    normalised parameters give 'the same phantom' at every size."""
    N1, N2, N3 = (int(d) for d in dims)
    ax = [(np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) / max(0.5 * (n - 1), 0.5)
          for n in (N1, N2, N3)]
    c = np.zeros((N3, N2, N1), dtype=np.float32)
    for cen, axes, rot, rho in (params if params is not None else ellipsoid_params(n_ell, seed)):
        # process one z-slice at a time to bound memory at 512^3
        X1, X2 = np.meshgrid(ax[0], ax[1], indexing="xy")  # [N2, N1]
        for k3 in range(N3):
            p = np.stack([X1 - cen[0], X2 - cen[1], np.full_like(X1, ax[2][k3] - cen[2])], axis=-1)
            loc = p @ rot  # coordinates in the ellipsoid frame
            inside = ((loc / axes) ** 2).sum(-1) <= 1.0
            c[k3][inside] += np.float32(rho)
    return c


def ellipsoid_line_integrals(dims, geom, params) -> np.ndarray:
    """Measured data for a continuous ellipsoid phantom: the exact line
    integral sum_e rho_e * (chord length of the line through ellipsoid e),
    for every detector pixel of ``geom`` (float64 [V, R, C]).

    This simulates acquisitions independently of any basis (the role the
    ASTRA toolbox plays in the paper's experiment).  Ellipsoids are given in
    the normalised coordinates of ``ellipsoid_params`` (xi = x / ((N-1)/2))."""
    N = np.asarray(dims, dtype=np.float64)
    D = 1.0 / np.maximum(0.5 * (N - 1), 0.5)
    V, R, C = geom.n_views, geom.det_rows, geom.det_cols
    vec = np.asarray(geom.vecs, dtype=np.float64)
    ci = np.arange(C) - 0.5 * (C - 1)
    cj = np.arange(R) - 0.5 * (R - 1)
    out = np.zeros((V, R, C))
    for v in range(V):
        e = vec[v]
        pix = e[3:6][None, None, :] + ci[None, :, None] * e[6:9] + cj[:, None, None] * e[9:12]
        if geom.kind == "parallel":
            d = np.broadcast_to(e[0:3], pix.shape)
            p = pix
        else:
            d = pix - e[0:3]
            p = np.broadcast_to(e[0:3], pix.shape)
        d = d / np.linalg.norm(d, axis=-1, keepdims=True)
        pn, dn = p * D, d * D
        for cen, axes, rot, rho in params:
            pp = ((pn - cen) @ rot) / axes
            dd = (dn @ rot) / axes
            a = (dd * dd).sum(-1)
            b = (pp * dd).sum(-1)
            c0 = (pp * pp).sum(-1) - 1.0
            disc = b * b - a * c0
            out[v] += rho * np.where(disc > 0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / a, 0.0)
    return out


def add_noise(c: np.ndarray, variance: float = 0.01, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (c + rng.standard_normal(c.shape).astype(np.float32) * np.float32(np.sqrt(variance))).astype(np.float32)


def smooth_field(dims, sigma: float = 4.0, seed: int = 6) -> np.ndarray:
    """i.i.d. N(0, 1) low-passed by a periodic Gaussian of std ``sigma`` voxels
    (FFT), then standardised to zero mean and unit std."""
    N1, N2, N3 = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((N3, N2, N1), dtype=np.float32)
    G = np.fft.rfftn(g)
    del g
    f3 = np.fft.fftfreq(N3)[:, None, None]
    f2 = np.fft.fftfreq(N2)[None, :, None]
    f1 = np.fft.rfftfreq(N1)[None, None, :]
    k2 = (2 * np.pi) ** 2 * (f1 * f1 + f2 * f2 + f3 * f3)
    G *= np.exp(-0.5 * sigma * sigma * k2)
    out = np.fft.irfftn(G, s=(N3, N2, N1), axes=(0, 1, 2)).astype(np.float32)
    out -= out.mean(dtype=np.float64)
    out /= out.std(dtype=np.float64)
    return out


def gaussian_volume(dims, seed: int) -> np.ndarray:
    N1, N2, N3 = (int(d) for d in dims)
    return np.random.default_rng(seed).standard_normal((N3, N2, N1), dtype=np.float32)


def sample_indices(total: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct indices in [0, total) (seeded)."""
    count = min(count, total)
    rng = np.random.default_rng(seed)
    idx = rng.choice(total, size=count, replace=False)
    return np.sort(idx.astype(np.int64))
