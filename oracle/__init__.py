"""FP64 oracle for the spline x-ray transform -- TEST INFRASTRUCTURE ONLY.

This package is the checker, not the product.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the HIP
library never calls it and shares no code with it.

It wraps ``oracle.c`` (plain C, FP64, OpenMP over rays) through ctypes and
adds the FP64 CGLS recurrence (``cgls.py``).  Geometry objects are duck-typed:
anything with ``kind`` ('parallel' | 'cone'), ``n_views``, ``det_rows``,
``det_cols`` and ``vecs`` (float32 [V, 12]) works.

Paper: SplineSplat (arXiv 2511.11078).  Each function cites the passage it
implements; ``oracle.c`` holds the details.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_SRC / ORACLE_LIB name another copy of the C source and its library:
# the mutation test uses them to run the pins against deliberately broken
# copies (tests/test_oracle_mutations.py)
_SRC = os.environ.get("ORACLE_SRC") or os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_KIND = {"parallel": 0, "cone": 1}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    L = ctypes.c_int64
    lib.or_bspline.restype = ctypes.c_double
    lib.or_bspline.argtypes = [I, ctypes.c_double]
    lib.or_bspline_tp.restype = ctypes.c_double
    lib.or_bspline_tp.argtypes = [I, ctypes.c_double]
    lib.or_bspline_many.argtypes = [I, L, P, P, I]
    lib.or_gauss_legendre.argtypes = [I, P, P]
    lib.or_footprint_many.argtypes = [I, L, P, P, P]
    geo = [I, I, I, I, P]
    lib.or_make_rays.argtypes = [I, I, I, I, P, P, L, P, P]
    lib.or_project.argtypes = [I, P, P] + geo + [P, L, P]
    lib.or_project_lines.argtypes = [I, P, P, L, P, P, P]
    lib.or_project_basis_sum.argtypes = [I, P, P] + geo + [P, L, P]
    lib.or_counts.argtypes = [I, P] + geo + [P, L, P, P]
    lib.or_direct_counts.argtypes = [I, P] + geo + [P, L, P]
    lib.or_backproject_subset.argtypes = [I, P, P] + geo + [P, L, P]
    lib.or_dense_matrix.argtypes = [I, P] + geo + [P, L, P]
    lib.or_num_threads.restype = I
    lib.or_set_num_threads.argtypes = [I]
    lib.or_set_num_threads.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _geom_args(geom):
    vecs = np.ascontiguousarray(np.asarray(geom.vecs, dtype=np.float32).reshape(-1, 12))
    if vecs.shape[0] != geom.n_views:
        raise ValueError("geometry vecs must be [n_views, 12]")
    return vecs, (_KIND[geom.kind], int(geom.n_views), int(geom.det_rows), int(geom.det_cols))


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int64).reshape(3))
    return d


def _idx(idx, total):
    if idx is None:
        return None, total
    a = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1))
    if a.size and (a.min() < 0 or a.max() >= total):
        raise ValueError("index out of range")
    return a, a.size


def num_threads() -> int:
    return _load().or_num_threads()


def set_num_threads(k: int) -> None:
    """Threads of the following oracle calls (k < 1: back to the default)."""
    _load().or_set_num_threads(int(k))


def bspline(n: int, x, truncated_power: bool = False) -> np.ndarray:
    """O1: centred B-spline beta^n (piecewise form, or the truncated-power form)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.empty_like(x)
    _load().or_bspline_many(n, x.size, _ptr(x), _ptr(out), 1 if truncated_power else 0)
    return out


def gauss_legendre(m: int):
    """O2: m-point Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    x = np.empty(m)
    w = np.empty(m)
    if _load().or_gauss_legendre(m, _ptr(x), _ptr(w)):
        raise ValueError("bad order")
    return x, w


def footprint(n: int, w, x) -> np.ndarray:
    """O4: P phi(w, x) = int phi(x + t w) dt (the contribution of eq. (4)).

    ``w`` and ``x`` are [..., 3] arrays (broadcast together); ``w`` should be
    a unit vector for the x-ray transform of eq. (2)."""
    w = np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    w, x = np.broadcast_arrays(w, x)
    shape = w.shape[:-1]
    w = np.ascontiguousarray(w.reshape(-1, 3))
    x = np.ascontiguousarray(x.reshape(-1, 3))
    out = np.empty(w.shape[0])
    if _load().or_footprint_many(n, w.shape[0], _ptr(w), _ptr(x), _ptr(out)):
        raise ValueError("bad degree")
    return out.reshape(shape)


def make_rays(geom, rays=None):
    """Anchor points and unit directions of the rays (eq. (1)), FP64."""
    vecs, g = _geom_args(geom)
    total = g[1] * g[2] * g[3]
    idx, cnt = _idx(rays, total)
    a = np.empty((cnt, 3))
    w = np.empty((cnt, 3))
    if _load().or_make_rays(*g, _ptr(vecs), None if idx is None else _ptr(idx), cnt, _ptr(a), _ptr(w)):
        raise ValueError("degenerate ray")
    return a, w


def project(c, geom, n: int = 3, rays=None) -> np.ndarray:
    """O3: x-ray transform (eq. (2)) of f = sum_k c_k phi(. - x_k) (eq. (3)).

    ``c`` is float32 [N3, N2, N1] (x fastest).  Returns FP64 values for the
    rays ``rays`` (flat indices into [V, R, C]) or for all rays."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float32))
    dims = _dims(c.shape[::-1])
    vecs, g = _geom_args(geom)
    total = g[1] * g[2] * g[3]
    idx, cnt = _idx(rays, total)
    out = np.empty(cnt)
    rc = _load().or_project(n, _ptr(c), _ptr(dims), *g, _ptr(vecs),
                            None if idx is None else _ptr(idx), cnt, _ptr(out))
    if rc:
        raise ValueError("oracle project failed")
    return out if rays is not None else out.reshape(g[1], g[2], g[3])


def project_lines(c, a, w, n: int = 3) -> np.ndarray:
    """O3 on explicit lines: y_k = int f(a_k + t w_k) dt (eq. (2)) for FP64
    anchors a [K, 3] and unit directions w [K, 3]."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float32))
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3))
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1, 3))
    out = np.empty(a.shape[0])
    N = _dims(c.shape[::-1])
    if _load().or_project_lines(n, _ptr(c), _ptr(N), a.shape[0], _ptr(a), _ptr(w), _ptr(out)):
        raise ValueError("bad degree or size")
    return out


def project_basis_sum(c, geom, n: int = 3, rays=None) -> np.ndarray:
    """O5: the same transform as sum_q c_q * footprint (eq. (4))."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float32))
    dims = _dims(c.shape[::-1])
    vecs, g = _geom_args(geom)
    total = g[1] * g[2] * g[3]
    idx, cnt = _idx(rays, total)
    out = np.empty(cnt)
    rc = _load().or_project_basis_sum(n, _ptr(c), _ptr(dims), *g, _ptr(vecs),
                                      None if idx is None else _ptr(idx), cnt, _ptr(out))
    if rc:
        raise ValueError("oracle basis-sum failed")
    return out if rays is not None else out.reshape(g[1], g[2], g[3])


def counts(dims, geom, n: int = 3, rays=None):
    """O9: per-ray number of (ray, basis) pairs with a non-empty chord, and the
    number of polynomial segments of their footprints."""
    dims = _dims(dims)
    vecs, g = _geom_args(geom)
    total = g[1] * g[2] * g[3]
    idx, cnt = _idx(rays, total)
    pairs = np.empty(cnt, dtype=np.int64)
    segs = np.empty(cnt, dtype=np.int64)
    rc = _load().or_counts(n, _ptr(dims), *g, _ptr(vecs), None if idx is None else _ptr(idx), cnt,
                           _ptr(pairs), _ptr(segs))
    if rc:
        raise ValueError("oracle counts failed")
    return pairs, segs


def direct_counts(dims, geom, n: int = 3, rays=None):
    """O9: per-ray number of polynomial segments of the direct integral (the
    knot cells of the support-padded box each line passes through)."""
    dims = _dims(dims)
    vecs, g = _geom_args(geom)
    total = g[1] * g[2] * g[3]
    idx, cnt = _idx(rays, total)
    segs = np.empty(cnt, dtype=np.int64)
    rc = _load().or_direct_counts(n, _ptr(dims), *g, _ptr(vecs), None if idx is None else _ptr(idx), cnt,
                                  _ptr(segs))
    if rc:
        raise ValueError("oracle direct counts failed")
    return segs


def backproject_subset(y, geom, dims, n: int = 3, coefs=None) -> np.ndarray:
    """O6: (A^T y)_q = sum_r y_r P phi(w_r, a_r - x_q), transpose of eq. (7),
    for the flat coefficient indices ``coefs`` (all if None).  ``dims`` is
    (N1, N2, N3)."""
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float32))
    dims = _dims(dims)
    vecs, g = _geom_args(geom)
    if y.size != g[1] * g[2] * g[3]:
        raise ValueError("sinogram size mismatch")
    total = int(dims.prod())
    idx, cnt = _idx(coefs, total)
    out = np.empty(cnt)
    rc = _load().or_backproject_subset(n, _ptr(y), _ptr(dims), *g, _ptr(vecs),
                                       None if idx is None else _ptr(idx), cnt, _ptr(out))
    if rc:
        raise ValueError("oracle backprojection failed")
    return out if coefs is not None else out.reshape(int(dims[2]), int(dims[1]), int(dims[0]))


def dense_matrix(dims, geom, n: int = 3, rays=None) -> np.ndarray:
    """O7: eq. (7) as a dense [rays, N3*N2*N1] FP64 matrix (tiny sizes only)."""
    dims = _dims(dims)
    vecs, g = _geom_args(geom)
    total = g[1] * g[2] * g[3]
    idx, cnt = _idx(rays, total)
    nq = int(dims.prod())
    if cnt * nq > 5e7:
        raise ValueError("dense matrix too large")
    A = np.empty((cnt, nq))
    rc = _load().or_dense_matrix(n, _ptr(dims), *g, _ptr(vecs), None if idx is None else _ptr(idx),
                                 cnt, _ptr(A))
    if rc:
        raise ValueError("oracle dense matrix failed")
    return A


from .cgls import cgls  # noqa: E402,F401
