"""ctypes binding of libsplinesplat.so (include/splinesplat.h).

Argument marshalling only: every step of the transform runs in the HIP
library.  Tensors are PyTorch CUDA (ROCm) tensors used for device memory and
streams; they are passed as raw device pointers together with torch's
current HIP stream.  If the library is missing this module raises: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsplinesplat.so")
ABI_VERSION = 2  # SS_ABI_VERSION of include/splinesplat.h

SS_OK, SS_EINVAL, SS_ENOMEM, SS_EDEVICE, SS_EUNSUPPORTED, SS_EBLOB = range(6)
FORMS = {"quad": 0, "mlp": 1, "pair": 2}
KINDS = {"parallel": 0, "cone": 1}
STATUS_NAMES = {0: "SS_OK", 1: "SS_EINVAL", 2: "SS_ENOMEM", 3: "SS_EDEVICE", 4: "SS_EUNSUPPORTED",
                5: "SS_EBLOB"}

EXPORTED = ["ss_create", "ss_destroy", "ss_project", "ss_backproject", "ss_footprint", "ss_dot_f64",
            "ss_cgls_scalars", "ss_axpy", "ss_xpay", "ss_validate_problem", "ss_last_error", "ss_query",
            "ss_abi_version", "ss_project_noalloc", "ss_set_scratch_limit"]


class SSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ss_geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_views", ctypes.c_int32), ("det_rows", ctypes.c_int32),
                ("det_cols", ctypes.c_int32), ("vecs", ctypes.c_void_p)]


_lib = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_11078_amd.build` "
                           "(the transform has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, L, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.ss_create.argtypes = [ctypes.POINTER(P), I, I, I, P, ctypes.c_size_t]
    lib.ss_destroy.argtypes = [P]
    lib.ss_project.argtypes = [P, P, P, ctypes.POINTER(ss_geometry), P, P]
    lib.ss_backproject.argtypes = [P, P, ctypes.POINTER(ss_geometry), P, P, P]
    lib.ss_project_noalloc.argtypes = [I, I, P, P, ctypes.POINTER(ss_geometry), P, P]
    lib.ss_footprint.argtypes = [P, P, P, L, P, P]
    lib.ss_set_scratch_limit.argtypes = [P, ctypes.c_size_t]
    lib.ss_dot_f64.argtypes = [P, P, P, L, P, P]
    lib.ss_cgls_scalars.argtypes = [P, P, P, P, P]
    lib.ss_axpy.argtypes = [P, P, I, P, P, L, P]
    lib.ss_xpay.argtypes = [P, P, P, P, L, P]
    lib.ss_validate_problem.argtypes = [P, ctypes.POINTER(ss_geometry)]
    lib.ss_last_error.restype = ctypes.c_char_p
    lib.ss_last_error.argtypes = []
    lib.ss_query.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.ss_abi_version.restype = I
    for name in EXPORTED:
        if name != "ss_last_error":
            getattr(lib, name).restype = I
    if lib.ss_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} reports ABI version {lib.ss_abi_version()}, the binding expects "
                           f"{ABI_VERSION}: rebuild it with `python -m paper_2511_11078_amd.build`")
    _lib = lib
    return lib


def last_error() -> str:
    return load().ss_last_error().decode()


def check(status: int):
    if status != SS_OK:
        raise SSError(status, last_error())


class GeometryArg:
    """Keeps the host vecs alive while the ss_geometry struct points at them."""

    def __init__(self, geom):
        self.vecs = np.ascontiguousarray(np.asarray(geom.vecs, dtype=np.float32).reshape(-1, 12))
        self.struct = ss_geometry(KINDS[geom.kind] if isinstance(geom.kind, str) else int(geom.kind),
                                  int(geom.n_views), int(geom.det_rows), int(geom.det_cols),
                                  self.vecs.ctypes.data_as(ctypes.c_void_p))

    def ref(self):
        return ctypes.byref(self.struct)


def dims_arg(dims):
    d = (ctypes.c_int64 * 3)(*[int(x) for x in dims])
    return d


def validate_problem(dims, geom):
    """Host-only validation (no GPU needed); raises SSError."""
    g = GeometryArg(geom)
    check(load().ss_validate_problem(dims_arg(dims), g.ref()))
