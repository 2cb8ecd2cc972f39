"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point the header declares, and rejects bad arguments before touching a
device.  Also checks the device quadrature constants against numpy."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2511_11078_amd import _lib, footprint_net, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "splinesplat.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ss_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert "ss_project" in names and "ss_backproject" in names
    for name in names:
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {_lib.LIB_PATH}").read()
    for name in names:
        assert re.search(rf"\bT {name}\b", out), f"{name} not exported"
    assert lib.ss_abi_version() == _lib.ABI_VERSION == 2


def test_validation_errors():
    g = synth.parallel_geometry(synth.fibonacci_directions(3), 4, 5)
    _lib.validate_problem((4, 5, 6), g)
    for dims in [(0, 4, 4), (4, -1, 4), (4, 4, 5000), (4096, 4096, 4096)]:
        with pytest.raises(_lib.SSError) as e:
            _lib.validate_problem(dims, g)
        assert e.value.status == _lib.SS_EINVAL
    bad = []
    g1 = synth.parallel_geometry(synth.fibonacci_directions(3), 4, 5)
    g1.vecs[1, 4] = np.inf
    bad.append(g1)
    g2 = synth.parallel_geometry(synth.fibonacci_directions(3), 4, 5)
    g2.vecs[0, 0:3] = 0.0
    bad.append(g2)
    g3 = synth.parallel_geometry(synth.fibonacci_directions(3), 4, 5)
    g3.vecs[2, 0:3] = g3.vecs[2, 6:9]  # direction inside the detector plane
    bad.append(g3)
    g4 = synth.cone_circular_geometry(2, 4, 4, 10.0, 15.0)
    g4.vecs[1, 0:3] = g4.vecs[1, 3:6]  # source on the detector
    bad.append(g4)
    g5 = synth.Geometry("cone", 0, 4, 4, np.zeros((0, 12), np.float32))
    bad.append(g5)
    g6 = synth.Geometry(7, 1, 4, 4, np.zeros((1, 12), np.float32))
    bad.append(g6)
    for g in bad:
        with pytest.raises(_lib.SSError) as e:
            _lib.validate_problem((4, 4, 4), g)
        assert e.value.status == _lib.SS_EINVAL
        assert _lib.last_error()
    big = synth.Geometry("parallel", 1, 50000, 50000, synth.parallel_geometry([[0, 0, 1.0]], 1, 1).vecs)
    with pytest.raises(_lib.SSError):
        _lib.validate_problem((4, 4, 4), big)


def _create(degree, form, blob=None, nbytes=None):
    lib = _lib.load()
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(blob, len(blob)) if blob is not None else None
    n = len(blob) if (blob is not None and nbytes is None) else (nbytes or 0)
    return lib.ss_create(ctypes.byref(h), 0, degree, form, buf, n), h


def test_create_argument_errors_need_no_gpu():
    lib = _lib.load()
    assert lib.ss_create(None, 0, 3, 0, None, 0) == _lib.SS_EINVAL
    assert _create(4, 0)[0] == _lib.SS_EINVAL
    assert _create(-1, 0)[0] == _lib.SS_EINVAL
    assert _create(3, 7)[0] == _lib.SS_EINVAL
    assert _create(0, 1)[0] == _lib.SS_EUNSUPPORTED
    assert _create(3, 1)[0] == _lib.SS_EBLOB            # no blob
    assert _create(3, 0, b"x" * 8)[0] == _lib.SS_EINVAL  # blob for the quadrature form
    assert _create(3, 2, b"x" * 8)[0] == _lib.SS_EINVAL  # blob for the per-pair exact form
    assert _create(3, 3)[0] == _lib.SS_EINVAL            # no such form
    good = bytearray(footprint_net.blob_bytes())
    assert _create(3, 1, bytes(good[:-1]))[0] == _lib.SS_EBLOB    # wrong size
    assert _create(3, 1, bytes(good))[0] == _lib.SS_EBLOB         # bad magic
    import struct
    hdr = struct.pack(footprint_net.HEADER_FMT, footprint_net.MAGIC, 1, 2, 5, 64, 4, 1, 1, 3, 0.0, 0.0)
    blob = hdr + bytes(footprint_net.blob_bytes() - len(hdr))
    st, _ = _create(3, 1, blob)
    assert st == _lib.SS_EBLOB and "degree" in _lib.last_error()
    hdr = struct.pack(footprint_net.HEADER_FMT, footprint_net.MAGIC, 1, 3, 5, 32, 4, 1, 1, 3, 0.0, 0.0)
    st, _ = _create(3, 1, hdr + bytes(footprint_net.blob_bytes() - len(hdr)))
    assert st == _lib.SS_EBLOB


def test_null_context_is_rejected():
    lib = _lib.load()
    g = _lib.GeometryArg(synth.parallel_geometry(synth.fibonacci_directions(2), 3, 3))
    d = _lib.dims_arg((3, 3, 3))
    P = ctypes.c_void_p(1)
    assert lib.ss_project(None, P, d, g.ref(), P, None) == _lib.SS_EINVAL
    assert lib.ss_backproject(None, P, g.ref(), d, P, None) == _lib.SS_EINVAL
    assert lib.ss_footprint(None, P, P, 4, P, None) == _lib.SS_EINVAL
    assert lib.ss_dot_f64(None, P, P, 4, P, None) == _lib.SS_EINVAL
    assert lib.ss_cgls_scalars(None, P, P, P, None) == _lib.SS_EINVAL
    assert lib.ss_axpy(None, P, 1, P, P, 4, None) == _lib.SS_EINVAL
    assert lib.ss_xpay(None, P, P, P, 4, None) == _lib.SS_EINVAL
    assert lib.ss_query(None, None, None, None) == _lib.SS_EINVAL
    assert lib.ss_set_scratch_limit(None, 1 << 20) == _lib.SS_EINVAL
    assert lib.ss_destroy(None) == _lib.SS_OK
    assert "NULL" in _lib.last_error() or "context" in _lib.last_error()


def test_device_gauss_legendre_constants():
    src = open(os.path.join(ROOT, "paper_2511_11078_amd", "csrc", "ss_math.hpp")).read()
    for m in (2, 4, 5):
        block = re.search(rf"struct GLRule<{m}> \{{(.*?)\n\}};", src, re.S).group(1)
        xs = sorted(set(abs(float(v)) for v in re.findall(r"(-?\d+\.\d+)f", block.split("w(")[0])))
        ws = sorted(set(float(v) for v in re.findall(r"(\d+\.\d+)f", block.split("w(")[1])))
        xr, wr = np.polynomial.legendre.leggauss(m)
        np.testing.assert_allclose(xs, sorted(set(np.round(np.abs(xr), 15))), atol=1e-15)
        np.testing.assert_allclose(ws, sorted(set(np.round(wr, 15))), atol=1e-15)


def test_binding_rejects_wrongly_sized_buffers():
    """The binding checks every buffer's shape before the library sees its
    pointer (no GPU: the check comes before any device access)."""
    import torch

    from paper_2511_11078_amd.ops import Context

    ctx = object.__new__(Context)  # no device context needed for argument checks
    ctx.device, ctx._h, ctx._lib = 0, None, None
    g = synth.parallel_geometry(synth.fibonacci_directions(3), 4, 5)
    c = torch.zeros(6, 5, 4)
    with pytest.raises(ValueError):
        ctx.project(c, g, out=torch.zeros(3, 4, 4))
    with pytest.raises(ValueError):
        ctx.project(c, g, out=torch.zeros(3 * 4 * 5))
    with pytest.raises(ValueError):
        ctx.backproject(torch.zeros(3, 4, 5), g, (4, 5, 6), out=torch.zeros(6, 5, 3))
    with pytest.raises(ValueError):
        ctx.backproject(torch.zeros(3, 5, 4), g, (4, 5, 6), out=torch.zeros(6, 5, 4))
    with pytest.raises(ValueError):
        ctx.footprint(torch.zeros(8, 3), torch.zeros(7, 3))
    with pytest.raises(ValueError):
        ctx.dot_f64(torch.zeros(4), torch.zeros(4), out=torch.zeros(2, dtype=torch.float64))
    with pytest.raises(ValueError):
        ctx.axpy(torch.zeros(2, dtype=torch.float64), 1, torch.zeros(4), torch.zeros(4))


def test_noalloc_forward_rejects_oversized_problems_before_any_device_call():
    lib = _lib.load()
    g = _lib.GeometryArg(synth.parallel_geometry(synth.fibonacci_directions(2), 3, 3))
    fake = ctypes.c_void_p(256)
    # (400 + 8)^3 padded floats exceed the 96 MiB static scratch
    assert lib.ss_project_noalloc(0, 3, fake, _lib.dims_arg((400, 400, 400)), g.ref(), fake, None) == _lib.SS_EINVAL
    assert "static scratch" in _lib.last_error()
    assert lib.ss_project_noalloc(0, 4, fake, _lib.dims_arg((8, 8, 8)), g.ref(), fake, None) == _lib.SS_EINVAL
    assert lib.ss_project_noalloc(0, 3, None, _lib.dims_arg((8, 8, 8)), g.ref(), fake, None) == _lib.SS_EINVAL
