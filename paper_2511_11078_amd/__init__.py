"""MI355X (gfx950) spline x-ray transform -- forward model of SplineSplat
(arXiv 2511.11078), its matched adjoint, autograd wiring and CGLS.

The HIP library (``libsplinesplat.so``, C ABI in ``include/splinesplat.h``)
does all the arithmetic; build it with ``python -m paper_2511_11078_amd.build``.
``synth`` and ``configs`` hold the seeded synthetic inputs.
"""
from . import configs, synth  # noqa: F401

__all__ = ["synth", "configs", "Context", "Projector", "Project", "Backproject", "project", "cgls"]


def __getattr__(name):
    if name in ("Context", "Projector", "Project", "Backproject", "project", "cgls"):
        from . import ops
        return getattr(ops, name)
    raise AttributeError(name)
