"""The five synthetic workloads, by size and acquisition.

The paper's experiment (Sec. 3) reconstructs a 180 x 180 x 50 BrainWeb volume
from 200 cone-beam views; those data are not available, so these seeded
phantoms and geometries stand in for it (see ``synth``).  Names describe
the workload; ``degree`` is the B-spline degree of the basis.

  small_parallel_32  32^3, 6 ellipsoids, parallel beam, 32 spherical-Fibonacci
                     directions, 48 x 48 detector (checker runs it in full)
  parallel_128       128^3, ellipsoids + N(0, 0.01) noise, parallel beam,
                     180 great-circle + 60 random directions, 192 x 192
  cone_256           256^3, ellipsoids, circular cone beam of 360 views,
                     source radius 640 (2.5 x extent), source-detector 768,
                     384 x 384 detector (magnification 1.5 at the near face)
  cone_512           512^3 smoothed random field (sigma 4), 720 views, same
                     ratios (radius 1280, source-detector 1536), 768 x 768,
                     processed in batches of 32 views
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import synth


@dataclass
class Workload:
    name: str
    dims: tuple            # (N1, N2, N3)
    degree: int
    views_per_batch: int = 0  # 0 = all views in one call
    notes: str = ""
    _geom: object = field(default=None, repr=False)

    def geometry(self):
        if self._geom is None:
            self._geom = _GEOMS[self.name]()
        return self._geom

    def volume(self) -> np.ndarray:
        return _VOLUMES[self.name](self.dims)


def _g_small():
    return synth.parallel_geometry(synth.fibonacci_directions(32), 48, 48)


def _g_p128():
    return synth.parallel_geometry(synth.great_circle_plus_tilts(180, 60, seed=2), 192, 192)


def _g_c256():
    return synth.cone_circular_geometry(360, 384, 384, src_radius=640.0, src_det=768.0)


def _g_c512():
    return synth.cone_circular_geometry(720, 768, 768, src_radius=1280.0, src_det=1536.0)


_GEOMS = {"small_parallel_32": _g_small, "parallel_128": _g_p128, "cone_256": _g_c256, "cone_512": _g_c512}
_VOLUMES = {
    "small_parallel_32": lambda d: synth.ellipsoid_phantom(d, 6, seed=0),
    "parallel_128": lambda d: synth.add_noise(synth.ellipsoid_phantom(d, 6, seed=0), 0.01, seed=1),
    "cone_256": lambda d: synth.ellipsoid_phantom(d, 6, seed=0),
    "cone_512": lambda d: synth.smooth_field(d, 4.0, seed=6),
}

WORKLOADS = {
    "small_parallel_32": Workload("small_parallel_32", (32, 32, 32), 3),
    "parallel_128": Workload("parallel_128", (128, 128, 128), 3),
    "cone_256": Workload("cone_256", (256, 256, 256), 3),
    "cone_512": Workload("cone_512", (512, 512, 512), 3, views_per_batch=32),
}


def get(name: str) -> Workload:
    return WORKLOADS[name]
