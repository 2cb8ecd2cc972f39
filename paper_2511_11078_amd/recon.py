"""Reconstruction-quality analog of the paper's experiment (Sec. 3).

The paper reconstructs a 180 x 180 x 50 BrainWeb volume from 200 cone-beam
views around one axis (detector 180 x 50, Gaussian noise of variance 1e-3,
50 iterations of least-squares conjugate gradients) with quadratic splines
and with voxels, and compares PSNR.  BrainWeb and ASTRA are not available, so
this analog uses a continuous ellipsoid phantom inside the inscribed
cylinder, whose measurements are exact analytic line integrals
(``synth.ellipsoid_line_integrals``), and reconstructs the same data with the
degree-2 spline basis and with the degree-0 (voxel) basis.  PSNR compares
the reconstructed function, sampled at the lattice points, with the phantom
sampled there.  The numbers are context, not a reproduction.

    python -m paper_2511_11078_amd.recon [--iters 50] [--noise-var 1e-3]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import synth

DIMS = (180, 180, 50)  # (N1, N2, N3); the rotation axis is e3 (50 samples)


def geometry(n_views: int = 200):
    # circular cone beam around e3; the detector passes through the rotation
    # axis (unit magnification there): 180 columns across, 50 rows along e3
    return synth.cone_circular_geometry(n_views, 50, 180, src_radius=450.0, src_det=450.0)


def phantom_params(seed: int = 11):
    # ellipsoids kept inside the cylinder the detector covers at every angle
    return synth.ellipsoid_params(8, seed=seed, centre_radius=0.4, max_axis=0.45)


def spline_samples(c: np.ndarray, degree: int) -> np.ndarray:
    """f(x_k) = sum_q c_q beta^n(k - q) (separable filter of the integer
    samples of beta^n)."""
    taps = {0: [1.0], 1: [1.0], 2: [0.125, 0.75, 0.125], 3: [1 / 6, 2 / 3, 1 / 6]}[degree]
    out = c.astype(np.float64)
    if len(taps) == 1:
        return out
    k = np.asarray(taps)
    for axis in range(3):
        pad = [(0, 0)] * 3
        pad[axis] = (1, 1)
        p = np.pad(out, pad)
        sl = [slice(None)] * 3
        acc = 0.0
        for i, t in enumerate(k):
            sl[axis] = slice(i, i + out.shape[axis])
            acc = acc + t * p[tuple(sl)]
        out = acc
    return out


def psnr(x, ref):
    mse = float(np.mean((x - ref) ** 2))
    return 10.0 * np.log10(float(ref.max() - ref.min()) ** 2 / mse)


def run(iters: int = 50, noise_var: float = 1e-3, seed: int = 12, degrees=(2, 0), log=print):
    import torch

    from .ops import Projector, cgls

    geom = geometry()
    params = phantom_params()
    truth = synth.ellipsoid_phantom(DIMS, params=params).astype(np.float64)
    y = synth.ellipsoid_line_integrals(DIMS, geom, params)
    rng = np.random.default_rng(seed)
    y = (y + rng.standard_normal(y.shape) * np.sqrt(noise_var)).astype(np.float32)
    yd = torch.from_numpy(y).cuda()
    res = {"dims": list(DIMS), "views": geom.n_views, "detector": [geom.det_rows, geom.det_cols],
           "noise_variance": noise_var, "iterations": iters}
    for n in degrees:
        P = Projector(DIMS, geom, degree=n, form="quad")
        x, hist = cgls(P, yd, iters=iters)
        torch.cuda.synchronize()
        f = spline_samples(x.cpu().numpy(), n)
        res[f"psnr_degree{n}"] = psnr(f, truth)
        res[f"residual_degree{n}"] = float((P.forward(x) - yd).double().norm() / yd.double().norm())
        log(f"degree {n}: PSNR {res[f'psnr_degree{n}']:.2f} dB, relative residual {res[f'residual_degree{n}']:.3e}")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--noise-var", type=float, default=1e-3)
    a = ap.parse_args()
    print(json.dumps(run(a.iters, a.noise_var)))


if __name__ == "__main__":
    main()
