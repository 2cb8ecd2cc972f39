"""Reconstruction analog of the paper's experiment (Sec. 3): 50 CGLS
iterations on analytic cone-beam data of a 180 x 180 x 50 ellipsoid phantom
with noise of variance 1e-3, quadratic splines vs voxels.  The paper's
qualitative finding -- the spline basis reconstructs with a higher PSNR than
the voxel basis -- must hold; the numbers themselves are context."""
import pytest

from paper_2511_11078_amd import recon

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_spline_beats_voxel_psnr():
    res = recon.run(iters=50, noise_var=1e-3, log=say)
    assert res["psnr_degree2"] > res["psnr_degree0"] + 1.0
