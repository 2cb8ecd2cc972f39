"""Input generators: geometries and the analytic ellipsoid line integrals
that simulate measured data for the reconstruction analog."""
import numpy as np

from paper_2511_11078_amd import synth


def test_sphere_chords():
    params = [(np.zeros(3), np.array([0.5, 0.5, 0.5]), np.eye(3), 2.0)]
    dims = (41, 41, 41)  # normalised radius 0.5 -> world radius 10
    offs = np.array([0.0, 3.0, 6.0, 9.5, 10.5])
    vecs = np.zeros((1, 12))
    vecs[0, 0:3] = [0.0, 0.0, 1.0]
    vecs[0, 6] = 1.0
    vecs[0, 10] = 1.0
    g = synth.Geometry("parallel", 1, 1, 1, vecs.astype(np.float32))
    for o in offs:
        g.vecs[0, 3] = o
        want = 2.0 * 2.0 * np.sqrt(max(0.0, 100.0 - o * o))
        assert abs(synth.ellipsoid_line_integrals(dims, g, params)[0, 0, 0] - want) < 1e-4


def test_rotated_ellipsoid_against_ray_marching():
    rng = np.random.default_rng(3)
    params = synth.ellipsoid_params(2, seed=4)
    dims = (30, 26, 22)
    geom = synth.cone_circular_geometry(2, 3, 4, src_radius=60.0, src_det=90.0, angle0=0.3)
    y = synth.ellipsoid_line_integrals(dims, geom, params)
    D = 1.0 / (0.5 * (np.array(dims) - 1.0))
    vec = geom.vecs.astype(np.float64)
    t = np.linspace(0.0, 200.0, 400001)
    dt = t[1] - t[0]
    for v in range(2):
        for j in range(3):
            for i in range(4):
                e = vec[v]
                pix = e[3:6] + (i - 1.5) * e[6:9] + (j - 1.0) * e[9:12]
                d = (pix - e[0:3]) / np.linalg.norm(pix - e[0:3])
                x = e[0:3][None, :] + t[:, None] * d[None, :]
                val = np.zeros(t.size)
                for cen, axes, rot, rho in params:
                    loc = ((x * D - cen) @ rot) / axes
                    val += rho * ((loc ** 2).sum(1) <= 1.0)
                assert abs(val.sum() * dt - y[v, j, i]) < 5e-3
