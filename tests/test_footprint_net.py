"""CPU pins of the training-side helpers of the footprint network: the FP64
label generator equals the oracle's single-basis footprint (O4), the fold
is invariant under the 48 signed axis permutations and keeps the line's
perpendicular offset, and the blob evaluator's arithmetic modes order as
expected."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2511_11078_amd import footprint_net as fn
from paper_2511_11078_amd import train_footprint as tf


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_training_labels_equal_oracle_footprint(n):
    rng = np.random.default_rng(11 + n)
    w, x = tf.sample_pairs(n, 20000, rng)
    # also lines parallel to a lattice axis and to a coordinate plane
    w2 = np.array([[0.0, 0.0, 1.0], [0.0, 0.6, 0.8], [1.0, 0.0, 0.0]] * 200)
    x2 = rng.uniform(-0.5 * (n + 1), 0.5 * (n + 1), (600, 3))
    w = np.concatenate([w, w2])
    x = np.concatenate([x, x2])
    got = fn.exact_footprint(n, w, x)
    want = oracle.footprint(n, w, x)
    assert np.max(np.abs(got - want)) <= 1e-13 * max(1.0, np.max(np.abs(want)))


def test_fold_is_invariant_and_keeps_the_offset():
    rng = np.random.default_rng(5)
    w, x = tf.sample_pairs(3, 2000, rng)
    f = fn.fold_features(w, x)
    assert np.all(f[:, 0] <= f[:, 1] + 1e-15) and np.all(f[:, 1] <= f[:, 2] + 1e-15) and np.all(f[:, 0] >= 0)
    # (u.x, v.x) is the offset of the line from the basis centre in a frame of its plane
    perp = x - (x * w).sum(1, keepdims=True) * w
    assert np.allclose(f[:, 3] ** 2 + f[:, 4] ** 2, (perp ** 2).sum(1), atol=1e-12)
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([-1.0, 1.0], repeat=3):
            s = np.array(signs)
            g = fn.fold_features(w[:, perm] * s, x[:, perm] * s)
            # equal up to the ordering of equal |w| components (measure zero here)
            assert np.allclose(g, f, atol=1e-12)


def test_blob_arithmetic_modes():
    blob = fn.parse_blob(open(fn.__file__.replace("footprint_net.py", "weights/mlp_n3.bin"), "rb").read())
    rng = np.random.default_rng(9)
    w, x = tf.sample_pairs(3, 20000, rng)
    f = fn.fold_features(w, x).astype(np.float32)
    exact = fn.blob_forward(blob, f, activations="fp32").astype(np.float64)
    split = fn.blob_forward(blob, f, activations="split").astype(np.float64)
    once = fn.blob_forward(blob, f, activations="bf16").astype(np.float64)
    e_split = np.linalg.norm(split - exact) / np.linalg.norm(exact)
    e_once = np.linalg.norm(once - exact) / np.linalg.norm(exact)
    # two BF16 terms keep ~16 bits of each activation, one keeps ~8
    assert e_split < 2e-5 < e_once
