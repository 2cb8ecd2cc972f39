"""Shared helpers of the GPU tests (parity against the FP64 oracle)."""
import numpy as np
import torch

from paper_2511_11078_amd import synth

DEV = 0


def dev():
    return torch.device("cuda", DEV)


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def to_np(t):
    return t.detach().cpu().numpy()


def rel_l2(got, want):
    got = np.asarray(got, dtype=np.float64).ravel()
    want = np.asarray(want, dtype=np.float64).ravel()
    den = np.linalg.norm(want)
    return float(np.linalg.norm(got - want) / (den if den > 0 else 1.0))


def say(msg):
    print(msg, flush=True)


def tilted_parallel(n_views, R, C, seed, pitch=1.0):
    return synth.parallel_geometry(synth.uniform_directions(n_views, seed=seed), R, C, pitch=pitch)
