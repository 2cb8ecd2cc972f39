"""O8: FP64 CGLS -- TEST INFRASTRUCTURE ONLY (part of the oracle).

The reconstruction of Sec. 3 runs 50 iterations of conjugate gradients on the
unregularised least-squares problem  min_c ||P c - y||^2  (eq. (6)).  This is
the textbook CGLS recurrence (CG applied to the normal equations without
forming them), x_0 = 0, no preconditioner:

    r = y, s = A^T r, p = s, gamma = <s, s>
    repeat:  q = A p;  alpha = gamma / <q, q>
             x += alpha p;  r -= alpha q
             s = A^T r;  gamma' = <s, s>;  beta = gamma' / gamma
             p = s + beta p;  gamma = gamma'
"""
from __future__ import annotations

import numpy as np


def cgls(A, At, y, iters: int, x_shape=None):
    """Run ``iters`` CGLS iterations in FP64.

    ``A`` and ``At`` are callables (x -> A x, r -> A^T r) on FP64 arrays.
    Returns (x, history) where history[k] = (||r_k||, ||s_k||) after k
    iterations (k = 0 is the start)."""
    y = np.asarray(y, dtype=np.float64)
    r = y.copy()
    s = np.asarray(At(r), dtype=np.float64)
    x = np.zeros_like(s)
    p = s.copy()
    gamma = float(np.vdot(s, s))
    hist = [(float(np.linalg.norm(r)), float(np.sqrt(gamma)))]
    for _ in range(iters):
        if gamma == 0.0:
            hist.append(hist[-1])
            continue
        q = np.asarray(A(p), dtype=np.float64)
        alpha = gamma / float(np.vdot(q, q))
        x = x + alpha * p
        r = r - alpha * q
        s = np.asarray(At(r), dtype=np.float64)
        gamma_new = float(np.vdot(s, s))
        beta = gamma_new / gamma
        p = s + beta * p
        gamma = gamma_new
        hist.append((float(np.linalg.norm(r)), float(np.sqrt(gamma))))
    if x_shape is not None:
        x = x.reshape(x_shape)
    return x, hist
