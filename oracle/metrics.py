"""Accuracy measures of section 5 (oracle; test infrastructure only)."""
from __future__ import annotations

import numpy as np


def probe_rel_error(ref_apply, test_apply, G=None):
    """|| (A_test - A_ref) G ||_F / || A_ref G ||_F on a probe block G.

    ``ref_apply``/``test_apply`` are callables returning A G, or arrays that
    already hold A G."""
    R = ref_apply(G) if callable(ref_apply) else np.asarray(ref_apply)
    T = test_apply(G) if callable(test_apply) else np.asarray(test_apply)
    return float(np.linalg.norm(T - R) / np.linalg.norm(R))


def power_norm(matvec, rmatvec, n, steps=20, rng=None, v0=None):
    """Operator 2-norm estimate of section 5: start from a random v_0 (or the
    given one) and take v_i = B^* B (v_{i-1} / ||v_{i-1}||), i = 1..steps;
    return sqrt(||v_steps||)."""
    if v0 is None:
        rng = np.random.default_rng(0) if rng is None else rng
        v = rng.standard_normal(n)
    else:
        v = np.array(v0, dtype=np.float64).reshape(n)
    for _ in range(steps):
        nv = np.linalg.norm(v)
        if nv == 0.0:  # B v_{i-1} = 0: the iteration has stopped at the zero vector
            return 0.0
        v = rmatvec(matvec(v / nv))
    return float(np.sqrt(np.linalg.norm(v)))


def power_rel_error(apply_a, rapply_a, apply_b, rapply_b, n, steps=20, seed=0):
    """||B - A|| / ||A|| with both norms estimated by ``power_norm``."""
    num = power_norm(lambda v: apply_b(v) - apply_a(v), lambda v: rapply_b(v) - rapply_a(v), n, steps,
                     np.random.default_rng(seed))
    den = power_norm(apply_a, rapply_a, n, steps, np.random.default_rng(seed + 1))
    return num / den
