"""Seeded synthetic inputs for black-box HBS compression.

This module only draws random numbers and lays out geometry.  It performs none
of the compression or apply arithmetic of the method, so the CPU oracle and the
GPU path can both take their inputs from here without sharing any code of the
method itself.

Streams: every workload id gets its own ``numpy.random.SeedSequence`` rooted at
``SEED_ROOT``; the spawned children are used in a fixed order

    0  generator factors of a synthetic HBS matrix (U, V, D per node)
    1  the test matrix Omega (N x s)
    2  the test matrix Psi (N x s)
    3  probe vectors for the apply error
    4  sampled row indices (log-kernel reference rows)

so that a given (workload, stream) pair is reproducible on any machine.
"""
from __future__ import annotations

import math

import numpy as np

SEED_ROOT = 220502990

STREAM_GENERATOR = 0
STREAM_OMEGA = 1
STREAM_PSI = 2
STREAM_PROBES = 3
STREAM_ROWS = 4

# The five workloads.  "leaf_max" is the leaf-size threshold of the cluster tree
# (nodes are split while any node at the level is larger than it).
WORKLOADS = {
    # exact-rank synthetic HBS, 32 leaves of 32, five levels below the root
    "hbs_exact_n1024_k16": dict(id=1, kind="synthetic", n=1024, k=16, leaf_max=32, s=58),
    # log|x_i - x_j| on 65536 ellipse points, k = 50, leaf threshold 100, s = 160
    "logkernel_ellipse_n65536_k50": dict(id=2, kind="logkernel", n=65536, k=50, leaf_max=100, s=160,
                                         a=1.0, b=0.5),
    # same kernel at N = 2^18, k = 64, leaf 128, s = 202
    "logkernel_ellipse_n262144_k64": dict(id=3, kind="logkernel", n=262144, k=64, leaf_max=128, s=202,
                                          a=1.0, b=0.5),
    # 512 independent exact-rank instances of uneven N
    "hbs_exact_batch512": dict(id=4, kind="batch", count=512, n_lo=2048, n_hi=32768, ks=(16, 32)),
    # one large exact-rank instance, 16 levels
    "hbs_exact_n4194304_k32": dict(id=5, kind="synthetic", n=4194304, k=32, leaf_max=64, s=106),
}


def streams(workload_id: int, count: int = 5, extra: tuple = ()) -> list:
    """Independent generators for one workload (order fixed in the module docstring)."""
    ss = np.random.SeedSequence([SEED_ROOT, int(workload_id), *[int(e) for e in extra]])
    return [np.random.default_rng(c) for c in ss.spawn(count)]


def gaussian(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """rows x cols matrix of i.i.d. standard normal FP64 entries, C-contiguous."""
    return np.ascontiguousarray(rng.standard_normal((rows, cols)))


def random_orthonormal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """rows x cols matrix with orthonormal columns: a Gaussian matrix whose
    columns are orthonormalised.  This only shapes the input distribution."""
    g = rng.standard_normal((rows, cols))
    q, _ = np.linalg.qr(g)
    return np.ascontiguousarray(q[:, :cols])


def synthetic_generators(rng: np.random.Generator, leaf_sizes, k: int) -> dict:
    """Random factors of an HBS matrix of exact block rank k.

    ``leaf_sizes`` lists the leaf sizes left to right (2^L of them, taken from
    the caller's own cluster tree).  Draw order, level by level from the
    leaves (L) up to level 1: one Gaussian block for every U of the level,
    one for every V, one for every D (nodes x m_max x m_max, node i keeping
    its leading m_i x m_i part); then the root block.  Leaf U, V are m x k
    with orthonormal columns; inner U, V are 2k x k; every D is standard
    normal (m x m at leaves, 2k x 2k above); the root block is 2k x 2k, or
    N x N when the tree is a single leaf.
    """
    leaf_sizes = [int(m) for m in leaf_sizes]
    nleaf = len(leaf_sizes)
    L = int(round(math.log2(nleaf)))
    if 2 ** L != nleaf:
        raise ValueError("leaf count must be a power of two")
    out = {"L": L, "k": int(k), "U": {}, "V": {}, "D": {}, "D0": None}
    if L == 0:
        out["D0"] = gaussian(rng, leaf_sizes[0], leaf_sizes[0])
        return out
    for lev in range(L, 0, -1):
        sizes = leaf_sizes if lev == L else [2 * k] * (2 ** lev)
        out["U"][lev] = _orthonormal_blocks(rng, sizes, k)
        out["V"][lev] = _orthonormal_blocks(rng, sizes, k)
        mm = max(sizes)
        Dall = rng.standard_normal((len(sizes), mm, mm))
        out["D"][lev] = [np.ascontiguousarray(Dall[i, :m, :m]) for i, m in enumerate(sizes)]
    out["D0"] = gaussian(rng, 2 * k, 2 * k)
    return out


def _orthonormal_blocks(rng, sizes, k):
    """One (len(sizes), max(sizes), k) Gaussian draw; node i keeps its first
    sizes[i] rows, whose columns are orthonormalised (batched per size)."""
    mm = max(sizes)
    G = rng.standard_normal((len(sizes), mm, k))
    out = [None] * len(sizes)
    for m in sorted(set(sizes)):
        idx = [i for i, x in enumerate(sizes) if x == m]
        q, _ = np.linalg.qr(G[idx, :m, :])
        for j, i in enumerate(idx):
            out[i] = np.ascontiguousarray(q[j])
    return out


def ellipse_points(n: int, a: float = 1.0, b: float = 0.5):
    """n points x_i = (a cos t_i, b sin t_i), t_i = 2 pi i / n (equispaced in
    the parameter).  Returns (x, y) as FP64 arrays."""
    t = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    return a * np.cos(t), b * np.sin(t)


def batch_instances(workload_id: int, count: int, n_lo: int, n_hi: int, ks=(16, 32)):
    """Sizes of independent instances: N log-uniform in [n_lo, n_hi] (rounded),
    k uniform over ``ks``; leaf threshold 2k and s = 3k + 10 per instance."""
    rng = streams(workload_id, 1, extra=(0xBA7C4,))[0]
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        k = int(ks[rng.integers(0, len(ks))])
        out.append(dict(index=i, n=n, k=k, leaf_max=2 * k, s=3 * k + 10))
    return out


def probes(rng: np.random.Generator, n: int, count: int = 8) -> np.ndarray:
    """n x count Gaussian probe block for the apply error."""
    return gaussian(rng, n, count)
