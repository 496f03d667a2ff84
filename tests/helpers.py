"""Shared helpers for the GPU tests: seeded inputs, oracle references, packing.

Only input drawing and the oracle are used to build expected values; nothing
here calls the HIP library except through the binding under test.
"""
from __future__ import annotations

import numpy as np

import inputs
from oracle import hbs as ohbs
from oracle import tree as otree


def synthetic_case(n, k, leaf_max, s, wid=1, extra=()):
    """Exact-rank synthetic HBS problem: generator factors (oracle dict),
    Omega, Psi, and the samples Y, Z computed by the oracle's Algorithm 1."""
    levels = otree.cluster_tree(n, leaf_max)
    rs = inputs.streams(wid, extra=(n, k, leaf_max, s, *extra))
    gen = ohbs.from_generators(levels, inputs.synthetic_generators(rs[0], otree.leaf_sizes(levels), k))
    Om = inputs.gaussian(rs[1], n, s)
    Ps = inputs.gaussian(rs[2], n, s)
    Y = ohbs.apply(gen, Om)
    Z = ohbs.apply(gen, Ps, transpose=True)
    G = inputs.probes(rs[3], n, 8)
    return dict(levels=levels, gen=gen, Om=Om, Ps=Ps, Y=Y, Z=Z, G=G, k=k, s=s, n=n)


def pack_level(blocks, mmax):
    """Pad a list of per-node matrices to (nodes, mmax, cols) with zeros."""
    out = np.zeros((len(blocks), mmax, blocks[0].shape[1]))
    for i, b in enumerate(blocks):
        out[i, :b.shape[0], :b.shape[1]] = b
    return out


def pack_square(blocks, mmax):
    out = np.zeros((len(blocks), mmax, mmax))
    for i, b in enumerate(blocks):
        out[i, :b.shape[0], :b.shape[1]] = b
    return out


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
