"""The log-kernel stand-in black box (oracle; test infrastructure only).

A(i, j) = log |x_i - x_j| for i != j and A(i, i) = 0, on points x_i of the
plane.  This is the single-layer logarithmic kernel used in section 5.2
without its -1/(2 pi) factor, quadrature weights or diagonal corrections; the
diagonal is simply set to zero.  The matrix is symmetric, so A^* Psi = A Psi.
"""
from __future__ import annotations

import numpy as np


def rows(x, y, idx):
    """Dense rows A(idx, :) as a len(idx) x N FP64 array."""
    idx = np.asarray(idx, dtype=np.int64)
    dx = x[idx][:, None] - x[None, :]
    dy = y[idx][:, None] - y[None, :]
    r = np.hypot(dx, dy)
    out = np.zeros_like(r)
    off = r > 0
    out[off] = np.log(r[off])
    out[np.arange(len(idx)), idx] = 0.0
    return out


def sample(x, y, G, row_idx=None, block=512):
    """A(row_idx, :) @ G (all rows when ``row_idx`` is None), forming the rows
    block by block."""
    n = x.shape[0]
    idx = np.arange(n) if row_idx is None else np.asarray(row_idx, dtype=np.int64)
    out = np.empty((len(idx), G.shape[1]))
    for s in range(0, len(idx), block):
        out[s:s + block] = rows(x, y, idx[s:s + block]) @ G
    return out
