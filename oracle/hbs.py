"""Compression (Algorithm 2), apply (Algorithm 1) and the telescoping
factorization (section 3.3) of HBS matrices, in FP64, one box at a time
(oracle; test infrastructure only).

Notation follows the paper.  Matrices are real, so A^* is the transpose.
``k`` is the width of every basis U_tau, V_tau (m_tau x k).  The sketch of a
box uses the whole nullspace of its test matrix: P_tau = null(Omega_tau, r)
with r = s - m_tau, which is the paper's own setting s = r + m (section 4.2,
remark on conditioning); the rank-k basis is then U_tau = col(Y_tau P_tau, k)
of the r-column sketch (section 2.4), read in one of two ways:

  truncation="qr"   the paper's truncated QR: Householder QR with column
                    pivoting stopped after k steps (linalg.col);
  truncation="svd"  the k leading left singular vectors of the sketch
                    (linalg.col_svd), the truncation step of the oversampled
                    range finder of section 2.3.

Factor container (a plain dict):
  levels  cluster tree, ``levels[l]`` = list of (start, stop) ranges
  k       basis width
  U, V, D dicts keyed by level l = 1..L, each a list over the nodes of level l,
          left to right: U_tau, V_tau (m_tau x k) and D_tau (m_tau x m_tau)
  D0      the root block D^(0)
"""
from __future__ import annotations

import numpy as np

from . import linalg
from .tree import depth


# ---------------------------------------------------------------------------
# Algorithm 2
# ---------------------------------------------------------------------------

def discrepancy(U, V, W, X):
    """eq. d_tau_formula (section 4.2):
        D_tau = (I - U U^*) Y_tau Omega_tau^dagger
              + U U^* ((I - V V^*) Z_tau Psi_tau^dagger)^*
    with W = Y_tau Omega_tau^dagger and X = Z_tau Psi_tau^dagger."""
    m = U.shape[0]
    I = np.eye(m)
    return (I - U @ U.T) @ W + U @ U.T @ ((I - V @ V.T) @ X).T


def truncate(B, k, truncation):
    """col(B, k) under the chosen reading (module docstring)."""
    if truncation == "qr":
        return linalg.col(B, k)
    if truncation == "svd":
        return linalg.col_svd(B, k)
    raise ValueError(f"unknown truncation {truncation!r}")


def box_factors(Om, Y, Ps, Z, k, truncation="qr"):
    """The block of Algorithm 2 for one node tau on a level l > 0:
    P = null(Omega_tau, r), Q = null(Psi_tau, r) with r = s - m_tau
    (sections 2.4, 4.1), U = col(Y_tau P, k), V = col(Z_tau Q, k)
    (eqs. u_tau_formula, v_tau_formula), D from eq. d_tau_formula."""
    m, s = Om.shape
    P = linalg.null(Om, s - m)
    Q = linalg.null(Ps, s - m)
    U = truncate(Y @ P, k, truncation)
    V = truncate(Z @ Q, k, truncation)
    W = Y @ linalg.pinv(Om)
    X = Z @ linalg.pinv(Ps)
    D = discrepancy(U, V, W, X)
    return U, V, D


def reduced_samples(U, V, D, Om, Y, Ps, Z):
    """One child's contribution to its parent's test and sample matrices
    (eq. newtestmatrix and eq. omega_tau_and_y_tau, section 4.3; the Psi and Z
    rows as written out in Algorithm 2):
        V^* Omega,   U^* (Y - D Omega),   U^* Psi,   V^* (Z - D^* Psi),
    returned in the order (Omega, Y, Psi, Z) used for every box."""
    return V.T @ Om, U.T @ (Y - D @ Om), U.T @ Ps, V.T @ (Z - D.T @ Ps)


def compress(levels, k, Omega, Y, Psi, Z, keep_samples=False, truncation="qr"):
    """Algorithm 2: compress level by level from the leaves (level L) to the
    root, given the test matrices Omega, Psi (N x s) and the samples
    Y = A Omega, Z = A^* Psi.

    Returns the factor dict (module docstring).  With ``keep_samples`` the dict
    also holds ``samples[l]`` = list of (Omega_tau, Y_tau, Psi_tau, Z_tau) used
    on level l.  ``truncation`` selects the reading of col ("qr" or "svd",
    module docstring).
    """
    L = depth(levels)
    fac = {"levels": levels, "k": int(k), "U": {}, "V": {}, "D": {}, "D0": None}
    if keep_samples:
        fac["samples"] = {}
    # leaf blocks: Omega(I_tau, :) etc.
    cur = [(Omega[a:b], Y[a:b], Psi[a:b], Z[a:b]) for a, b in levels[L]]
    for lev in range(L, 0, -1):
        if keep_samples:
            fac["samples"][lev] = cur
        Us, Vs, Ds, red = [], [], [], []
        for Om_t, Y_t, Ps_t, Z_t in cur:
            U, V, D = box_factors(Om_t, Y_t, Ps_t, Z_t, k, truncation)
            Us.append(U)
            Vs.append(V)
            Ds.append(D)
            red.append(reduced_samples(U, V, D, Om_t, Y_t, Ps_t, Z_t))
        fac["U"][lev], fac["V"][lev], fac["D"][lev] = Us, Vs, Ds
        # parent of children (2t, 2t+1) stacks their reduced blocks
        cur = [tuple(np.vstack((red[2 * t][i], red[2 * t + 1][i])) for i in range(4))
               for t in range(len(red) // 2)]
    Om0, Y0, _, _ = cur[0]
    if keep_samples:
        fac["samples"][0] = cur
    # root: Y_tau = D^(0) Omega_tau, so D^(0) = Y_tau Omega_tau^dagger
    fac["D0"] = Y0 @ linalg.pinv(Om0)
    return fac


# ---------------------------------------------------------------------------
# Algorithm 1 and the telescoping factorization
# ---------------------------------------------------------------------------

def _transposed(fac):
    """Factors of A^*: swap U and V and transpose every D (section 3.3)."""
    L = depth(fac["levels"])
    return {"levels": fac["levels"], "k": fac["k"],
            "U": {l: fac["V"][l] for l in range(1, L + 1)},
            "V": {l: fac["U"][l] for l in range(1, L + 1)},
            "D": {l: [D.T for D in fac["D"][l]] for l in range(1, L + 1)},
            "D0": fac["D0"].T}


def apply(fac, q, transpose=False):
    """Algorithm 1: u = A q (or A^* q) from the telescoping factors.

    The printed listing has three slips, read as follows: the upward loop runs
    over the nodes of level l (not level L), the downward pass loops over the
    nodes of each level, and the root block is D^(0).
    """
    if transpose:
        fac = _transposed(fac)
    q = np.asarray(q, dtype=np.float64)
    vec = q.ndim == 1
    if vec:
        q = q[:, None]
    levels = fac["levels"]
    L = depth(levels)
    if L == 0:
        u = fac["D0"] @ q
        return u[:, 0] if vec else u
    k = fac["k"]
    # upward pass
    qhat = {L: [fac["V"][L][t].T @ q[a:b] for t, (a, b) in enumerate(levels[L])]}
    for lev in range(L - 1, 0, -1):
        qhat[lev] = [fac["V"][lev][t].T @ np.vstack((qhat[lev + 1][2 * t], qhat[lev + 1][2 * t + 1]))
                     for t in range(2 ** lev)]
    # downward pass
    r = fac["D0"] @ np.vstack((qhat[1][0], qhat[1][1]))
    uhat = {1: [r[:k], r[k:]]}
    for lev in range(1, L):
        nxt = []
        for t in range(2 ** lev):
            r = fac["U"][lev][t] @ uhat[lev][t] + fac["D"][lev][t] @ np.vstack(
                (qhat[lev + 1][2 * t], qhat[lev + 1][2 * t + 1]))
            nxt += [r[:k], r[k:]]
        uhat[lev + 1] = nxt
    u = np.empty_like(q)
    for t, (a, b) in enumerate(levels[L]):
        u[a:b] = fac["U"][L][t] @ uhat[L][t] + fac["D"][L][t] @ q[a:b]
    return u[:, 0] if vec else u


def _block_diag(blocks):
    rows = sum(b.shape[0] for b in blocks)
    cols = sum(b.shape[1] for b in blocks)
    out = np.zeros((rows, cols))
    r = c = 0
    for b in blocks:
        out[r:r + b.shape[0], c:c + b.shape[1]] = b
        r += b.shape[0]
        c += b.shape[1]
    return out


def dense(fac):
    """The N x N matrix of a telescoping factorization (eqs. telescoping_leaf,
    telescoping_parent): start from D^(0) = A~^(1) and build
    A~^(l+1) = U^(l) A~^(l) (V^(l))^* + D^(l) down to A = A~^(L+1), with the
    block-diagonal U^(l), V^(l), D^(l) of section 3.3 formed explicitly."""
    L = depth(fac["levels"])
    At = np.array(fac["D0"], dtype=np.float64)
    for lev in range(1, L + 1):
        Ul = _block_diag(fac["U"][lev])
        Vl = _block_diag(fac["V"][lev])
        Dl = _block_diag(fac["D"][lev])
        At = Ul @ At @ Vl.T + Dl
    return At


def from_generators(levels, gen):
    """Wrap generator factors (``inputs.synthetic_generators``) as a factor dict."""
    L = depth(levels)
    fac = {"levels": levels, "k": gen["k"], "U": {}, "V": {}, "D": {}, "D0": gen["D0"]}
    for lev in range(1, L + 1):
        fac["U"][lev] = gen["U"][lev]
        fac["V"][lev] = gen["V"][lev]
        fac["D"][lev] = gen["D"][lev]
    return fac


def floats_per_dof(fac):
    """Storage of the factors in floating-point values per degree of freedom
    (quantity (4) of section 5)."""
    L = depth(fac["levels"])
    n = fac["levels"][0][0][1]
    total = fac["D0"].size
    for lev in range(1, L + 1):
        total += sum(x.size for x in fac["U"][lev]) + sum(x.size for x in fac["V"][lev])
        total += sum(x.size for x in fac["D"][lev])
    return total / n
