"""Dense primitives of sections 2.2-2.4 and the least-squares step of
section 4.2 (oracle; test infrastructure only).

Every routine is the textbook definition on top of LAPACK: Householder QR
(``scipy.linalg.qr``) and, for the second reading of col, the singular value
decomposition (``scipy.linalg.svd``, driver dgesvd).  The remark closing
section 2.4 explains why no pivoting is needed for null and the
pseudo-inverse: these routines only see random matrices or products with
random matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def col(B: np.ndarray, k: int) -> np.ndarray:
    """col(B, k), section 2.4: k orthonormal columns spanning the column space of
    B (rank <= k), from a truncated QR factorization.

    B may have more than k columns (here B = Y_tau P_tau has s - m_tau).  The
    truncated QR is the rank-revealing one: Householder QR with column
    pivoting (largest remaining column norm first), stopped after k steps; the
    k columns of Q it has produced are returned.  When B has exactly k columns
    this is the plain thin QR up to a column permutation.
    """
    Q, _, _ = sla.qr(B, mode="economic", pivoting=True)
    return Q[:, :k]


def col_svd(B: np.ndarray, k: int) -> np.ndarray:
    """col(B, k), section 2.4, read as truncation of the singular value
    decomposition: the k leading left singular vectors of B, in order of
    decreasing singular value.

    Section 2.3 asks for orthonormal columns Q that make ||B - Q Q^* B||
    small; among all k orthonormal columns the leading left singular vectors
    make it smallest (Eckart-Young), and they depend only on B B^*, not on the
    order or the particular mixture of B's columns.  For B = Y_tau P_tau with
    the whole nullspace P_tau this is the oversampled range finder of section
    2.3 (sample, then truncate), so the basis no longer depends on which k of
    the sketch columns a pivoted QR happens to pick.  Signs of the singular
    vectors are LAPACK's (any sign is equally valid).
    """
    U, _, _ = sla.svd(B, full_matrices=False, lapack_driver="gesvd")
    return U[:, :k]


def null(B: np.ndarray, k: int) -> np.ndarray:
    """null(B, k), section 2.4: the last k columns of the Q factor of the full
    QR factorization of B^*, so that B @ null(B, k) = 0."""
    Q, _ = sla.qr(B.T, mode="full")
    return Q[:, Q.shape[1] - k:]


def pinv(B: np.ndarray) -> np.ndarray:
    """Moore-Penrose pseudo-inverse of an m x s matrix of full row rank m <= s,
    as used in the least-squares step of section 4.2 (eq. d_tau_part_1).

    With the thin QR B^* = Q1 R1 (eq. QR restricted to the first m columns),
    B = R1^* Q1^* and B^dagger = Q1 R1^{-*}.
    """
    m = B.shape[0]
    Q, R = sla.qr(B.T, mode="economic")
    Q1, R1 = Q[:, :m], R[:m, :m]
    # Q1 R1^{-T} = (R1^{-1} Q1^T)^T
    return sla.solve_triangular(R1, Q1.T, lower=False).T
