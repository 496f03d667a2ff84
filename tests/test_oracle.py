"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: the paper's tree
figure, closed forms, invariants (Omega P = 0, orthonormality, Penrose
conditions), special cases with textbook answers (root least squares), brute
force on small dense matrices (exact recovery of an exactly HBS matrix), and a
set of planted mistakes that the pins must catch.
"""
import math
import os

import numpy as np
import pytest

import inputs
from oracle import hbs, linalg, logkernel, metrics, tree


# --------------------------------------------------------------------------
# helpers (inputs only; no arithmetic of the method)
# --------------------------------------------------------------------------

def synthetic_problem(n, k, leaf_max, s, wid=1):
    levels = tree.cluster_tree(n, leaf_max)
    rs = inputs.streams(wid, extra=(n, k, leaf_max, s))
    gen = hbs.from_generators(levels, inputs.synthetic_generators(rs[0], tree.leaf_sizes(levels), k))
    Om = inputs.gaussian(rs[1], n, s)
    Ps = inputs.gaussian(rs[2], n, s)
    return levels, gen, Om, Ps, rs


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# --------------------------------------------------------------------------
# section 3.1: the cluster tree
# --------------------------------------------------------------------------

def test_tree_matches_paper_figure(golden_dir):
    rows = []
    n = leaf = None
    with open(os.path.join(golden_dir, "tree_fig_400.txt")) as f:
        for line in f:
            if line.startswith("# n="):
                kv = dict(p.split("=") for p in line[2:].split())
                n, leaf = int(kv["n"]), int(kv["leaf_max"])
            elif line.strip() and not line.startswith("#"):
                rows.append(tuple(int(x) for x in line.split()))
    levels = tree.cluster_tree(n, leaf)
    got = []
    node = 1
    for lev, nodes in enumerate(levels):
        for a, b in nodes:
            got.append((lev, node, a + 1, b))  # 1-based inclusive as printed
            node += 1
    assert got == rows


@pytest.mark.parametrize("n,leaf", [(1, 4), (7, 4), (100, 7), (1000, 24), (1023, 32), (1025, 32),
                                    (4096, 64), (65536, 100), (3001, 64)])
def test_tree_properties(n, leaf):
    levels = tree.cluster_tree(n, leaf)
    L = tree.depth(levels)
    assert L == (0 if n <= leaf else math.ceil(math.log2(n / leaf)))
    for lev, nodes in enumerate(levels):
        assert len(nodes) == 2 ** lev
        # contiguous partition of [0, n)
        assert nodes[0][0] == 0 and nodes[-1][1] == n
        assert all(nodes[i][1] == nodes[i + 1][0] for i in range(len(nodes) - 1))
        sizes = [b - a for a, b in nodes]
        assert set(sizes) <= {n // 2 ** lev, -(-n // 2 ** lev)}
        if lev > 0:  # children: ceil half first
            for t, (a, b) in enumerate(levels[lev - 1]):
                assert nodes[2 * t] == (a, a + -(-(b - a) // 2))
        if lev < L:
            assert max(sizes) > leaf
    assert max(tree.leaf_sizes(levels)) <= leaf


def test_tree_workload_shapes():
    w = inputs.WORKLOADS
    c1 = tree.cluster_tree(w["hbs_exact_n1024_k16"]["n"], w["hbs_exact_n1024_k16"]["leaf_max"])
    assert tree.depth(c1) == 5 and tree.leaf_sizes(c1) == [32] * 32
    c2 = tree.cluster_tree(65536, 100)
    assert tree.depth(c2) == 10 and set(tree.leaf_sizes(c2)) == {64}
    c3 = tree.cluster_tree(262144, 128)
    assert tree.depth(c3) == 11 and set(tree.leaf_sizes(c3)) == {128}
    c5 = tree.cluster_tree(4194304, 64)
    assert tree.depth(c5) == 16 and len(c5[-1]) == 65536


def test_tree_rejects_empty_nodes():
    with pytest.raises(ValueError):
        tree.cluster_tree(3, 1)


# --------------------------------------------------------------------------
# sections 2.2-2.4 and 4.2: null, col, pseudo-inverse
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,s", [(32, 58), (64, 106), (100, 160), (7, 30)])
def test_null_invariants(m, s):
    rng = np.random.default_rng(m * 1000 + s)
    B = rng.standard_normal((m, s))
    r = s - m
    P = linalg.null(B, r)
    assert P.shape == (s, r)
    assert np.linalg.norm(B @ P) <= 1e-14 * np.linalg.norm(B) * math.sqrt(s)
    assert np.linalg.norm(P.T @ P - np.eye(r)) <= 1e-14 * s
    # whole nullspace: P P^T is the orthogonal projector I - B^+ B (SVD pinv)
    proj = np.eye(s) - np.linalg.pinv(B) @ B
    assert np.linalg.norm(P @ P.T - proj) <= 1e-13
    # a narrower call returns the trailing columns of the same Q
    P5 = linalg.null(B, 5)
    assert np.linalg.norm(B @ P5) <= 1e-13 and P5.shape == (s, 5)


@pytest.mark.parametrize("m,s", [(32, 58), (64, 106), (100, 160), (58, 58)])
def test_pinv_penrose(m, s):
    rng = np.random.default_rng(7 + m + s)
    B = rng.standard_normal((m, s))
    X = linalg.pinv(B)
    assert X.shape == (s, m)
    # Penrose conditions and full row rank: B X = I
    assert np.linalg.norm(B @ X - np.eye(m)) <= 1e-12
    assert np.linalg.norm(X @ B @ X - X) <= 1e-12 * np.linalg.norm(X)
    assert np.linalg.norm((X @ B).T - X @ B) <= 1e-12
    # unique: equals the SVD-based pseudo-inverse
    assert rel(X, np.linalg.pinv(B)) <= 1e-12


@pytest.mark.parametrize("m,r,k", [(32, 26, 16), (100, 60, 50), (64, 42, 32), (16, 8, 8)])
def test_col_rank_k(m, r, k):
    rng = np.random.default_rng(m + r + k)
    B = rng.standard_normal((m, k)) @ rng.standard_normal((k, r))  # rank k
    U = linalg.col(B, k)
    assert U.shape == (m, k)
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= 1e-14 * m
    assert np.linalg.norm(B - U @ (U.T @ B)) <= 1e-13 * np.linalg.norm(B)
    # spans the dominant k-dimensional subspace found by an SVD
    W = np.linalg.svd(B, full_matrices=False)[0][:, :k]
    assert np.linalg.norm(U @ U.T - W @ W.T, 2) <= 1e-12


def test_col_is_rank_revealing():
    """Truncated QR keeps the numerically dominant columns: with one column
    far larger than the rest, it is picked first."""
    rng = np.random.default_rng(3)
    B = rng.standard_normal((20, 10))
    B[:, 7] *= 1e6
    U = linalg.col(B, 1)
    x = B[:, 7] / np.linalg.norm(B[:, 7])
    assert abs(abs(U[:, 0] @ x) - 1.0) <= 1e-12


def _known_svd(rng, m, n, sv):
    """B = U0 diag(sv) W0^* with orthonormal U0 (m x len(sv)), W0 (n x len(sv))
    drawn as inputs; the singular values are given, in any order."""
    p = len(sv)
    U0 = inputs.random_orthonormal(rng, m, p)
    W0 = inputs.random_orthonormal(rng, n, p)
    return U0, W0, (U0 * np.asarray(sv)) @ W0.T


@pytest.mark.parametrize("m,n,k", [(64, 42, 32), (100, 60, 50), (32, 26, 16), (8, 12, 3)])
def test_col_svd_closed_form(m, n, k):
    """col by SVD truncation returns the k leading left singular vectors of a
    matrix built from known singular triples (given out of order), up to sign,
    and the Eckart-Young residuals: ||B - Q Q^* B||_F^2 = sum of the dropped
    sigma_i^2 and ||B - Q Q^* B||_2 = sigma_{k+1}."""
    rng = np.random.default_rng(m * 1000 + n + k)
    p = min(m, n)
    sv = np.geomspace(1.0, 1e-9, p) * (1.0 + 0.5 * rng.random(p))
    sv = np.sort(sv)[::-1]
    perm = rng.permutation(p)
    U0, W0, B = _known_svd(rng, m, n, sv[perm])
    Q = linalg.col_svd(B, k)
    assert Q.shape == (m, k)
    order = np.argsort(perm)  # order[i]: position of the i-th largest in the construction
    for i in range(k):
        u = U0[:, order[i]]
        assert abs(abs(Q[:, i] @ u) - 1.0) <= 1e-9, i
    assert np.linalg.norm(Q.T @ Q - np.eye(k)) <= 1e-14 * m
    R = B - Q @ (Q.T @ B)
    assert np.linalg.norm(R) == pytest.approx(np.sqrt(np.sum(sv[k:] ** 2)), rel=1e-6, abs=1e-15)
    assert np.linalg.norm(R, 2) == pytest.approx(sv[k], rel=1e-6)


def test_col_svd_depends_only_on_the_column_space_structure():
    """Right-multiplying the sketch by any orthogonal matrix (reordering or
    mixing its columns) leaves the SVD truncation unchanged, while the
    pivoted-QR truncation moves with it when B is not of exact rank k."""
    rng = np.random.default_rng(8)
    m, n, k = 64, 42, 32
    sv = np.geomspace(1.0, 1e-3, n)
    _, _, B = _known_svd(rng, m, n, sv)
    M = inputs.random_orthonormal(rng, n, n)
    P1, P2 = linalg.col_svd(B, k), linalg.col_svd(B @ M, k)
    assert np.linalg.norm(P1 @ P1.T - P2 @ P2.T, 2) <= 1e-12
    Q1, Q2 = linalg.col(B, k), linalg.col(B @ M, k)
    assert np.linalg.norm(Q1 @ Q1.T - Q2 @ Q2.T, 2) > 1e-6


def test_col_svd_planted_mistakes_are_caught():
    """Plausible slips in the SVD truncation fail the closed-form pin: the
    trailing instead of the leading singular vectors, the right instead of
    the left ones (a transposed operand), and the first k columns of B
    orthonormalised (truncated QR without pivoting)."""
    rng = np.random.default_rng(21)
    m, k = 16, 5
    sv = np.linspace(3.0, 0.1, m)
    perm = rng.permutation(m)
    U0, W0, B = _known_svd(rng, m, m, sv[perm])
    order = np.argsort(perm)
    want = U0[:, order[:k]]

    def ok(Q):
        return Q.shape == (m, k) and np.linalg.norm(Q @ Q.T - want @ want.T, 2) <= 1e-9

    slips = {
        "trailing vectors": lambda Bm, kk: np.linalg.svd(Bm)[0][:, -kk:],
        "right vectors": lambda Bm, kk: np.linalg.svd(Bm)[2].T[:, :kk],
        "first k columns": lambda Bm, kk: np.linalg.qr(Bm)[0][:, :kk],
    }
    assert ok(linalg.col_svd(B, k))
    for name, fn in slips.items():
        assert not ok(fn(B, k)), name


# --------------------------------------------------------------------------
# section 3.3 and Algorithm 1: telescoping factorization and apply
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,k,leaf", [(256, 8, 16), (1000, 12, 24), (64, 4, 8), (40, 6, 40)])
def test_apply_matches_dense_telescoping(n, k, leaf):
    levels, gen, _, _, rs = synthetic_problem(n, k, leaf, 3 * k + 10)
    A = hbs.dense(gen)
    q = rs[3].standard_normal((n, 3))
    assert rel(hbs.apply(gen, q), A @ q) <= 1e-14
    assert rel(hbs.apply(gen, q, transpose=True), A.T @ q) <= 1e-14
    v = q[:, 0]
    assert rel(hbs.apply(gen, v), A @ v) <= 1e-14


def test_generator_is_hbs_of_rank_k():
    """Section 3.2 condition (1): for every leaf the row block A(I_tau, I_tau^c)
    has rank k with column space U_tau; its column block has row space V_tau."""
    n, k, leaf = 512, 8, 16
    levels, gen, _, _, _ = synthetic_problem(n, k, leaf, 3 * k + 10)
    A = hbs.dense(gen)
    L = tree.depth(levels)
    for t, (a, b) in enumerate(levels[L]):
        rest = np.r_[0:a, b:n]
        sv = np.linalg.svd(A[a:b][:, rest], compute_uv=False)
        assert sv[k] <= 1e-13 * sv[0] and sv[k - 1] > 1e-6 * sv[0]
        U = gen["U"][L][t]
        blk = A[a:b][:, rest]
        assert np.linalg.norm(blk - U @ (U.T @ blk)) <= 1e-13 * np.linalg.norm(blk)
        cb = A[rest][:, a:b]
        V = gen["V"][L][t]
        assert np.linalg.norm(cb - (cb @ V) @ V.T) <= 1e-13 * np.linalg.norm(cb)


# --------------------------------------------------------------------------
# Algorithm 2: compression
# --------------------------------------------------------------------------

@pytest.mark.parametrize("truncation", ["qr", "svd"])
@pytest.mark.parametrize("n,k,leaf,s,tol", [
    (1024, 16, 32, 58, 1e-12),   # the five-level exact-rank workload, full size
    (1000, 12, 24, 46, 1e-12),   # N not a power of two: uneven leaves
    (512, 8, 16, 34, 1e-12),
    (96, 8, 48, 58, 1e-12),      # one level below the root
    (32, 8, 15, 34, 1e-12),      # leaves of exactly k rows
])
def test_exact_recovery_brute_force(n, k, leaf, s, tol, truncation):
    levels, gen, Om, Ps, _ = synthetic_problem(n, k, leaf, s)
    A = hbs.dense(gen)
    Y, Z = A @ Om, A.T @ Ps
    fac = hbs.compress(levels, k, Om, Y, Ps, Z, truncation=truncation)
    assert rel(hbs.dense(fac), A) <= tol


@pytest.mark.parametrize("n,k,leaf,s", [(1024, 16, 32, 58), (1000, 12, 24, 46), (96, 8, 48, 58),
                                        (32, 8, 15, 34), (40, 4, 64, 52)])
def test_floats_per_dof_closed_form(n, k, leaf, s):
    """Storage (quantity (4) of section 5) counted from the tree alone: every
    box tau stores U_tau, V_tau (m_tau x k) and D_tau (m_tau x m_tau), with
    m_tau the leaf size at level L and 2k above; plus the root block D^(0)
    (2k x 2k, or N x N for a single box)."""
    levels, gen, Om, Ps, _ = synthetic_problem(n, k, leaf, s)
    A = hbs.dense(gen)
    fac = hbs.compress(levels, k, Om, A @ Om, Ps, A.T @ Ps)
    L = tree.depth(levels)
    total = 0
    for lev in range(1, L + 1):
        for a, b in levels[lev]:
            m = (b - a) if lev == L else 2 * k
            total += 2 * m * k + m * m
    n0 = n if L == 0 else 2 * k
    total += n0 * n0
    assert hbs.floats_per_dof(fac) == total / n


def test_root_only_is_least_squares():
    """L = 0: D^(0) = Y Omega^dagger recovers any dense A when s >= N."""
    rng = np.random.default_rng(11)
    n, s = 40, 52
    A = rng.standard_normal((n, n))
    Om, Ps = rng.standard_normal((n, s)), rng.standard_normal((n, s))
    levels = tree.cluster_tree(n, 64)
    fac = hbs.compress(levels, 4, Om, A @ Om, Ps, A.T @ Ps)
    assert rel(fac["D0"], A) <= 1e-13
    assert rel(fac["D0"], np.linalg.lstsq(Om.T, (A @ Om).T, rcond=None)[0].T) <= 1e-13


def test_leaf_projectors_and_discrepancy_closed_form():
    n, k, leaf, s = 512, 8, 16, 34
    levels, gen, Om, Ps, _ = synthetic_problem(n, k, leaf, s)
    A = hbs.dense(gen)
    fac = hbs.compress(levels, k, Om, A @ Om, Ps, A.T @ Ps)
    L = tree.depth(levels)
    for t, (a, b) in enumerate(levels[L]):
        U, V, D = fac["U"][L][t], fac["V"][L][t], fac["D"][L][t]
        Ug, Vg = gen["U"][L][t], gen["V"][L][t]
        assert np.linalg.norm(U.T @ U - np.eye(k)) <= 1e-13
        assert np.linalg.norm(U @ U.T - Ug @ Ug.T, 2) <= 1e-12
        assert np.linalg.norm(V @ V.T - Vg @ Vg.T, 2) <= 1e-12
        Att = A[a:b, a:b]  # eq. define_d_tau
        assert rel(D, Att - U @ U.T @ Att @ V @ V.T) <= 1e-12


def test_nothing_lost_and_in_sample():
    """(I - U U^*)(Y_tau - D_tau Omega_tau) = 0 for every box of every level
    (eq. newtestmatrix), and the factors reproduce the samples."""
    n, k, leaf, s = 1024, 16, 32, 58
    levels, gen, Om, Ps, _ = synthetic_problem(n, k, leaf, s)
    Y, Z = hbs.apply(gen, Om), hbs.apply(gen, Ps, transpose=True)
    fac = hbs.compress(levels, k, Om, Y, Ps, Z, keep_samples=True)
    for lev in range(tree.depth(levels), 0, -1):
        for t, (Om_t, Y_t, Ps_t, Z_t) in enumerate(fac["samples"][lev]):
            U, V, D = fac["U"][lev][t], fac["V"][lev][t], fac["D"][lev][t]
            R = Y_t - D @ Om_t
            assert np.linalg.norm(R - U @ (U.T @ R)) <= 1e-12 * np.linalg.norm(Y_t)
            R = Z_t - D.T @ Ps_t
            assert np.linalg.norm(R - V @ (V.T @ R)) <= 1e-12 * np.linalg.norm(Z_t)
    assert rel(hbs.apply(fac, Om), Y) <= 1e-12
    assert rel(hbs.apply(fac, Ps, transpose=True), Z) <= 1e-12


def test_svd_truncation_error_stays_flat_to_depth_9():
    """With the SVD reading of col the exact-rank error at the largest
    workload's shape (k = 32, leaf 64, s = 106) stays near machine precision
    through nine levels (section 5.4: little growth with depth), whereas the
    pivoted-QR reading grows by a factor of about 2.5 per level."""
    errs = {}
    for depth in (5, 7, 9):
        n = 64 * 2 ** depth
        levels, gen, Om, Ps, rs = synthetic_problem(n, 32, 64, 106, wid=5)
        Y, Z = hbs.apply(gen, Om), hbs.apply(gen, Ps, transpose=True)
        G = inputs.probes(rs[3], n)
        ref = hbs.apply(gen, G)
        for tr in ("qr", "svd"):
            fac = hbs.compress(levels, 32, Om, Y, Ps, Z, truncation=tr)
            errs[tr, depth] = metrics.probe_rel_error(ref, hbs.apply(fac, G))
    assert max(errs["svd", d] for d in (5, 7, 9)) <= 4e-13, errs
    assert errs["svd", 9] <= 10 * errs["svd", 5], errs
    assert errs["qr", 9] >= 10 * errs["svd", 9], errs


def test_error_does_not_grow_with_depth():
    """Exact-rank inputs of growing depth at fixed k stay near machine
    precision (minimal error aggregation across levels)."""
    errs = []
    for n in (256, 1024, 4096):
        levels, gen, Om, Ps, rs = synthetic_problem(n, 16, 32, 58)
        Y, Z = hbs.apply(gen, Om), hbs.apply(gen, Ps, transpose=True)
        fac = hbs.compress(levels, 16, Om, Y, Ps, Z)
        G = inputs.probes(rs[3], n)
        errs.append(metrics.probe_rel_error(hbs.apply(gen, G), hbs.apply(fac, G)))
    assert max(errs) <= 1e-12, errs


def test_leaf_sketch_is_gaussian():
    """Remark on why the leaf sketch is Gaussian: Omega(I_tau^c, :) P_tau has
    i.i.d. N(0, 1) entries (loose moment bounds)."""
    rng = np.random.default_rng(5)
    n, m, s = 4096, 32, 58
    Om = rng.standard_normal((n, s))
    P = linalg.null(Om[:m], s - m)
    G = Om[m:] @ P
    assert abs(G.mean()) < 0.01
    assert abs(G.var() - 1.0) < 0.02
    assert abs(np.mean(G ** 4) - 3.0) < 0.1


# --------------------------------------------------------------------------
# planted mistakes: the pins above must catch each of them
# --------------------------------------------------------------------------

def _recovery_error():
    levels, gen, Om, Ps, _ = synthetic_problem(256, 8, 16, 34)
    A = hbs.dense(gen)
    fac = hbs.compress(levels, 8, Om, A @ Om, Ps, A.T @ Ps)
    return rel(hbs.dense(fac), A)


def test_planted_mistakes_are_caught(monkeypatch):
    assert _recovery_error() <= 1e-12
    mistakes = {
        "drop second term of D": lambda U, V, W, X: (np.eye(U.shape[0]) - U @ U.T) @ W,
        "no transpose in second term": lambda U, V, W, X: (np.eye(U.shape[0]) - U @ U.T) @ W
        + U @ U.T @ ((np.eye(U.shape[0]) - V @ V.T) @ X),
        "U in place of V": lambda U, V, W, X: (np.eye(U.shape[0]) - U @ U.T) @ W
        + U @ U.T @ ((np.eye(U.shape[0]) - U @ U.T) @ X).T,
    }
    orig = hbs.discrepancy
    for name, fn in mistakes.items():
        monkeypatch.setattr(hbs, "discrepancy", fn)
        assert _recovery_error() > 1e-6, name
    monkeypatch.setattr(hbs, "discrepancy", orig)

    orig_red = hbs.reduced_samples
    monkeypatch.setattr(hbs, "reduced_samples",
                        lambda U, V, D, Om, Y, Ps, Z: (V.T @ Om, U.T @ (Y - D @ Om), U.T @ Ps,
                                                       V.T @ (Z - D @ Ps)))
    assert _recovery_error() > 1e-6, "D in place of D^* in the Z reduction"
    monkeypatch.setattr(hbs, "reduced_samples",
                        lambda U, V, D, Om, Y, Ps, Z: (U.T @ Om, U.T @ (Y - D @ Om), U.T @ Ps,
                                                       V.T @ (Z - D.T @ Ps)))
    assert _recovery_error() > 1e-6, "U in place of V for the new test matrix"
    monkeypatch.setattr(hbs, "reduced_samples", orig_red)

    orig_null = linalg.null
    monkeypatch.setattr(linalg, "null", lambda B, k: np.linalg.qr(B.T, mode="complete")[0][:, :k])
    assert _recovery_error() > 1e-6, "leading instead of trailing columns of Q"
    monkeypatch.setattr(linalg, "null", orig_null)

    orig_pinv = linalg.pinv
    def wrong_pinv(B):
        Q, R = np.linalg.qr(B.T)
        return Q @ np.linalg.inv(R)  # R^{-1} in place of R^{-T}
    monkeypatch.setattr(linalg, "pinv", wrong_pinv)
    assert _recovery_error() > 1e-6, "pseudo-inverse with R^-1"
    monkeypatch.setattr(linalg, "pinv", orig_pinv)
    assert _recovery_error() <= 1e-12


def test_planted_apply_mistake_is_caught():
    levels, gen, _, _, rs = synthetic_problem(256, 8, 16, 34)
    A = hbs.dense(gen)
    q = rs[3].standard_normal((256, 2))
    assert rel(hbs.apply(gen, q), A @ q) <= 1e-14
    # transposing the factor set must give A^T, not A
    assert rel(hbs.apply(gen, q, transpose=True), A @ q) > 1e-3


# --------------------------------------------------------------------------
# log kernel and section 5 metrics
# --------------------------------------------------------------------------

def test_logkernel_closed_form(golden_dir):
    vals = []
    with open(os.path.join(golden_dir, "logkernel_4pt.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                vals.append([eval(e, {"log": math.log}) for e in line.split("|")])
    x, y = inputs.ellipse_points(4, 1.0, 0.5)
    A = logkernel.rows(x, y, np.arange(4))
    assert np.allclose(A, np.array(vals), rtol=0, atol=1e-15)


def test_logkernel_rows_and_sample():
    n = 300
    x, y = inputs.ellipse_points(n)
    A = logkernel.rows(x, y, np.arange(n))
    assert np.all(np.diag(A) == 0)
    assert np.array_equal(A, A.T) or np.abs(A - A.T).max() <= 1e-15
    i, j = 17, 123
    assert A[i, j] == pytest.approx(math.log(math.hypot(x[i] - x[j], y[i] - y[j])), abs=1e-15)
    G = np.random.default_rng(0).standard_normal((n, 5))
    idx = np.array([0, 5, 299, 150])
    assert rel(logkernel.sample(x, y, G, idx, block=3), A[idx] @ G) <= 1e-15
    assert rel(logkernel.sample(x, y, G, block=64), A @ G) <= 1e-15


def test_probe_rel_error_hand_computed():
    """|| (A_test - A_ref) G ||_F / || A_ref G ||_F on a case worked by hand:
    A_ref G = [[3, 0], [0, 4]] (Frobenius norm 5), A_test G differs by
    [[0, 1], [0, 0]] (norm 1), so the error is 1/5; arrays and callables
    give the same number, and equal inputs give 0."""
    ref = np.array([[3.0, 0.0], [0.0, 4.0]])
    test = np.array([[3.0, 1.0], [0.0, 4.0]])
    assert metrics.probe_rel_error(ref, test) == 0.2
    G = np.eye(2)
    assert metrics.probe_rel_error(lambda g: ref @ g, lambda g: test @ g, G) == 0.2
    assert metrics.probe_rel_error(ref, ref) == 0.0


def test_power_norm_estimate():
    rng = np.random.default_rng(2)
    Q1, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    Q2, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    sv = np.linspace(1.0, 0.1, 60)
    sv[0] = 10.0
    B = Q1 @ np.diag(sv) @ Q2.T
    est = metrics.power_norm(lambda v: B @ v, lambda v: B.T @ v, 60)
    assert est == pytest.approx(np.linalg.norm(B, 2), rel=1e-12)
    # a given start vector takes the same iteration
    v0 = np.random.default_rng(0).standard_normal(60)
    assert metrics.power_norm(lambda v: B @ v, lambda v: B.T @ v, 60, v0=v0) == est
    # the zero operator, and a start vector in the nullspace, give 0
    Z = np.zeros((60, 60))
    assert metrics.power_norm(lambda v: Z @ v, lambda v: Z.T @ v, 60) == 0.0
    P = np.eye(60)
    P[0, 0] = 0.0
    e0 = np.zeros(60)
    e0[0] = 1.0
    assert metrics.power_norm(lambda v: P @ v, lambda v: P @ v, 60, v0=e0) == 0.0


def test_logkernel_compression_accuracy():
    """The ellipse log kernel at k = 50 with the 100-point leaf threshold is
    reproduced far below the 1e-8 level (truncation error: parity unpinned,
    no value printed in the paper)."""
    n, k, leaf, s = 1024, 50, 100, 160
    x, y = inputs.ellipse_points(n)
    levels = tree.cluster_tree(n, leaf)
    rs = inputs.streams(2, extra=(n,))
    Om, Ps = inputs.gaussian(rs[1], n, s), inputs.gaussian(rs[2], n, s)
    A = logkernel.rows(x, y, np.arange(n))
    fac = hbs.compress(levels, k, Om, A @ Om, Ps, A.T @ Ps)
    assert rel(hbs.dense(fac), A) <= 1e-8
