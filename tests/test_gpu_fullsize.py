"""GPU checks at the workloads' full sizes, in the launch configuration the
benchmark times (same inputs, same library calls).

At these sizes the oracle cannot run the whole sweep, so the checks are the
ones that hold at any size, with every expected value computed by the CPU
oracle from the seeded inputs:
  - the sampler on seeded rows against dense oracle rows;
  - the compressed operator on 8 Gaussian probes at 256 seeded rows against
    the oracle's dense rows (log kernel), or on all rows against the oracle's
    Algorithm 1 of the known generator (exact-rank HBS: exact recovery);
  - orthonormality of every basis U_tau, V_tau of every level;
  - in-sample consistency A~ Omega ~ Y.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import inputs  # noqa: E402
from oracle import hbs as ohbs  # noqa: E402
from oracle import logkernel as olog  # noqa: E402
from oracle import tree as otree  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hbs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02990_amd import hbs as h
    h.load()
    return h


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def check_orthonormal(f, tree, k, tol=1e-12):
    for lev in range(1, tree.levels + 1):
        lv = f.level(lev)
        m = lv["m"]
        for key in ("U", "V"):
            B = lv[key]  # (nodes, m, k), zero-padded rows past m_tau
            G = torch.matmul(B.transpose(1, 2).contiguous(), B)
            err = float((G - torch.eye(k, dtype=G.dtype, device=G.device)).abs().max())
            assert err <= tol, (lev, key, err)
        del lv


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["logkernel_ellipse_n65536_k50", "logkernel_ellipse_n262144_k64"])
def test_logkernel_full_size(hbs, name, progress):
    wl = inputs.WORKLOADS[name]
    n, k, leaf, s = wl["n"], wl["k"], wl["leaf_max"], wl["s"]
    progress(f"[fullsize] {name}: N={n} k={k} leaf_max={leaf} s={s}")
    rs = inputs.streams(wl["id"])
    x, y = inputs.ellipse_points(n, wl["a"], wl["b"])
    Om = inputs.gaussian(rs[inputs.STREAM_OMEGA], n, s)
    Ps = inputs.gaussian(rs[inputs.STREAM_PSI], n, s)
    xd, yd, Omd, Psd = dev(x), dev(y), dev(Om), dev(Ps)
    Yd, Zd = hbs.sample_logkernel(xd, yd, Omd, Psd)
    R = np.sort(rs[inputs.STREAM_ROWS].choice(n, 256, replace=False))
    # sampler against dense oracle rows
    assert rel(Yd[torch.from_numpy(R).cuda()].cpu().numpy(), olog.sample(x, y, Om, R)) <= 1e-13
    assert rel(Zd[torch.from_numpy(R).cuda()].cpu().numpy(), olog.sample(x, y, Ps, R)) <= 1e-13
    tree = hbs.Tree(n, leaf)
    f = hbs.Factors.create(tree, k, s)
    f.compress_into(Omd, Yd, Psd, Zd)
    f.check()
    # compressed operator on probes at seeded rows, against dense oracle rows
    G = inputs.probes(rs[inputs.STREAM_PROBES], n, 8)
    TG = f.apply(dev(G)).cpu().numpy()
    AG_R = olog.sample(x, y, G, R)
    err = rel(TG[R], AG_R)
    progress(f"[fullsize] {name}: relative apply error on 256 rows x 8 probes {err:.3e}")
    assert err <= 1e-9
    TtG = f.apply(dev(G), transpose=True).cpu().numpy()
    assert rel(TtG[R], AG_R) <= 1e-9  # A is symmetric
    # in-sample consistency
    assert float(torch.linalg.norm(f.apply(Omd) - Yd) / torch.linalg.norm(Yd)) <= 1e-9
    check_orthonormal(f, tree, k)


@pytest.mark.timeout(600)
def test_logkernel_n262144_precision_paths(hbs, progress):
    """The three precision paths on the N = 2^18 log-kernel workload, against
    dense oracle rows: FP64 samples with the split-precision sweep, and BF16
    samples with the FP64 sweep (bounds 1e-9 and 1e-4; the FP64 path itself
    is checked above)."""
    wl = inputs.WORKLOADS["logkernel_ellipse_n262144_k64"]
    n, k, leaf, s = wl["n"], wl["k"], wl["leaf_max"], wl["s"]
    rs = inputs.streams(wl["id"])
    x, y = inputs.ellipse_points(n, wl["a"], wl["b"])
    Om = inputs.gaussian(rs[inputs.STREAM_OMEGA], n, s)
    Ps = inputs.gaussian(rs[inputs.STREAM_PSI], n, s)
    xd, yd, Omd, Psd = dev(x), dev(y), dev(Om), dev(Ps)
    R = np.sort(rs[inputs.STREAM_ROWS].choice(n, 256, replace=False))
    G = inputs.probes(rs[inputs.STREAM_PROBES], n, 8)
    AG_R = olog.sample(x, y, G, R)
    tree = hbs.Tree(n, leaf)
    Yd, Zd = hbs.sample_logkernel(xd, yd, Omd, Psd)
    f = hbs.compress(tree, k, Omd, Yd, Psd, Zd, precision="split")
    f.check()
    e_split = rel(f.apply(dev(G)).cpu().numpy()[R], AG_R)
    del f
    Yb, Zb = hbs.sample_logkernel(xd, yd, Omd, Psd, precision="bf16")
    Rd = torch.from_numpy(R).cuda()
    e_samp = rel(Yb[Rd].cpu().numpy(), olog.sample(x, y, Om, R))
    f = hbs.compress(tree, k, Omd, Yb, Psd, Zb)
    f.check()
    e_bf16 = rel(f.apply(dev(G)).cpu().numpy()[R], AG_R)
    progress(f"[fullsize] N={n}: split sweep {e_split:.3e}; bf16 sampler rows {e_samp:.3e}, "
             f"bf16 samples + FP64 sweep {e_bf16:.3e}")
    assert e_split <= 1e-9
    assert e_samp <= 1e-4 and e_bf16 <= 1e-4


@pytest.mark.timeout(900)
def test_exact_rank_n4194304_full_size(hbs, progress):
    """Exact recovery of the 16-level exact-rank HBS matrix from samples that
    the oracle's Algorithm 1 draws from the known generator, with the SVD
    truncation of the sketch (whose rounding does not grow from level to
    level): FP64 path to 1e-11 and split path to 1e-10 against the
    generator, on probes and for section 5's 2-norm estimate."""
    wl = inputs.WORKLOADS["hbs_exact_n4194304_k32"]
    n, k, leaf, s = wl["n"], wl["k"], wl["leaf_max"], wl["s"]
    progress(f"[fullsize] exact-rank N={n} k={k} leaf_max={leaf} s={s}: generating")
    levels = otree.cluster_tree(n, leaf)
    rs = inputs.streams(wl["id"])
    gen = inputs.synthetic_generators(rs[inputs.STREAM_GENERATOR], otree.leaf_sizes(levels), k)
    fac = ohbs.from_generators(levels, gen)
    tree = hbs.Tree(n, leaf)
    assert tree.levels == 16
    progress("[fullsize] sampling through the generator (oracle)")
    Om = inputs.gaussian(rs[inputs.STREAM_OMEGA], n, s)
    Omd = dev(Om)
    Yd = dev(ohbs.apply(fac, Om))
    del Om
    Ps = inputs.gaussian(rs[inputs.STREAM_PSI], n, s)
    Psd = dev(Ps)
    Zd = dev(ohbs.apply(fac, Ps, transpose=True))
    del Ps
    G = inputs.probes(rs[inputs.STREAM_PROBES], n, 8)
    AG = ohbs.apply(fac, G)  # the oracle's Algorithm 1 on the generator
    AtG = ohbs.apply(fac, G, transpose=True)
    # the library's Algorithm 1 on the imported generator agrees with the oracle's
    lv = {}
    for l in range(1, tree.levels + 1):
        lv[l] = {"U": dev(np.stack(gen["U"][l])), "V": dev(np.stack(gen["V"][l])),
                 "D": dev(np.stack(gen["D"][l]))}
    A = hbs.import_factors(tree, k, lv, dev(gen["D0"]))
    del lv
    assert rel(A.apply(dev(G)).cpu().numpy(), AG) <= 1e-14
    assert rel(A.apply(dev(G), transpose=True).cpu().numpy(), AtG) <= 1e-14
    v0 = [dev(inputs.gaussian(r, n, 1)[:, 0].copy()) for r in inputs.streams(wl["id"], 2, extra=(0x50,))]
    for path, bound in (("fp64", 1e-11), ("split", 1e-10)):
        progress(f"[fullsize] compressing ({path}, SVD truncation)")
        f = hbs.Factors.create(tree, k, s, path, "svd")
        f.compress_into(Omd, Yd, Psd, Zd)
        f.check()
        err = rel(f.apply(dev(G)).cpu().numpy(), AG)
        errt = rel(f.apply(dev(G), transpose=True).cpu().numpy(), AtG)
        pw = hbs.power_rel_error(f, A, *v0)
        progress(f"[fullsize] exact-rank N={n} {path}: probe error vs the generator {err:.3e} (transpose "
                 f"{errt:.3e}), 2-norm estimate {pw:.3e}")
        assert err <= bound and errt <= bound
        # the 2-norm weighs the top levels' 2k-dimensional subspaces fully,
        # the probes average them over N rows: allow sqrt(N / 2k) = 256 times
        assert pw <= 256 * bound
        if path == "fp64":
            check_orthonormal(f, tree, k)
        del f


@pytest.mark.timeout(600)
def test_exact_rank_depth11_truncated_qr(hbs, progress):
    """The truncated-QR reading of col at the 16-level workload's parameters
    (k = 32, leaf 64, s = 106), N = 131072 (11 levels), where the oracle runs
    the whole sweep.  Under this reading rounding grows about 2.5x per level
    (oracle and GPU each about 2.5e-11 from the generator at depth 11), so GPU
    and oracle agree to that order, not to 1e-12; the bound is twice the
    measured error.  The SVD reading restores 1e-12 at the same depth
    (test_gpu_svd.test_svd_truncation_depth_11)."""
    n, k, leaf, s = 131072, 32, 64, 106
    levels = otree.cluster_tree(n, leaf)
    rs = inputs.streams(5, extra=(n,))
    gen = ohbs.from_generators(levels, inputs.synthetic_generators(rs[0], otree.leaf_sizes(levels), k))
    Om, Ps = inputs.gaussian(rs[1], n, s), inputs.gaussian(rs[2], n, s)
    Y, Z = ohbs.apply(gen, Om), ohbs.apply(gen, Ps, transpose=True)
    progress("[fullsize] depth-11 oracle sweep")
    orc = ohbs.compress(levels, k, Om, Y, Ps, Z)
    tree = hbs.Tree(n, leaf)
    f = hbs.compress(tree, k, dev(Om), dev(Y), dev(Ps), dev(Z))
    f.check()
    G = inputs.probes(rs[3], n, 8)
    AG, OG = ohbs.apply(gen, G), ohbs.apply(orc, G)
    TG = f.apply(dev(G)).cpu().numpy()
    e_orc, e_gpu, e_par = rel(OG, AG), rel(TG, AG), rel(TG, OG)
    progress(f"[fullsize] depth 11: oracle {e_orc:.3e}, GPU {e_gpu:.3e} vs generator; GPU vs oracle {e_par:.3e}")
    assert e_orc <= 5e-11 and e_gpu <= 5e-11
    assert e_par <= 5e-11


@pytest.mark.timeout(900)
def test_logkernel_n65536_against_oracle_sweep(hbs, progress):
    """The 65536-point log-kernel workload at full size against the oracle's
    whole sweep on the oracle's own samples (formed on the CPU, 320 columns
    of the dense kernel), FP64 and split paths, both readings of col.

    These sketches have no gap at k (the kernel's singular values decay
    smoothly), so the truncated basis is not unique to rounding: with the
    pivoted QR, near-equal column norms are ranked differently by the two
    reduction orders; with the SVD, the k-th and (k+1)-th directions are close
    in value.  GPU and oracle then keep different but equally good bases, and
    their operators differ by about the truncation error itself.  What is
    unique is the accuracy: on 256 seeded rows of the dense kernel the GPU's
    error must be within 1.5 times the oracle's, and the two operators may
    differ by at most 2.5 times the oracle's error (the sum of two errors of
    that size)."""
    import threadpoolctl
    wl = inputs.WORKLOADS["logkernel_ellipse_n65536_k50"]
    n, k, leaf, s = wl["n"], wl["k"], wl["leaf_max"], wl["s"]
    x, y = inputs.ellipse_points(n, wl["a"], wl["b"])
    rs = inputs.streams(wl["id"])
    Om = inputs.gaussian(rs[inputs.STREAM_OMEGA], n, s)
    Ps = inputs.gaussian(rs[inputs.STREAM_PSI], n, s)
    progress(f"[fullsize] log kernel N={n}: the oracle's samples (dense rows, CPU)")
    YZ = olog.sample(x, y, np.hstack((Om, Ps)), block=2048)
    Y, Z = np.ascontiguousarray(YZ[:, :s]), np.ascontiguousarray(YZ[:, s:])
    del YZ
    G = inputs.probes(rs[inputs.STREAM_PROBES], n, 8)
    R = np.sort(rs[inputs.STREAM_ROWS].choice(n, 256, replace=False))
    AG_R = olog.sample(x, y, G, R)
    levels = otree.cluster_tree(n, leaf)
    tree = hbs.Tree(n, leaf)
    for trunc in ("qr", "svd"):
        progress(f"[fullsize] oracle sweep, {trunc} reading (one BLAS thread: faster on these small boxes)")
        with threadpoolctl.threadpool_limits(1):
            orc = ohbs.compress(levels, k, Om, Y, Ps, Z, truncation=trunc)
        OG = ohbs.apply(orc, G)
        e_o = rel(OG[R], AG_R)
        for path in ("fp64", "split"):
            f = hbs.compress(tree, k, dev(Om), dev(Y), dev(Ps), dev(Z), precision=path, truncation=trunc)
            f.check()
            TG = f.apply(dev(G)).cpu().numpy()
            e_g, e_p = rel(TG[R], AG_R), rel(TG, OG)
            progress(f"[fullsize] log kernel N={n} {trunc}/{path}: error on 256 kernel rows GPU {e_g:.3e}, "
                     f"oracle {e_o:.3e}; GPU vs oracle {e_p:.3e}")
            assert e_g <= 1.5 * e_o + 1e-13
            assert e_p <= 2.5 * e_o
            del f
