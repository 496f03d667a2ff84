"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
identical seeded inputs.

Tolerances.  Both sides run the same FP64 algorithm; they differ only by
rounding order, and the sweep passes rounding differences up the tree.  On
exact-rank inputs the oracle reproduces A to ~1e-14 (see the oracle pins), so
the GPU factors must reproduce the oracle's operator to 1e-12 (relative
Frobenius error of the applied operator on 8 Gaussian probes).  Leaf
projectors U U^* are unique for exact rank and compared at 1e-12 too.  The
log-kernel sampler is a plain product, compared at 1e-13.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import inputs  # noqa: E402
from oracle import hbs as ohbs  # noqa: E402
from oracle import logkernel as olog  # noqa: E402
from oracle import tree as otree  # noqa: E402
from tests.helpers import pack_level, pack_square, rel, synthetic_case  # noqa: E402

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


def host(t):
    return t.detach().cpu().numpy()


def import_generator(hbs, tree, case):
    gen, k = case["gen"], case["k"]
    L = tree.levels
    levels = {}
    for l in range(1, L + 1):
        mm = max(U.shape[0] for U in gen["U"][l])
        levels[l] = {"U": dev(pack_level(gen["U"][l], mm)), "V": dev(pack_level(gen["V"][l], mm)),
                     "D": dev(pack_square(gen["D"][l], mm))}
    return hbs.import_factors(tree, k, levels, dev(gen["D0"]))


def gpu_compress(hbs, case, leaf_max):
    tree = hbs.Tree(case["n"], leaf_max)
    f = hbs.compress(tree, case["k"], dev(case["Om"]), dev(case["Y"]), dev(case["Ps"]), dev(case["Z"]))
    f.check()
    return tree, f


CASES = [
    # n, k, leaf_max, s
    (1024, 16, 32, 58),   # the five-level exact-rank workload
    (1000, 12, 24, 46),   # N not a power of two, uneven leaves
    (3001, 16, 32, 58),   # uneven, seven levels, ragged last tile
    (4096, 32, 64, 106),  # the k = 32 tile class (leaf 64, s = 106)
    (96, 8, 48, 58),      # one level below the root
    (32, 8, 15, 34),      # leaves of exactly k rows
]


@pytest.mark.parametrize("n,k,leaf,s", CASES)
def test_compress_matches_oracle(hbs, n, k, leaf, s):
    print(f"[parity] compress n={n} k={k} leaf={leaf} s={s}", flush=True)
    case = synthetic_case(n, k, leaf, s)
    orc = ohbs.compress(case["levels"], k, case["Om"], case["Y"], case["Ps"], case["Z"])
    tree, f = gpu_compress(hbs, case, leaf)
    G = case["G"]
    ref = ohbs.apply(orc, G)
    got = host(f.apply(dev(G)))
    assert rel(got, ref) <= 1e-12
    reft = ohbs.apply(orc, G, transpose=True)
    gott = host(f.apply(dev(G), transpose=True))
    assert rel(gott, reft) <= 1e-12
    # exact recovery of the generator
    assert rel(got, ohbs.apply(case["gen"], G)) <= 1e-12
    # leaf projectors and leaf D (unique for exact rank)
    L = tree.levels
    lv = f.level(L)
    U, V, D = host(lv["U"]), host(lv["V"]), host(lv["D"])
    for t, (a, b) in enumerate(case["levels"][L]):
        m = b - a
        Uo, Vo, Do = orc["U"][L][t], orc["V"][L][t], orc["D"][L][t]
        Ug, Vg = U[t, :m], V[t, :m]
        assert np.linalg.norm(Ug.T @ Ug - np.eye(k)) <= 1e-13
        assert np.linalg.norm(Ug @ Ug.T - Uo @ Uo.T, 2) <= 1e-12
        assert np.linalg.norm(Vg @ Vg.T - Vo @ Vo.T, 2) <= 1e-12
        # D_tau vanishes when m_tau = k (square bases): compare on the scale
        # of the diagonal block it is carved from
        scale = max(np.linalg.norm(Do), np.linalg.norm(case["gen"]["D"][L][t]))
        assert np.linalg.norm(D[t, :m, :m] - Do) <= 1e-12 * scale
        assert np.all(U[t, m:] == 0) and np.all(D[t, m:] == 0) and np.all(D[t, :, m:] == 0)


@pytest.mark.parametrize("n,k,leaf,s", CASES)
def test_split_precision_matches_oracle(hbs, n, k, leaf, s):
    """Split-precision bulk products (7-bit integer slices on the int8 matrix
    cores): the FP64 oracle's operator to 1e-10, bases still orthonormal."""
    print(f"[parity] split compress n={n} k={k} leaf={leaf} s={s}", flush=True)
    case = synthetic_case(n, k, leaf, s)
    orc = ohbs.compress(case["levels"], k, case["Om"], case["Y"], case["Ps"], case["Z"])
    tree = hbs.Tree(n, leaf)
    f = hbs.compress(tree, k, dev(case["Om"]), dev(case["Y"]), dev(case["Ps"]), dev(case["Z"]), precision="split")
    f.check()
    G = case["G"]
    e = rel(host(f.apply(dev(G))), ohbs.apply(orc, G))
    et = rel(host(f.apply(dev(G), transpose=True)), ohbs.apply(orc, G, transpose=True))
    print(f"[parity] split vs oracle {e:.2e} (transpose {et:.2e})", flush=True)
    assert e <= 1e-10 and et <= 1e-10
    assert rel(host(f.apply(dev(G))), ohbs.apply(case["gen"], G)) <= 1e-10
    for lev in range(1, tree.levels + 1):
        U = f.level(lev)["U"]
        Gm = torch.matmul(U.transpose(1, 2).contiguous(), U)
        assert float((Gm - torch.eye(k, dtype=Gm.dtype, device=Gm.device)).abs().max()) <= 1e-13


def test_root_only_least_squares(hbs):
    """L = 0: the whole matrix is the root block D^(0) = Y Omega^dagger."""
    rng = np.random.default_rng(11)
    n, s = 40, 52
    A = rng.standard_normal((n, n))
    Om, Ps = rng.standard_normal((n, s)), rng.standard_normal((n, s))
    tree = hbs.Tree(n, 64)
    assert tree.levels == 0
    f = hbs.compress(tree, 4, dev(Om), dev(A @ Om), dev(Ps), dev(A.T @ Ps))
    f.check()
    assert rel(host(f.root()), A) <= 1e-12
    assert rel(host(f.apply(dev(np.eye(n)))), A) <= 1e-12


@pytest.mark.parametrize("n,k,leaf", [(1024, 16, 32), (1000, 12, 24), (40, 6, 40)])
@pytest.mark.parametrize("nvec", [1, 7])
def test_apply_matches_oracle(hbs, n, k, leaf, nvec):
    case = synthetic_case(n, k, leaf, 3 * k + 10)
    tree = hbs.Tree(n, leaf)
    f = import_generator(hbs, tree, case)
    q = case["G"][:, :nvec]
    for tr in (False, True):
        got = host(f.apply(dev(q), transpose=tr))
        assert rel(got, ohbs.apply(case["gen"], q, transpose=tr)) <= 1e-14


def test_apply_vector_input(hbs):
    case = synthetic_case(256, 8, 16, 34)
    tree = hbs.Tree(256, 16)
    f = import_generator(hbs, tree, case)
    v = case["G"][:, 0]
    got = host(f.apply(dev(v)))
    assert got.shape == (256,)
    assert rel(got, ohbs.apply(case["gen"], v)) <= 1e-14


@pytest.mark.parametrize("n,s", [(1000, 58), (257, 160), (2048, 202), (64, 1)])
def test_logkernel_sampler_matches_dense_rows(hbs, n, s):
    print(f"[parity] logkernel n={n} s={s}", flush=True)
    x, y = inputs.ellipse_points(n)
    rs = inputs.streams(2, extra=(n, s))
    Om, Ps = inputs.gaussian(rs[1], n, s), inputs.gaussian(rs[2], n, s)
    Yg, Zg = hbs.sample_logkernel(dev(x), dev(y), dev(Om), dev(Ps))
    Yr = olog.sample(x, y, Om)
    Zr = olog.sample(x, y, Ps)
    assert rel(host(Yg), Yr) <= 1e-13
    assert rel(host(Zg), Zr) <= 1e-13


@pytest.mark.parametrize("n,s", [(1000, 58), (257, 160), (2048, 202), (64, 1)])
def test_logkernel_sampler_bf16(hbs, n, s):
    """BF16 hi/lo operand pairs with FP32 accumulation: about 1e-5 relative,
    bound 1e-4; worse than FP64 by construction."""
    x, y = inputs.ellipse_points(n)
    rs = inputs.streams(2, extra=(n, s, 16))
    Om, Ps = inputs.gaussian(rs[1], n, s), inputs.gaussian(rs[2], n, s)
    Yg, Zg = hbs.sample_logkernel(dev(x), dev(y), dev(Om), dev(Ps), precision="bf16")
    ey, ez = rel(host(Yg), olog.sample(x, y, Om)), rel(host(Zg), olog.sample(x, y, Ps))
    print(f"[parity] bf16 sampler n={n} s={s}: {ey:.2e} {ez:.2e}", flush=True)
    assert ey <= 1e-4 and ez <= 1e-4


def test_logkernel_compress_matches_oracle(hbs):
    """General (not exactly HBS) input: the log kernel, k = 50, leaf threshold
    100 (leaves of 64), s = 160, on 2048 ellipse points; samples from the oracle."""
    n, k, leaf, s = 2048, 50, 100, 160
    x, y = inputs.ellipse_points(n)
    rs = inputs.streams(2, extra=(n,))
    Om, Ps = inputs.gaussian(rs[1], n, s), inputs.gaussian(rs[2], n, s)
    A = olog.rows(x, y, np.arange(n))
    Y, Z = A @ Om, A @ Ps
    levels = otree.cluster_tree(n, leaf)
    orc = ohbs.compress(levels, k, Om, Y, Ps, Z)
    tree = hbs.Tree(n, leaf)
    f = hbs.compress(tree, k, dev(Om), dev(Y), dev(Ps), dev(Z))
    f.check()
    G = inputs.probes(rs[3], n)
    ref = ohbs.apply(orc, G)
    got = host(f.apply(dev(G)))
    err_orc = rel(ref, A @ G)
    # both sides approximate A to err_orc; they agree far below it
    assert rel(got, ref) <= max(1e-12, 0.1 * err_orc)
    assert rel(got, A @ G) <= 2 * err_orc + 1e-13


def test_logkernel_compress_split_matches_oracle(hbs):
    """The same log-kernel problem on the split-precision path."""
    n, k, leaf, s = 2048, 50, 100, 160
    x, y = inputs.ellipse_points(n)
    rs = inputs.streams(2, extra=(n,))
    Om, Ps = inputs.gaussian(rs[1], n, s), inputs.gaussian(rs[2], n, s)
    A = olog.rows(x, y, np.arange(n))
    Y, Z = A @ Om, A @ Ps
    orc = ohbs.compress(otree.cluster_tree(n, leaf), k, Om, Y, Ps, Z)
    tree = hbs.Tree(n, leaf)
    f = hbs.compress(tree, k, dev(Om), dev(Y), dev(Ps), dev(Z), precision="split")
    f.check()
    G = inputs.probes(rs[3], n)
    ref = ohbs.apply(orc, G)
    got = host(f.apply(dev(G)))
    err_orc = rel(ref, A @ G)
    print(f"[parity] log kernel split: vs oracle {rel(got, ref):.2e}, oracle vs A {err_orc:.2e}", flush=True)
    assert rel(got, ref) <= max(1e-10, 0.1 * err_orc)
    assert rel(got, A @ G) <= 2 * err_orc + 1e-10


def test_numeric_flag_on_nonfinite_input(hbs):
    case = synthetic_case(256, 8, 16, 34)
    Y = case["Y"].copy()
    Y[5, 3] = np.nan
    tree = hbs.Tree(256, 16)
    f = hbs.compress(tree, 8, dev(case["Om"]), dev(Y), dev(case["Ps"]), dev(case["Z"]))
    with pytest.raises(hbs.HBSError) as e:
        f.check()
    assert e.value.status == hbs.HBS_ENUMERIC
    f.check()  # the flag is cleared by the check


def test_numeric_flag_on_rank_deficient_test_matrix(hbs):
    case = synthetic_case(256, 8, 16, 34)
    Om = case["Om"].copy()
    Om[1] = Om[0]  # two equal rows: Omega_tau loses rank
    tree = hbs.Tree(256, 16)
    f = hbs.compress(tree, 8, dev(Om), dev(case["Y"]), dev(case["Ps"]), dev(case["Z"]))
    with pytest.raises(hbs.HBSError) as e:
        f.check()
    assert e.value.status == hbs.HBS_ENUMERIC


def test_compress_is_deterministic(hbs):
    case = synthetic_case(1024, 16, 32, 58)
    tree = hbs.Tree(1024, 32)
    f = hbs.Factors.create(tree, 16, 58)
    args = [dev(case[x]) for x in ("Om", "Y", "Ps", "Z")]
    f.compress_into(*args)
    a = [host(v) for v in f.level(tree.levels).values() if hasattr(v, "cpu")] + [host(f.root())]
    f.compress_into(*args)
    b = [host(v) for v in f.level(tree.levels).values() if hasattr(v, "cpu")] + [host(f.root())]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_compress_into_reuses_factor_set_with_ld(hbs):
    """Inputs with a leading dimension larger than s (views of wider buffers)."""
    n, k, leaf, s = 1024, 16, 32, 58
    case = synthetic_case(n, k, leaf, s)
    wide = {x: np.zeros((n, s + 6)) for x in ("Om", "Y", "Ps", "Z")}
    for x in wide:
        wide[x][:, :s] = case[x]
    tree = hbs.Tree(n, leaf)
    f = hbs.Factors.create(tree, k, s)
    views = [dev(wide[x])[:, :s] for x in ("Om", "Y", "Ps", "Z")]
    f.compress_into(*views)
    f.check()
    G = case["G"]
    assert rel(host(f.apply(dev(G))), ohbs.apply(case["gen"], G)) <= 1e-12


@pytest.mark.parametrize("n,k,leaf,s", [(3001, 16, 32, 58), (4096, 32, 64, 106)])
def test_autotuned_and_heuristic_tiles_agree(hbs, n, k, leaf, s, monkeypatch):
    """The tile autotuner (first compression) and the built-in heuristic
    (HBS_AUTOTUNE=0) both reproduce the oracle; the plan reports the choice."""
    case = synthetic_case(n, k, leaf, s, extra=(91,))
    orc = ohbs.compress(case["levels"], k, case["Om"], case["Y"], case["Ps"], case["Z"])
    G = case["G"]
    ref = ohbs.apply(orc, G)
    args = [dev(case[x]) for x in ("Om", "Y", "Ps", "Z")]
    tree = hbs.Tree(n, leaf)
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("HBS_AUTOTUNE", mode)
        f = hbs.Factors.create(tree, k, s)
        assert not any(p["tuned"] for p in f.plan())
        f.compress_into(*args)
        f.check()
        plan = f.plan()
        assert len(plan) == tree.levels + 1 and plan[-1]["root"]
        assert all(p["tuned"] for p in plan) == (mode == "1")
        for p in plan:
            lq = p["lq"]
            assert lq["threads"] // lq["lanes_per_row"] * lq["test_slots"] >= p["mmax"]
            assert lq["lanes_per_row"] * lq["col_slots"] >= p["s"]
        out[mode] = host(f.apply(dev(G)))
        e = rel(out[mode], ref)
        print(f"[parity] autotune={mode} n={n}: vs oracle {e:.2e}; plan "
              f"{[(p['lq']['threads'], p['lq']['chunks'], p['tail_b']) for p in plan]}", flush=True)
        assert e <= 1e-12
    assert rel(out["1"], out["0"]) <= 1e-12


def test_back_to_back_calls_without_host_sync(hbs):
    """Two compressions of different inputs into one factor set, each followed
    by an apply, enqueued with no host synchronisation between them while the
    stream is still busy with earlier work: every result matches its own
    oracle (the inputs are captured per call, never rewritten under a queued
    upload).  Then a compression on one stream and an apply on another: the
    library orders them."""
    n, k, leaf, s = 3001, 16, 32, 58
    ca = synthetic_case(n, k, leaf, s, extra=(1,))
    cb = synthetic_case(n, k, leaf, s, extra=(2,))
    oa = ohbs.compress(ca["levels"], k, ca["Om"], ca["Y"], ca["Ps"], ca["Z"])
    ob = ohbs.compress(cb["levels"], k, cb["Om"], cb["Y"], cb["Ps"], cb["Z"])
    G = ca["G"]
    tree = hbs.Tree(n, leaf)
    f = hbs.Factors.create(tree, k, s)
    ia = [dev(ca[x]) for x in ("Om", "Y", "Ps", "Z")]
    ib = [dev(cb[x]) for x in ("Om", "Y", "Ps", "Z")]
    Gd = dev(G)
    f.compress_into(*ia)  # first call: tiles tuned, graph captured
    torch.cuda.synchronize()
    big = torch.randn(4096, 4096, dtype=torch.float64, device="cuda")
    for rep in range(3):
        busy = big @ big  # keeps the stream busy while the host runs ahead
        f.compress_into(*ia)
        out_a = f.apply(Gd)
        f.compress_into(*ib)
        out_b = f.apply(Gd)
        del busy
        torch.cuda.synchronize()
        ea = rel(host(out_a), ohbs.apply(oa, G))
        eb = rel(host(out_b), ohbs.apply(ob, G))
        assert ea <= 1e-12 and eb <= 1e-12, (rep, ea, eb)
    # compress on a side stream, apply on the current one, no sync between
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        busy = big @ big
        f.compress_into(*ia)
    out = f.apply(Gd)
    torch.cuda.synchronize()
    assert rel(host(out), ohbs.apply(oa, G)) <= 1e-12
    f.check()
