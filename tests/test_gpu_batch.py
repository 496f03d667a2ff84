"""GPU parity of batched compression (many independent instances in one sweep)
against the FP64 CPU oracle, instance by instance.

Every instance's inputs are drawn and sampled on the CPU (the oracle's
Algorithm 1 on a seeded exact-rank generator), so every expected value comes
from the oracle.  Instances of different depth and different (k, s) share the
sweep's launches; each must still reproduce what the oracle computes for it
alone.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import inputs  # noqa: E402
from oracle import hbs as ohbs  # noqa: E402
from oracle import tree as otree  # noqa: E402
from tests.helpers import rel, synthetic_case  # noqa: E402

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


# n, k, leaf_max, s: depths 5, 7, 6, 6, 0 (root only), 3; three (k, s) classes
MIXED = [(1024, 16, 32, 58), (3001, 16, 32, 58), (4096, 32, 64, 106), (1000, 12, 24, 46),
         (20, 8, 32, 30), (500, 16, 32, 58)]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("split", 1e-10)])
def test_mixed_batch_matches_oracle(hbs, precision, tol):
    print(f"[batch] mixed batch {MIXED}, {precision}", flush=True)
    cases = [synthetic_case(n, k, leaf, s, extra=(77,)) for n, k, leaf, s in MIXED]
    trees = [hbs.Tree(n, leaf) for n, _, leaf, _ in MIXED]
    ks = [k for _, k, _, _ in MIXED]
    ss = [s for _, _, _, s in MIXED]
    b = hbs.Batch(trees, ks, ss, precision)
    Om = [dev(c["Om"]) for c in cases]
    Ps = [dev(c["Ps"]) for c in cases]
    Y = [dev(c["Y"]) for c in cases]
    Z = [dev(c["Z"]) for c in cases]
    b.compress(Om, Y, Ps, Z)
    fs = [b.factors(i) for i in range(len(MIXED))]
    fs[0].check()
    for i, (c, (n, k, leaf, s)) in enumerate(zip(cases, MIXED)):
        orc = ohbs.compress(c["levels"], k, c["Om"], c["Y"], c["Ps"], c["Z"])
        G = c["G"]
        got = host(fs[i].apply(dev(G)))
        gott = host(fs[i].apply(dev(G), transpose=True))
        e = rel(got, ohbs.apply(orc, G))
        et = rel(gott, ohbs.apply(orc, G, transpose=True))
        print(f"[batch] instance {i} n={n} k={k}: vs oracle {e:.2e} (transpose {et:.2e})", flush=True)
        assert e <= tol and et <= tol, (i, e, et)
        assert rel(got, ohbs.apply(c["gen"], G)) <= tol
    # second sweep of the same batch (graph replay) on new samples: those of 2A
    Y2 = [2.0 * y for y in Y]
    Z2 = [2.0 * z for z in Z]
    b.compress(Om, Y2, Ps, Z2)
    fs[0].check()
    for i, c in enumerate(cases):
        G = c["G"]
        e = rel(host(fs[i].apply(dev(G))), 2.0 * ohbs.apply(c["gen"], G))
        assert e <= tol, (i, e)


def test_compress_batched_single_call(hbs):
    """hbs_compress_batched agrees with a batch built by hand, bit for bit."""
    sel = MIXED[:3]
    cases = [synthetic_case(n, k, leaf, s, extra=(78,)) for n, k, leaf, s in sel]
    trees = [hbs.Tree(n, leaf) for n, _, leaf, _ in sel]
    ks = [k for _, k, _, _ in sel]
    args = [[dev(c[key]) for c in cases] for key in ("Om", "Y", "Ps", "Z")]
    fs = hbs.compress_batched(trees, ks, *args)
    b = hbs.Batch(trees, ks, [s for *_, s in sel]).compress(*args)
    for i, c in enumerate(cases):
        G = dev(c["G"])
        assert torch.equal(fs[i].apply(G), b.factors(i).apply(G))


def test_batch_rejects_bad_arguments(hbs):
    t = hbs.Tree(1024, 32)
    with pytest.raises(hbs.HBSError):
        hbs.Batch([t], [16], [40])  # s - m_leaf < k
    b = hbs.Batch([t], [16], [58])
    with pytest.raises(hbs.HBSError):
        b.factors(1)


@pytest.mark.timeout(900)
def test_batch512_full_size(hbs, progress):
    """The 512-instance workload (N log-uniform in [2048, 32768], k in {16, 32},
    leaf 2k, s = 3k + 10) in one batch: every instance reproduces its
    generator; four sampled instances are compared with the oracle's own sweep."""
    wl = inputs.WORKLOADS["hbs_exact_batch512"]
    spec = inputs.batch_instances(wl["id"], wl["count"], wl["n_lo"], wl["n_hi"], wl["ks"])
    progress(f"[batch512] {len(spec)} instances, total N = {sum(x['n'] for x in spec)}")
    trees, gens, G, Om, Ps, Y, Z = [], [], [], [], [], [], []
    for j, x in enumerate(spec):
        if j % 128 == 0:
            progress(f"[batch512] drawing and sampling instance {j}")
        levels = otree.cluster_tree(x["n"], x["leaf_max"])
        rs = inputs.streams(wl["id"], extra=(x["index"],))
        gen = ohbs.from_generators(levels, inputs.synthetic_generators(rs[inputs.STREAM_GENERATOR],
                                                                      otree.leaf_sizes(levels), x["k"]))
        om = inputs.gaussian(rs[inputs.STREAM_OMEGA], x["n"], x["s"])
        ps = inputs.gaussian(rs[inputs.STREAM_PSI], x["n"], x["s"])
        gens.append((levels, gen, om, ps))
        G.append(inputs.probes(rs[inputs.STREAM_PROBES], x["n"], 8))
        Om.append(dev(om))
        Ps.append(dev(ps))
        Y.append(dev(ohbs.apply(gen, om)))
        Z.append(dev(ohbs.apply(gen, ps, transpose=True)))
        trees.append(hbs.Tree(x["n"], x["leaf_max"]))
    AGs = [ohbs.apply(gens[i][1], G[i]) for i in range(len(spec))]  # each generator on its probes
    progress("[batch512] inputs ready; compressing")
    ks, ss = [x["k"] for x in spec], [x["s"] for x in spec]
    worst = {}
    batches = {}
    modes = [("fp64", "qr"), ("split", "qr"), ("fp64", "svd"), ("split", "svd")]
    for precision, trunc in modes:
        b = hbs.Batch(trees, ks, ss, precision, trunc)
        b.compress(Om, Y, Ps, Z)  # the first sweep also autotunes the tiles
        b.factors(0).check()
        progress(f"[batch512] {precision}/{trunc}: compressed; checking every instance")
        w = 0.0
        for i, x in enumerate(spec):
            e = rel(host(b.factors(i).apply(dev(G[i]))), AGs[i])
            w = max(w, e)
        worst[precision, trunc] = w
        batches[precision, trunc] = b
        progress(f"[batch512] {precision}/{trunc}: worst relative apply error vs generator {w:.3e}")
    # depth <= 10 here.  The truncated-QR reading passes rounding up the tree
    # (about 2.5x per level: 5e-12 at depth 9, 2.5e-11 at 11 with k = 32), the
    # SVD reading does not.
    assert worst["fp64", "qr"] <= 2e-11 and worst["split", "qr"] <= 2e-11
    assert worst["fp64", "svd"] <= 2e-12
    assert worst["split", "svd"] <= 1e-10
    order = sorted(range(len(spec)), key=lambda i: spec[i]["n"])
    rng = inputs.streams(wl["id"], 1, extra=(0x5A3,))[0]
    pick = sorted({order[0], order[-1], *rng.choice(len(spec), 2, replace=False).tolist()})
    for i in pick:
        levels, gen, om, ps = gens[i]
        x = spec[i]
        for trunc in ("qr", "svd"):
            orc = ohbs.compress(levels, x["k"], om, host(Y[i]), ps, host(Z[i]), truncation=trunc)
            OG = ohbs.apply(orc, G[i])
            e = {p: rel(host(batches[p, trunc].factors(i).apply(dev(G[i]))), OG) for p in ("fp64", "split")}
            progress(f"[batch512] instance {i} n={x['n']} k={x['k']} depth {otree.depth(levels)} {trunc}: vs oracle "
                     f"fp64 {e['fp64']:.3e}, split {e['split']:.3e}")
            assert e["fp64"] <= (2e-11 if trunc == "qr" else 1e-12) and e["split"] <= 1e-10
