"""The streamed sampling path (hbs_compress_logkernel): the leaf level runs
on the rows the sampler has just written, chunk by chunk, on a second stream.
It must give the results of sampling everything first and compressing after
(hbs_sample_logkernel + hbs_compress_into) bit for bit: the same kernels and
tile choices run on the same values, and the sampler's rows do not depend on
how the rows are grouped into launches.  The unstreamed path is itself held to
the oracle in test_gpu_parity.py; one case here is also compared with the
oracle directly."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import inputs  # noqa: E402
from oracle import hbs as ohbs  # noqa: E402
from oracle import logkernel as olog  # noqa: E402
from oracle import tree as otree  # noqa: E402
from tests.helpers import rel  # noqa: E402

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


def case(n, s, seed):
    x, y = inputs.ellipse_points(n)
    rs = inputs.streams(2, extra=(n, s, seed))
    return x, y, inputs.gaussian(rs[1], n, s), inputs.gaussian(rs[2], n, s)


def same_factors(f1, f2, levels):
    for l in range(1, levels + 1):
        a, b = f1.level(l), f2.level(l)
        for key in ("U", "V", "D"):
            if not torch.equal(a[key], b[key]):
                return f"level {l} {key}"
    if not torch.equal(f1.root(), f2.root()):
        return "root"
    return None


@pytest.mark.parametrize("n,k,leaf,s,chunks,path,truncation,sampler", [
    (8192, 50, 100, 160, 8, "fp64", "qr", "fp64"),
    (3000, 16, 32, 58, 5, "fp64", "svd", "fp64"),
    (3000, 16, 32, 58, 3, "split", "qr", "bf16"),
    (4096, 32, 64, 106, 200, "fp64", "qr", "fp64"),   # more chunks than leaves
])
def test_streamed_matches_sample_then_compress(hbs, progress, n, k, leaf, s, chunks, path, truncation, sampler):
    progress(f"[stream] n={n} k={k} s={s} chunks={chunks} {path}/{truncation} sampler {sampler}")
    x, y, Om, Ps = case(n, s, chunks)
    xd, yd, Omd, Psd = dev(x), dev(y), dev(Om), dev(Ps)
    tree = hbs.Tree(n, leaf)
    # reference: sample everything, then compress
    Y1, Z1 = hbs.sample_logkernel(xd, yd, Omd, Psd, precision=sampler)
    f1 = hbs.Factors.create(tree, k, s, path, truncation)
    f1.compress_into(Omd, Y1, Psd, Z1)
    # streamed: the first call times the tiles (unstreamed), the second streams
    f2 = hbs.Factors.create(tree, k, s, path, truncation)
    Y2, Z2 = torch.empty_like(Omd), torch.empty_like(Psd)
    f2.compress_logkernel(xd, yd, Omd, Psd, Y2, Z2, sampler, chunks)
    Y2.fill_(float("nan"))
    Z2.fill_(float("nan"))
    f2.compress_logkernel(xd, yd, Omd, Psd, Y2, Z2, sampler, chunks)
    torch.cuda.synchronize()
    f1.check()
    f2.check()
    assert torch.equal(Y1, Y2) and torch.equal(Z1, Z2), "samples differ"
    diff = same_factors(f1, f2, tree.levels)
    assert diff is None, f"factors differ at {diff}"


def test_streamed_against_oracle(hbs, progress):
    """The streamed path against the oracle's Algorithm 2 on the oracle's own
    samples: the log kernel on 2048 ellipse points, k = 50, leaves of 64,
    s = 160, 4 chunks; operator on 8 probes within 1e-12 (the FP64 bound of
    the unstreamed parity test)."""
    n, k, leaf, s = 2048, 50, 100, 160
    progress("[stream] against the oracle, n=2048")
    x, y, Om, Ps = case(n, s, 4)
    A = olog.rows(x, y, np.arange(n))
    orc = ohbs.compress(otree.cluster_tree(n, leaf), k, Om, A @ Om, Ps, A @ Ps)
    tree = hbs.Tree(n, leaf)
    f = hbs.Factors.create(tree, k, s)
    xd, yd, Omd, Psd = dev(x), dev(y), dev(Om), dev(Ps)
    Y, Z = torch.empty_like(Omd), torch.empty_like(Psd)
    f.compress_logkernel(xd, yd, Omd, Psd, Y, Z, "fp64", 4)
    f.compress_logkernel(xd, yd, Omd, Psd, Y, Z, "fp64", 4)
    G = inputs.probes(inputs.streams(2, extra=(n, 99))[3], n, 8)
    got = f.apply(dev(G)).cpu().numpy()
    assert rel(got, ohbs.apply(orc, G)) <= 1e-12
