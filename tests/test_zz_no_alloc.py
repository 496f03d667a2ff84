"""hbs_apply_static (the apply that allocates nothing, its level blocks in a
static device array) through the C ABI, against hbs_apply on the same
factors: identical kernels, so identical bits; two calls in a row, the
second with a smaller input (fewer vectors, then a smaller factor set)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import hbs as ohbs  # noqa: E402
from tests.helpers import synthetic_case  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _static(hbs, f, X, transpose=False):
    lib = hbs.load()
    out = torch.empty_like(X)
    st = lib.hbs_apply_static(f._h, 1 if transpose else 0, ctypes.c_void_p(X.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), X.shape[1], X.stride(0),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == hbs.HBS_OK, st
    return out


def test_apply_static_matches_apply():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02990_amd import hbs
    lib = hbs.load()
    big = synthetic_case(3001, 16, 32, 58)
    small = synthetic_case(1000, 12, 24, 46)
    fb = hbs.compress(hbs.Tree(3001, 32), 16, *[dev(big[x]) for x in ("Om", "Y", "Ps", "Z")])
    fs = hbs.compress(hbs.Tree(1000, 24), 12, *[dev(small[x]) for x in ("Om", "Y", "Ps", "Z")])
    assert lib.hbs_apply_static_max(fb._h) >= 64
    Xb = dev(np.random.default_rng(0).standard_normal((3001, 24)))
    for X, f, case in ((Xb, fb, big), (Xb[:, :5].contiguous(), fb, big),
                       (dev(np.random.default_rng(1).standard_normal((1000, 3))), fs, small)):
        for tr in (False, True):
            got = _static(hbs, f, X, tr)
            ref = f.apply(X, transpose=tr)
            torch.cuda.synchronize()
            assert torch.equal(got, ref)
            want = ohbs.apply(case["gen"], X.cpu().numpy(), transpose=tr)
            assert np.linalg.norm(got.cpu().numpy() - want) <= 1e-12 * np.linalg.norm(want)
    # beyond the static array: refused before anything is enqueued
    too_many = lib.hbs_apply_static_max(fs._h) + 1
    st = lib.hbs_apply_static(fs._h, 0, ctypes.c_void_p(8), ctypes.c_void_p(8), too_many, too_many, None)
    assert st == hbs.HBS_EUNSUPPORTED
