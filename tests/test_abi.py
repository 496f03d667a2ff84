"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/hbs.h, builds the same cluster tree as
section 3.1 describes (compared with the oracle's tree), and rejects invalid
arguments synchronously before touching the device."""
import ctypes
import os
import re

import pytest

from oracle import tree as otree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hbs.h")


def _lib():
    from paper_2205_02990_amd import hbs
    if not os.path.exists(hbs.LIB_PATH):
        pytest.skip("libhbs.so not built (run python -m paper_2205_02990_amd.build)")
    return hbs


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"typedef[^;]*;", "", text)  # function-pointer types are not symbols
    return sorted(set(re.findall(r"\b(hbs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hbs_compress", "hbs_compress_into", "hbs_apply", "hbs_factors_import", "hbs_check",
                     "hbs_tree_create", "hbs_sample_logkernel", "hbs_level", "hbs_root"):
        assert required in names


def test_library_exports_every_declared_symbol():
    hbs = _lib()
    lib = ctypes.CDLL(hbs.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("n,leaf", [(1, 4), (400, 100), (1000, 24), (1023, 32), (65536, 100), (3001, 64),
                                    (4194304, 64), (262144, 128)])
def test_library_tree_matches_section_3_1(n, leaf):
    hbs = _lib()
    t = hbs.Tree(n, leaf)
    ref = otree.cluster_tree(n, leaf)
    assert t.levels == otree.depth(ref)
    for lev in range(min(t.levels, 12) + 1):
        assert t.ranges(lev) == ref[lev]
    if t.levels > 12:
        # deep trees: compare the leaf level only at a few nodes
        for i in (0, 1, 2 ** t.levels // 2, 2 ** t.levels - 1):
            a, m = t.node(t.levels, i)
            assert (a, a + m) == ref[t.levels][i]


def test_tree_rejects_bad_arguments():
    hbs = _lib()
    for n, leaf in [(0, 4), (10, 0), (3, 1)]:
        with pytest.raises(hbs.HBSError) as e:
            hbs.Tree(n, leaf)
        assert e.value.status == hbs.HBS_EINVAL


@pytest.mark.parametrize("precision", ["fp64", "split"])
@pytest.mark.parametrize("truncation", ["qr", "svd"])
@pytest.mark.parametrize("n,leaf,k,s,status", [
    (1024, 32, 16, 47, "EINVAL"),   # s - m < k at the leaves
    (1024, 32, 16, 32 + 16 - 1, "EINVAL"),
    (1024, 32, 33, 200, "EINVAL"),  # leaves smaller than k
    (1024, 32, 0, 58, "EINVAL"),
    (1024, 32, 16, 0, "EINVAL"),
    (1024, 32, 16, 3 * 16 - 1, "EINVAL"),  # inner boxes of 2k rows need s >= 3k
    (1024, 64, 16, 63, "EINVAL"),   # s < 2k + ... : leaves of 64 rows leave no k-column sketch
    (40, 64, 4, 39, "EINVAL"),      # root-only: s must be >= N
    (1024, 512, 16, 600, "EUNSUPPORTED"),  # leaves of 512 rows: no compiled tile class
])
def test_factor_creation_validates_before_device_work(n, leaf, k, s, status, truncation, precision):
    hbs = _lib()
    t = hbs.Tree(n, leaf)
    with pytest.raises(hbs.HBSError) as e:
        hbs.Factors.create(t, k, s, precision, truncation)
    assert e.value.status == getattr(hbs, "HBS_" + status)


@pytest.mark.parametrize("truncation", ["qr", "svd"])
def test_split_precision_rejects_boxes_over_128_rows(truncation):
    """The split-precision products contract over at most 128 box rows (as
    many as the largest QR tile holds): a factor set with larger boxes
    (leaves of 200 rows, or k = 80 so that the inner boxes have 160) is
    refused at creation, before any launch, never at compression time."""
    hbs = _lib()
    for n, leaf, k, s in [(1600, 200, 60, 400), (2560, 160, 80, 250)]:
        t = hbs.Tree(n, leaf)
        with pytest.raises(hbs.HBSError) as e:
            hbs.Factors.create(t, k, s, "split", truncation)
        assert e.value.status == hbs.HBS_EUNSUPPORTED, (n, leaf, k, s)


def test_unknown_mode_bits_are_rejected():
    hbs = _lib()
    lib = hbs.load()
    t = hbs.Tree(1024, 32)
    h = ctypes.c_void_p()
    assert lib.hbs_factors_create(t._h, 16, 58, 0x1000, ctypes.byref(h)) == hbs.HBS_EINVAL
    assert lib.hbs_factors_create(t._h, 16, 58, 0x100 | 7, ctypes.byref(h)) == hbs.HBS_EUNSUPPORTED


def test_reporting_entry_points_validate_before_device_work():
    """hbs_power_norm and hbs_floats_per_dof reject bad arguments synchronously
    (no operator, no start vector, no steps, NULL outputs)."""
    hbs = _lib()
    lib = hbs.load()
    out = ctypes.c_double()
    dummy = ctypes.c_void_p(8)  # never dereferenced: every call below fails its argument checks first
    fn = ctypes.cast(lib.hbs_matvec_factors, ctypes.c_void_p)
    assert lib.hbs_power_norm(None, None, None, 16, dummy, 20, ctypes.byref(out), None) == hbs.HBS_EINVAL
    assert lib.hbs_power_norm(None, fn, None, 0, dummy, 20, ctypes.byref(out), None) == hbs.HBS_EINVAL
    assert lib.hbs_power_norm(None, fn, None, 16, None, 20, ctypes.byref(out), None) == hbs.HBS_EINVAL
    assert lib.hbs_power_norm(None, fn, None, 16, dummy, 0, ctypes.byref(out), None) == hbs.HBS_EINVAL
    assert lib.hbs_power_norm(None, fn, None, 16, dummy, 20, None, None) == hbs.HBS_EINVAL
    assert lib.hbs_floats_per_dof(None, ctypes.byref(out)) == hbs.HBS_EINVAL
    lib.hbs_matvec_logkernel.restype = ctypes.c_int32
    lib.hbs_matvec_logkernel.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]
    assert lib.hbs_matvec_logkernel(None, 0, dummy, dummy, None) == hbs.HBS_EINVAL
    pts = hbs.LogKernelPoints(0, 8, 8)
    assert lib.hbs_matvec_logkernel(ctypes.cast(ctypes.pointer(pts), ctypes.c_void_p), 0, dummy, dummy,
                                    None) == hbs.HBS_EINVAL


def test_streamed_sampling_rejects_null_arguments():
    """hbs_compress_logkernel checks its arguments before any device work:
    a NULL factor set or NULL arrays are HBS_EINVAL (no GPU needed)."""
    hbs = _lib()
    lib = hbs.load()
    one = ctypes.c_void_p(8)
    assert lib.hbs_compress_logkernel(None, one, one, one, one, one, one, 160, 0, 8, None) == hbs.HBS_EINVAL
    assert lib.hbs_compress_logkernel(None, None, one, one, one, one, one, 160, 0, 8, None) == hbs.HBS_EINVAL
