"""Python binding of libhbs (argument marshalling only).

Every operation runs inside the HIP library ``libhbs.so`` built next to this
file (``python -m paper_2205_02990_amd.build``).  PyTorch supplies device
memory and the current HIP stream; nothing here computes any part of the
method, and there is no fallback: if the library or a GPU is missing the
calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhbs.so")

HBS_OK, HBS_EINVAL, HBS_ENOMEM, HBS_EDEVICE, HBS_ENUMERIC, HBS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PRECISION = {"fp64": 0, "split": 1, "fp32_split": 1, "bf16": 2}
TRUNCATION = {"qr": 0, "svd": 0x100}  # hbs_truncation, OR-ed into the precision argument


def _mode(precision: str, truncation: str) -> int:
    return PRECISION[precision] | TRUNCATION[truncation]
PLAN_COLS = 20  # HBS_PLAN_COLS

_lib = None
_hip = None


class HBSError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = load().hbs_status_str(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


class LevelView(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("nodes", ctypes.c_int32), ("m", ctypes.c_int32),
                ("k", ctypes.c_int32), ("m_tau", ctypes.c_void_p), ("U", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("D", ctypes.c_void_p)]


def load():
    """Load libhbs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2205_02990_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, VP = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    sigs = {
        "hbs_tree_create": (I32, [I64, I32, ctypes.POINTER(P)]),
        "hbs_tree_destroy": (None, [P]),
        "hbs_tree_levels": (I32, [P]),
        "hbs_tree_node": (I32, [P, I32, I64, ctypes.POINTER(I64), ctypes.POINTER(I64)]),
        "hbs_factors_create": (I32, [P, I32, I32, I32, ctypes.POINTER(P)]),
        "hbs_factors_destroy": (None, [P]),
        "hbs_compress_into": (I32, [P, VP, VP, VP, VP, I64, VP]),
        "hbs_compress": (I32, [P, I32, I32, VP, VP, VP, VP, I64, I32, VP, ctypes.POINTER(P)]),
        "hbs_apply": (I32, [P, ctypes.c_int, VP, VP, I64, I64, VP]),
        "hbs_apply_static": (I32, [P, ctypes.c_int, VP, VP, I64, I64, VP]),
        "hbs_apply_static_max": (I64, [P]),
        "hbs_factors_import": (I32, [P, I32, ctypes.POINTER(LevelView), VP, VP, ctypes.POINTER(P)]),
        "hbs_level": (I32, [P, I32, ctypes.POINTER(LevelView)]),
        "hbs_root": (I32, [P, ctypes.POINTER(P), ctypes.POINTER(I32)]),
        "hbs_check": (I32, [P]),
        "hbs_status_str": (ctypes.c_char_p, [I32]),
        "hbs_sample_logkernel": (I32, [I64, VP, VP, VP, VP, VP, VP, I32, I64, I32, VP]),
        "hbs_compress_logkernel": (I32, [P, VP, VP, VP, VP, VP, VP, I64, I32, I32, VP]),
        "hbs_profile": (I32, [P, ctypes.c_int]),
        "hbs_profile_read": (I32, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64), I32]),
        "hbs_batch_create": (I32, [I32, ctypes.POINTER(P), ctypes.POINTER(I32), ctypes.POINTER(I32), I32,
                                   ctypes.POINTER(P)]),
        "hbs_batch_destroy": (None, [P]),
        "hbs_batch_compress": (I32, [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(P), ctypes.POINTER(I64), VP]),
        "hbs_batch_factors": (I32, [P, I32, ctypes.POINTER(P)]),
        "hbs_compress_batched": (I32, [I32, ctypes.POINTER(P), ctypes.POINTER(I32), ctypes.POINTER(I32),
                                       ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                       ctypes.POINTER(P), ctypes.POINTER(I64), I32, VP, ctypes.POINTER(P)]),
        "hbs_floats_per_dof": (I32, [P, ctypes.POINTER(ctypes.c_double)]),
        "hbs_power_norm": (I32, [P, VP, VP, I64, VP, I32, ctypes.POINTER(ctypes.c_double), VP]),
        "hbs_sweep_plan": (I32, [P, ctypes.POINTER(I32), I32, ctypes.POINTER(I32)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _hiprt():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.restype = ctypes.c_int
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.c_void_p]
    return _hip


def _check(status: int, what: str):
    if status != HBS_OK:
        raise HBSError(status, what)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
        raise ValueError(f"{name} must be a 2-D row-major float64 GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _copy_out(ptr: int, shape, stream=None) -> torch.Tensor:
    """Copy device memory owned by the library into a new torch tensor."""
    out = torch.empty(shape, dtype=torch.float64, device="cuda")
    nbytes = out.numel() * 8
    if nbytes:
        st = _hiprt().hipMemcpyAsync(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), nbytes, 3,
                                     _stream(stream))
        if st != 0:
            raise RuntimeError(f"hipMemcpyAsync failed ({st})")
    return out


class Tree:
    """Cluster tree of section 3.1 (built by the library)."""

    def __init__(self, n: int, leaf_max: int):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.hbs_tree_create(int(n), int(leaf_max), ctypes.byref(h)), "hbs_tree_create")
        self._h = h
        self.n = int(n)
        self.leaf_max = int(leaf_max)
        self.levels = lib.hbs_tree_levels(h)

    def node(self, level: int, i: int):
        st, sz = ctypes.c_int64(), ctypes.c_int64()
        _check(load().hbs_tree_node(self._h, int(level), int(i), ctypes.byref(st), ctypes.byref(sz)),
               "hbs_tree_node")
        return st.value, sz.value

    def ranges(self, level: int):
        return [(a, a + m) for a, m in (self.node(level, i) for i in range(2 ** level))]

    def leaf_sizes(self):
        return [m for _, m in (self.node(self.levels, i) for i in range(2 ** self.levels))]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbs_tree_destroy(self._h)
            self._h = None


class Factors:
    """Telescoping factors of an HBS matrix held by the library."""

    def __init__(self, handle, tree: Tree, k: int):
        self._h = handle
        self.tree = tree
        self.k = int(k)

    @classmethod
    def create(cls, tree: Tree, k: int, s: int, precision: str = "fp64", truncation: str = "qr"):
        h = ctypes.c_void_p()
        _check(load().hbs_factors_create(tree._h, int(k), int(s), _mode(precision, truncation), ctypes.byref(h)),
               "hbs_factors_create")
        f = cls(h, tree, k)
        f.s = int(s)
        return f

    def compress_into(self, Om, Y, Ps, Z, stream=None):
        ld = Om.stride(0)
        for t in (Y, Ps, Z):
            if t.stride(0) != ld:
                raise ValueError("Omega, Y, Psi, Z must share one leading dimension")
        _check(load().hbs_compress_into(self._h, _dev_f64(Om, "Omega"), _dev_f64(Y, "Y"), _dev_f64(Ps, "Psi"),
                                        _dev_f64(Z, "Z"), ld, _stream(stream)), "hbs_compress_into")
        return self

    def compress_logkernel(self, x: torch.Tensor, y: torch.Tensor, Om: torch.Tensor, Ps: torch.Tensor,
                           Y: torch.Tensor, Z: torch.Tensor, sampler: str = "fp64", chunks: int = 8, stream=None):
        """Sample the log kernel on points (x, y) into Y, Z and compress them,
        the leaf level streamed behind the sampler in `chunks` row ranges
        (hbs_compress_logkernel)."""
        ld = Om.stride(0)
        for t in (Y, Ps, Z):
            if t.stride(0) != ld:
                raise ValueError("Omega, Y, Psi, Z must share one leading dimension")
        _check(load().hbs_compress_logkernel(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                             _dev_f64(Om, "Omega"), _dev_f64(Ps, "Psi"), _dev_f64(Y, "Y"),
                                             _dev_f64(Z, "Z"), ld, PRECISION[sampler], int(chunks), _stream(stream)),
               "hbs_compress_logkernel")
        return self

    def apply(self, X: torch.Tensor, transpose: bool = False, out: torch.Tensor | None = None, stream=None):
        vec = X.dim() == 1
        X2 = X.reshape(-1, 1) if vec else X
        if X2.stride(1) != 1:
            X2 = X2.contiguous()
        if out is None:
            out = torch.empty((X2.shape[0], X2.shape[1]), dtype=torch.float64, device=X2.device)
        if out.stride(0) != X2.stride(0):
            raise ValueError("out must share X's leading dimension")
        _check(load().hbs_apply(self._h, 1 if transpose else 0, _dev_f64(X2, "X"), _dev_f64(out, "out"),
                                X2.shape[1], X2.stride(0), _stream(stream)), "hbs_apply")
        return out.reshape(-1) if vec else out

    def check(self):
        st = load().hbs_check(self._h)
        if st == HBS_ENUMERIC:
            raise HBSError(st, "hbs_check")
        _check(st, "hbs_check")

    def profile(self, enable: bool = True):
        """Bracket every later sweep kernel with HIP events (see hbs_profile)."""
        _check(load().hbs_profile(self._h, 1 if enable else 0), "hbs_profile")

    def profile_read(self) -> dict:
        """Summed device ms and launch counts per kernel class since the last read."""
        return _profile_read(self._h)

    def level(self, level: int, stream=None) -> dict:
        v = LevelView()
        _check(load().hbs_level(self._h, int(level), ctypes.byref(v)), "hbs_level")
        return {"m": v.m, "nodes": v.nodes,
                "U": _copy_out(v.U, (v.nodes, v.m, v.k), stream),
                "V": _copy_out(v.V, (v.nodes, v.m, v.k), stream),
                "D": _copy_out(v.D, (v.nodes, v.m, v.m), stream)}

    def floats_per_dof(self) -> float:
        """Stored FP64 values per degree of freedom (quantity (4) of section 5)."""
        out = ctypes.c_double()
        _check(load().hbs_floats_per_dof(self._h, ctypes.byref(out)), "hbs_floats_per_dof")
        return out.value

    def _matvec(self):
        return ctypes.cast(load().hbs_matvec_factors, ctypes.c_void_p), self._h

    def plan(self) -> list:
        """Tile plan of the sweep, one dict per launch step (hbs_sweep_plan)."""
        lib = load()
        n = ctypes.c_int32()
        _check(lib.hbs_sweep_plan(self._h, None, 0, ctypes.byref(n)), "hbs_sweep_plan")
        rows = (ctypes.c_int32 * (PLAN_COLS * max(n.value, 1)))()
        _check(lib.hbs_sweep_plan(self._h, rows, n.value, ctypes.byref(n)), "hbs_sweep_plan")
        out = []
        for i in range(n.value):
            r = rows[PLAN_COLS * i:PLAN_COLS * (i + 1)]
            out.append({"step": r[0], "boxes": r[1], "mmax": r[2], "s": r[3], "k": r[4], "root": bool(r[5]),
                        "tuned": bool(r[6]), "lq": {"threads": r[7], "lanes_per_row": r[8], "test_slots": r[9],
                                                    "sample_slots": r[10], "col_slots": r[11], "chunks": r[12],
                                                    "waves_per_simd_cap": r[18]},
                        "col": None if r[5] else {"threads": r[13], "lanes_per_row": r[14], "row_slots": r[15],
                                                  "col_slots": r[16], "waves_per_simd_cap": r[19]},
                        "tail_b": None if r[5] else r[17]})
        return out

    def root(self, stream=None) -> torch.Tensor:
        p, n = ctypes.c_void_p(), ctypes.c_int32()
        _check(load().hbs_root(self._h, ctypes.byref(p), ctypes.byref(n)), "hbs_root")
        return _copy_out(p.value, (n.value, n.value), stream)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbs_factors_destroy(self._h)
            self._h = None


PROFILE_CLASSES = ("lq", "col", "tail_a", "tail_b", "tail_c", "root")


def _profile_read(h) -> dict:
    nc = len(PROFILE_CLASSES)
    ms = (ctypes.c_double * nc)()
    n = (ctypes.c_int64 * nc)()
    _check(load().hbs_profile_read(h, ms, n, nc), "hbs_profile_read")
    return {PROFILE_CLASSES[i]: (ms[i], n[i]) for i in range(nc)}


def _ptrs(ts, name):
    return (ctypes.c_void_p * len(ts))(*[_dev_f64(t, f"{name}[{i}]").value for i, t in enumerate(ts)])


class Batch:
    """Independent compressions sharing one sweep (hbs_batch_*)."""

    def __init__(self, trees, ks, ss, precision: str = "fp64", truncation: str = "qr"):
        lib = load()
        c = len(trees)
        self.trees = list(trees)
        self.ks = [int(x) for x in ks]
        self.ss = [int(x) for x in ss]
        th = (ctypes.c_void_p * c)(*[t._h.value for t in self.trees])
        h = ctypes.c_void_p()
        _check(lib.hbs_batch_create(c, th, (ctypes.c_int32 * c)(*self.ks), (ctypes.c_int32 * c)(*self.ss),
                                    _mode(precision, truncation), ctypes.byref(h)), "hbs_batch_create")
        self._h = h

    def __len__(self):
        return len(self.trees)

    def compress(self, Om, Y, Ps, Z, stream=None):
        """Om, Y, Ps, Z: lists of per-instance N_i x s_i device tensors."""
        c = len(self.trees)
        if not all(len(x) == c for x in (Om, Y, Ps, Z)):
            raise ValueError("one panel of each kind per instance")
        ld = []
        for i in range(c):
            l0 = Om[i].stride(0)
            if any(t.stride(0) != l0 for t in (Y[i], Ps[i], Z[i])):
                raise ValueError("the panels of one instance must share a leading dimension")
            ld.append(l0)
        _check(load().hbs_batch_compress(self._h, _ptrs(Om, "Omega"), _ptrs(Y, "Y"), _ptrs(Ps, "Psi"),
                                         _ptrs(Z, "Z"), (ctypes.c_int64 * c)(*ld), _stream(stream)),
               "hbs_batch_compress")
        return self

    def factors(self, i: int) -> Factors:
        h = ctypes.c_void_p()
        _check(load().hbs_batch_factors(self._h, int(i), ctypes.byref(h)), "hbs_batch_factors")
        f = Factors(h, self.trees[i], self.ks[i])
        f.s = self.ss[i]
        return f

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbs_batch_destroy(self._h)
            self._h = None


def compress_batched(trees, ks, Om, Y, Ps, Z, precision: str = "fp64", stream=None, truncation: str = "qr"):
    """hbs_compress_batched: one Factors per instance."""
    c = len(trees)
    ld = [t.stride(0) for t in Om]
    th = (ctypes.c_void_p * c)(*[t._h.value for t in trees])
    ss = [t.shape[1] for t in Om]
    out = (ctypes.c_void_p * c)()
    _check(load().hbs_compress_batched(c, th, (ctypes.c_int32 * c)(*[int(k) for k in ks]),
                                       (ctypes.c_int32 * c)(*ss), _ptrs(Om, "Omega"), _ptrs(Y, "Y"),
                                       _ptrs(Ps, "Psi"), _ptrs(Z, "Z"), (ctypes.c_int64 * c)(*ld),
                                       _mode(precision, truncation), _stream(stream), out),
           "hbs_compress_batched")
    res = []
    for i in range(c):
        f = Factors(ctypes.c_void_p(out[i]), trees[i], ks[i])
        f.s = ss[i]
        res.append(f)
    return res


def compress(tree: Tree, k: int, Om, Y, Ps, Z, precision: str = "fp64", stream=None,
             truncation: str = "qr") -> Factors:
    """Algorithm 2 on the GPU: allocate a factor set and fill it."""
    f = Factors.create(tree, k, Om.shape[1], precision, truncation)
    return f.compress_into(Om, Y, Ps, Z, stream)


def import_factors(tree: Tree, k: int, levels: dict, D0: torch.Tensor, stream=None) -> Factors:
    """Wrap known factors (e.g. a synthetic generator) as a factor set.

    ``levels[l]`` (l = 1..L) is a dict with device tensors U, V of shape
    (nodes, m, k) and D of shape (nodes, m, m), padded with zeros to the
    largest node m of the level."""
    L = tree.levels
    views = (LevelView * max(L, 1))()
    keep = []
    for l in range(1, L + 1):
        U, V, D = (levels[l][x].contiguous() for x in ("U", "V", "D"))
        keep += [U, V, D]
        views[l - 1] = LevelView(l, U.shape[0], U.shape[1], int(k), None, U.data_ptr(), V.data_ptr(), D.data_ptr())
    D0c = D0.contiguous()
    h = ctypes.c_void_p()
    _check(load().hbs_factors_import(tree._h, int(k), views, ctypes.c_void_p(D0c.data_ptr()), _stream(stream),
                                     ctypes.byref(h)), "hbs_factors_import")
    torch.cuda.current_stream().synchronize()
    return Factors(h, tree, k)


def sample_logkernel(x: torch.Tensor, y: torch.Tensor, Om: torch.Tensor, Ps: torch.Tensor,
                     precision: str = "fp64", stream=None):
    """Y = A Omega and Z = A Psi for A(i, j) = log|x_i - x_j| (i != j), 0 on the diagonal."""
    n, s = Om.shape
    Y = torch.empty_like(Om)
    Z = torch.empty_like(Ps)
    _check(load().hbs_sample_logkernel(n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       _dev_f64(Om, "Omega"), _dev_f64(Ps, "Psi"), _dev_f64(Y, "Y"),
                                       _dev_f64(Z, "Z"), s, Om.stride(0), PRECISION[precision], _stream(stream)),
           "hbs_sample_logkernel")
    return Y, Z


class LogKernelPoints(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class LogKernelBox:
    """The log-kernel black box (hbs_matvec_logkernel) on device point
    coordinates x, y (1-D float64 GPU tensors)."""

    def __init__(self, x: torch.Tensor, y: torch.Tensor):
        if not (x.is_cuda and y.is_cuda and x.dtype == y.dtype == torch.float64 and x.dim() == y.dim() == 1
                and x.shape == y.shape and x.is_contiguous() and y.is_contiguous()):
            raise ValueError("x, y must be contiguous 1-D float64 GPU tensors of one length")
        self.x, self.y = x, y
        self.pts = LogKernelPoints(x.shape[0], x.data_ptr(), y.data_ptr())

    def _matvec(self):
        return ctypes.cast(load().hbs_matvec_logkernel, ctypes.c_void_p), ctypes.cast(ctypes.pointer(self.pts),
                                                                                    ctypes.c_void_p)


def power_norm(factors: Factors | None, black_box, v0: torch.Tensor, steps: int = 20, stream=None) -> float:
    """Section 5's power-iteration estimate of ||A~ - B||_2 (hbs_power_norm);
    either operand may be None.  ``black_box`` is a Factors or LogKernelBox."""
    if not (v0.is_cuda and v0.dtype == torch.float64 and v0.dim() == 1 and v0.is_contiguous()):
        raise ValueError("v0 must be a contiguous 1-D float64 GPU tensor")
    fn, ctx = black_box._matvec() if black_box is not None else (None, None)
    out = ctypes.c_double()
    _check(load().hbs_power_norm(factors._h if factors is not None else None, fn, ctx, v0.shape[0],
                                 ctypes.c_void_p(v0.data_ptr()), int(steps), ctypes.byref(out), _stream(stream)),
           "hbs_power_norm")
    return out.value


def power_rel_error(factors: Factors, black_box, v0_err: torch.Tensor, v0_norm: torch.Tensor,
                    steps: int = 20, stream=None) -> float:
    """||A~ - B|| / ||B||, both by power_norm (section 5's accuracy measure)."""
    return power_norm(factors, black_box, v0_err, steps, stream) / power_norm(None, black_box, v0_norm, steps,
                                                                               stream)
