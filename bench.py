#!/usr/bin/env python3
"""Benchmark: HBS compression rows/s on one MI355X, mixed against FP64 path.

One step = one full compression sweep (Algorithm 2: every level from the
leaves to the root, all boxes of a level at once) of an N x N matrix from its
samples {Omega, Y = A Omega, Psi, Z = A^* Psi}, which are resident in HBM when
the timed region starts; for the batched workload (the default: 512
independent exact-rank instances of uneven N) one sweep covers every
instance.  The samples come from a stand-in black box, timed separately like
the paper's compression time without the matvec: Algorithm 1 on seeded
exact-rank generators, or the log-kernel sampler.

Both arithmetic paths run on the same inputs in one invocation: the
split-precision path (bulk products from exact 7-bit integer slices on the
int8 matrix cores) gives `value`, the plain FP64 path its own figures in
`paths.fp64`; errors against the generator (and, in the tests, the oracle)
are reported per path.

Output: one JSON line on stdout (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "HBS compression rows/s at fixed rel. apply error; mixed vs FP64 path, 1 GPU"
PEAK_FP64_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # CUs x SIMDs x FP64 lanes x FMA x clock = 78.6
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# flop model (LAPACK operation counts of what one box computes)
# --------------------------------------------------------------------------

def lq_flops(m, s):
    """One side of one box in the QR kernel: Householder QR of the m x s test
    block (2 s m^2 - 2/3 m^3), its m reflectors applied to the m x s sample
    block (4 m^2 s - 2 m^3), and the triangular solve for Y Omega^dagger (m^3)."""
    return 2 * s * m * m - 2 * m ** 3 / 3 + 4 * m * m * s - 2 * m ** 3 + m ** 3


def col_flops(m, s, k):
    """One side of one box in the basis kernel: truncated column-pivoted QR of
    the m x r sketch, r = s - m, stopped after k steps
    (4 m r k - 2 (m + r) k^2 + 4/3 k^3), plus forming its m x k Q
    (2 m k^2 - 2/3 k^3)."""
    r = s - m
    return 4 * m * r * k - 2 * (m + r) * k * k + 4 * k ** 3 / 3 + 2 * m * k * k - 2 * k ** 3 / 3


def tail_flops(m, s, k):
    """The products after the bases: X U, W V, U^* W, and U times the k x m
    term of D (2 m^2 k each); V^* F, U^* Q, V G, U G2 (2 m k^2 each); and the
    six k x m x s products with the test and sample blocks (2 k m s each)."""
    return 8 * m * m * k + 8 * m * k * k + 12 * k * m * s


def nominal_side(m, s, k):
    """The fixed flop model used for every fraction reported: the literal
    Algorithm 2 with LAPACK operation counts, per side (Omega/Y or Psi/Z) of
    one box of m rows: Householder QR of the s x m test block, forming the k
    null columns P, Y P, thin QR of Y P with its Q, the pseudo-inverse through
    the explicit Q1 and Y Omega^dagger, the projections, and the parent
    blocks.  Returns the terms by name."""
    return {"qr": 2 * m * m * (s - m / 3), "form_p": 4 * s * k * m - 2 * k * m * m, "yp": 2 * m * s * k,
            "thin_qr": 4 * m * k * k - 4 * k ** 3 / 3,
            "pinv": 2 * s * m * m - 2 * m ** 3 / 3 + 2 * m * m * s + m ** 3,
            "proj": 4 * m * m * k, "parent": 2 * m * m * s + 4 * k * m * s}


def nominal_lq(m, s, k):
    """The part of the fixed model the QR kernel carries out, per side: the
    QR of the test block, the null columns applied to the samples (P, Y P)
    and Y Omega^dagger."""
    t = nominal_side(m, s, k)
    return t["qr"] + t["form_p"] + t["yp"] + t["pinv"]


def nominal_box(m, s, k):
    """The fixed model for one box: both sides, plus 4 m^2 k to combine D."""
    return 2 * sum(nominal_side(m, s, k).values()) + 4 * m * m * k


def sweep_model(leaf_sizes, k, s):
    """Per-step flop totals by kernel class, algorithmic HBM bytes of the QR
    kernel, and the launch count of each per-level kernel."""
    L = int(round(math.log2(len(leaf_sizes))))
    lq = col = tail = 0.0
    lq_bytes = 0
    nom = nom_lq = 0.0
    for lev in range(L, 0, -1):
        ms = leaf_sizes if lev == L else [2 * k] * (2 ** lev)
        for m in ms:
            lq += 2 * lq_flops(m, s)
            col += 2 * col_flops(m, s, k)
            tail += tail_flops(m, s, k)
            nom += nominal_box(m, s, k)
            nom_lq += 2 * nominal_lq(m, s, k)
            # each side reads its two m x s panels, writes W (m x m) and the
            # transposed m x (s - m) nullspace sketch
            lq_bytes += 2 * 8 * (2 * m * s + m * m + m * (s - m))
    m0 = 2 * k if L > 0 else leaf_sizes[0]
    root = lq_flops(m0, s)
    t0 = nominal_side(m0, s, k)
    nom += t0["qr"] + t0["pinv"]  # the root: D^(0) = Y Omega^dagger
    return {"lq": lq, "col": col, "tail": tail, "root": root, "launches": L,
            "lq_bytes": lq_bytes, "nominal": nom, "nominal_lq": nom_lq}


# --------------------------------------------------------------------------
# CPU baseline (the oracle on a bounded sample of the workload)
# --------------------------------------------------------------------------

def _threads():
    import threadpoolctl
    info = threadpoolctl.threadpool_info()
    return int(max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1]))


def _timed_oracle(jobs, single_thread=False):
    """Time the FP64 oracle's Algorithm 2 on each (levels, k, Om, Y, Ps, Z)
    job; returns (rows, seconds, threads used)."""
    import threadpoolctl

    from oracle import hbs as ohbs
    rows = sum(j[2].shape[0] for j in jobs)
    with threadpoolctl.threadpool_limits(1 if single_thread else None):
        threads = _threads()
        t0 = time.perf_counter()
        for levels, k, Om, Y, Ps, Z in jobs:
            ohbs.compress(levels, k, Om, Y, Ps, Z)
        dt = time.perf_counter() - t0
    return rows, dt, threads


def _oracle_synthetic(inputs, n, k, leaf, s, rs):
    """An exact-rank instance drawn and sampled by the oracle alone (CPU)."""
    from oracle import hbs as ohbs
    from oracle import tree as otree
    levels = otree.cluster_tree(n, leaf)
    gen = ohbs.from_generators(levels, inputs.synthetic_generators(rs[inputs.STREAM_GENERATOR],
                                                                  otree.leaf_sizes(levels), k))
    Om = inputs.gaussian(rs[inputs.STREAM_OMEGA], n, s)
    Ps = inputs.gaussian(rs[inputs.STREAM_PSI], n, s)
    return levels, k, Om, ohbs.apply(gen, Om), Ps, ohbs.apply(gen, Ps, transpose=True)


def cpu_result(jobs, multi_jobs, sample):
    """The oracle's rate on `jobs` with BLAS held to one thread (faster on
    these small boxes: threads cost more than the products they split) and,
    for comparison, on `multi_jobs` with the host's default BLAS threads."""
    rows, dt, _ = _timed_oracle(jobs, single_thread=True)
    out = {"value": rows / dt, "unit": "rows/s", "cores": 1, "kind": "oracle",
           "sample": f"{sample}; {rows} rows in {dt:.1f} s with BLAS held to one thread; "
                     f"host os.cpu_count()={os.cpu_count()}"}
    if multi_jobs:
        r1, d1, thr = _timed_oracle(multi_jobs)
        out["default_threads"] = {"value": r1 / d1, "unit": "rows/s", "cores": thr,
                                  "sample": f"{r1} rows in {d1:.1f} s with the default BLAS threads"}
    return out


# --------------------------------------------------------------------------
# workloads: inputs on the device once, then a factor set per path
# --------------------------------------------------------------------------

class Problem:
    pass


def _power_starts(inputs, wid, n, torch, dev):
    """Seeded starting vectors of the two power iterations (error, norm)."""
    rs = inputs.streams(wid, 2, extra=(0x50,))
    return tuple(torch.from_numpy(inputs.gaussian(r, n, 1)[:, 0].copy()).to(dev) for r in rs)


def setup_logkernel(wl, args, hbs, torch, inputs, dev):
    n, k, leaf, s = wl["n"], wl["k"], wl["leaf_max"], wl["s"]
    rs = inputs.streams(wl["id"])
    x, y = inputs.ellipse_points(n, wl["a"], wl["b"])
    Om = inputs.gaussian(rs[inputs.STREAM_OMEGA], n, s)
    Ps = inputs.gaussian(rs[inputs.STREAM_PSI], n, s)
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    Omd, Psd = torch.from_numpy(Om).to(dev), torch.from_numpy(Ps).to(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    Yd, Zd = hbs.sample_logkernel(xd, yd, Omd, Psd, precision=args.sampler)  # warm
    e0.record()
    Yd, Zd = hbs.sample_logkernel(xd, yd, Omd, Psd, precision=args.sampler)
    e1.record()
    torch.cuda.synchronize()
    P = Problem()
    P.sampler_ms = e0.elapsed_time(e1)
    tree = hbs.Tree(n, leaf)
    P.rows = n
    P.leaf_sets = [(tree.leaf_sizes(), k, s)]
    P.config = {"N": n, "k": k, "leaf_max": leaf, "leaf": tree.leaf_sizes()[0], "s": s, "levels": tree.levels,
                "sampler": args.sampler}
    G = torch.from_numpy(inputs.probes(rs[inputs.STREAM_PROBES], n, 8)).to(dev)

    def build(path):
        f = hbs.Factors.create(tree, k, s, path, args.truncation)

        def error():
            AG, _ = hbs.sample_logkernel(xd, yd, G, G)
            e = float(torch.linalg.norm(f.apply(G) - AG) / torch.linalg.norm(AG))
            ins = float(torch.linalg.norm(f.apply(Omd) - Yd) / torch.linalg.norm(Yd))
            pw = hbs.power_rel_error(f, hbs.LogKernelBox(xd, yd), *_power_starts(inputs, wl["id"], n, torch, dev))
            return {"rel_apply_err": e, "in_sample_err": ins, "reference": "the black box on 8 Gaussian probes",
                    "power_rel_err": pw, "floats_per_dof": f.floats_per_dof()}
        return (lambda: f.compress_into(Omd, Yd, Psd, Zd)), f, error
    P.build = build

    def streamed(path, chunks, steps):
        """Sampling plus compression, one after the other (chunks = 1) and with
        the leaf level streamed behind the sampler (hbs_compress_logkernel)."""
        f = hbs.Factors.create(tree, k, s, path, args.truncation)
        Y2, Z2 = torch.empty_like(Omd), torch.empty_like(Psd)
        f.compress_logkernel(xd, yd, Omd, Psd, Y2, Z2, args.sampler, 1)  # times the tiles
        out = {"chunks": chunks, "path": path}
        for name, c in (("sample_then_sweep_ms", 1), ("streamed_ms", chunks)):
            f.compress_logkernel(xd, yd, Omd, Psd, Y2, Z2, args.sampler, c)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                f.compress_logkernel(xd, yd, Omd, Psd, Y2, Z2, args.sampler, c)
            e1.record()
            torch.cuda.synchronize()
            f.check()
            out[name] = e0.elapsed_time(e1) / steps
        out["saved_ms"] = out["sample_then_sweep_ms"] - out["streamed_ms"]
        return out
    P.streamed = streamed

    def cpu():
        from oracle import logkernel as olog
        from oracle import tree as otree
        levels = otree.cluster_tree(n, leaf)
        a, b = levels[args.cpu_subtree_level][0]
        sub = otree.cluster_tree(b - a, leaf)
        YZ = olog.sample(x, y, np.hstack((Om, Ps)), np.arange(a, b))  # the oracle's samples of those rows
        job = (sub, k, Om[a:b], YZ[:, :s], Ps[a:b], YZ[:, s:])
        return cpu_result([job], [job], f"oracle Algorithm 2 on the {b - a}-row subtree under the first node of "
                                        f"level {args.cpu_subtree_level} of {args.workload} (all its "
                                        f"{otree.depth(sub)} levels)")
    P.cpu = cpu
    return P


def _synthetic_instance(hbs, torch, inputs, dev, n, k, leaf, s, rs):
    """Import a seeded exact-rank generator; samples by the library's Algorithm 1."""
    tree = hbs.Tree(n, leaf)
    gen = inputs.synthetic_generators(rs[inputs.STREAM_GENERATOR], tree.leaf_sizes(), k)
    lv = {}
    for l in range(1, tree.levels + 1):
        mm = max(U.shape[0] for U in gen["U"][l])
        pad = lambda blocks, c: np.stack([np.pad(b_, ((0, mm - b_.shape[0]), (0, c - b_.shape[1]))) for b_ in blocks])
        lv[l] = {"U": torch.from_numpy(pad(gen["U"][l], k)).to(dev), "V": torch.from_numpy(pad(gen["V"][l], k)).to(dev),
                 "D": torch.from_numpy(pad(gen["D"][l], mm)).to(dev)}
    A = hbs.import_factors(tree, k, lv, torch.from_numpy(gen["D0"]).to(dev))
    del lv
    Om = torch.from_numpy(inputs.gaussian(rs[inputs.STREAM_OMEGA], n, s)).to(dev)
    Ps = torch.from_numpy(inputs.gaussian(rs[inputs.STREAM_PSI], n, s)).to(dev)
    Y = A.apply(Om)
    Z = A.apply(Ps, transpose=True)
    G = torch.from_numpy(inputs.probes(rs[inputs.STREAM_PROBES], n, 8)).to(dev)
    return tree, A, Om, Y, Ps, Z, G


def setup_synthetic(wl, args, hbs, torch, inputs, dev):
    n, k, leaf, s = wl["n"], wl["k"], wl["leaf_max"], wl["s"]
    t0 = time.perf_counter()
    tree, A, Om, Y, Ps, Z, G = _synthetic_instance(hbs, torch, inputs, dev, n, k, leaf, s, inputs.streams(wl["id"]))
    torch.cuda.synchronize()
    log(f"generator and samples ready in {time.perf_counter() - t0:.1f} s")
    P = Problem()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    A.apply(Om)
    A.apply(Ps, transpose=True)
    e1.record()
    torch.cuda.synchronize()
    P.sampler_ms = e0.elapsed_time(e1)
    P.rows = n
    P.leaf_sets = [(tree.leaf_sizes(), k, s)]
    P.config = {"N": n, "k": k, "leaf_max": leaf, "leaf": tree.leaf_sizes()[0], "s": s, "levels": tree.levels,
                "sampler": "Algorithm 1 on the generator"}

    def build(path):
        f = hbs.Factors.create(tree, k, s, path, args.truncation)

        def error():
            AG = A.apply(G)
            e = float(torch.linalg.norm(f.apply(G) - AG) / torch.linalg.norm(AG))
            ins = float(torch.linalg.norm(f.apply(Om) - Y) / torch.linalg.norm(Y))
            pw = hbs.power_rel_error(f, A, *_power_starts(inputs, wl["id"], n, torch, dev))
            return {"rel_apply_err": e, "in_sample_err": ins, "reference": "the exact generator on 8 Gaussian probes",
                    "power_rel_err": pw, "floats_per_dof": f.floats_per_dof()}
        return (lambda: f.compress_into(Om, Y, Ps, Z)), f, error
    P.build = build

    def cpu():
        # a smaller instance of the same shape, drawn and sampled by the oracle
        nc = min(n, leaf * 2 ** 10)
        job = _oracle_synthetic(inputs, nc, k, leaf, s, inputs.streams(wl["id"], extra=(0xC0,)))
        multi = [job] if nc <= leaf * 2 ** 7 else \
            [_oracle_synthetic(inputs, leaf * 2 ** 7, k, leaf, s, inputs.streams(wl["id"], extra=(0xC1,)))]
        return cpu_result([job], multi, f"oracle Algorithm 2 on an exact-rank instance of {nc} rows with the "
                                        f"workload's k = {k}, leaf {leaf}, s = {s}, drawn and sampled on the CPU")
    P.cpu = cpu
    return P


def setup_batch(wl, args, hbs, torch, inputs, dev):
    spec = inputs.batch_instances(wl["id"], wl["count"], wl["n_lo"], wl["n_hi"], wl["ks"])
    t0 = time.perf_counter()
    inst = []
    for x in spec:
        rs = inputs.streams(wl["id"], extra=(x["index"],))
        inst.append(_synthetic_instance(hbs, torch, inputs, dev, x["n"], x["k"], x["leaf_max"], x["s"], rs))
    torch.cuda.synchronize()
    log(f"{len(spec)} generators and samples ready in {time.perf_counter() - t0:.1f} s")
    trees = [i[0] for i in inst]
    Om, Y, Ps, Z = ([i[j] for i in inst] for j in (2, 3, 4, 5))
    P = Problem()
    P.sampler_ms = float("nan")
    P.rows = sum(x["n"] for x in spec)
    P.leaf_sets = [(t.leaf_sizes(), x["k"], x["s"]) for t, x in zip(trees, spec)]
    P.config = {"instances": len(spec), "N_total": P.rows, "N_range": [wl["n_lo"], wl["n_hi"]], "k": list(wl["ks"]),
                "leaf_max": "2k", "s": "3k + 10", "levels": [min(t.levels for t in trees), max(t.levels for t in trees)]}

    def build(path):
        b = hbs.Batch(trees, [x["k"] for x in spec], [x["s"] for x in spec], path, args.truncation)

        def error():
            worst = 0.0
            for i, (tree, A, om, yy, ps, zz, G) in enumerate(inst):
                AG = A.apply(G)
                worst = max(worst, float(torch.linalg.norm(b.factors(i).apply(G) - AG) / torch.linalg.norm(AG)))
            i = max(range(len(spec)), key=lambda j: spec[j]["n"])
            pw = hbs.power_rel_error(b.factors(i), inst[i][1], *_power_starts(inputs, wl["id"], spec[i]["n"], torch,
                                                                                  dev))
            return {"rel_apply_err": worst, "reference": "each instance's exact generator on 8 Gaussian probes (worst)",
                    "power_rel_err": pw, "power_reference": f"largest instance ({spec[i]['n']} rows)",
                    "floats_per_dof": sum(b.factors(j).floats_per_dof() * spec[j]["n"] for j in range(len(spec)))
                    / P.rows}
        return (lambda: b.compress(Om, Y, Ps, Z)), b.factors(0), error
    P.build = build

    def cpu():
        # the first 32 instances (multi-threaded) and the first 8 (one thread),
        # drawn and sampled by the oracle with each instance's own seeds
        jobs = [_oracle_synthetic(inputs, x["n"], x["k"], x["leaf_max"], x["s"],
                                  inputs.streams(wl["id"], extra=(x["index"],))) for x in spec[:32]]
        return cpu_result(jobs, jobs[:4], "oracle Algorithm 2 on the first 32 of the 512 instances, each drawn and "
                                          "sampled on the CPU from its own seeds (default threads: the first 4)")
    P.cpu = cpu
    return P


def run_path(P, path, args, torch):
    """Warm up, time K sweeps (the captured graph), then K traced sweeps for
    per-kernel device time; returns the path's figures."""
    compress, f, error = P.build(path)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):
        compress()
    torch.cuda.synchronize()
    f.check()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        compress()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    f.check()
    rows_per_s = P.rows / (ms_per_step / 1e3)
    log(f"[{path}] {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f} ms), "
        f"{rows_per_s:.4g} rows/s")
    # the same K sweeps launched directly, each launch bracketed by HIP events
    # on the stream it runs on
    f.profile(True)
    f.profile_read()
    e0.record()
    for _ in range(args.steps):
        compress()
    e1.record()
    torch.cuda.synchronize()
    traced_ms = e0.elapsed_time(e1) / args.steps
    prof = f.profile_read()
    f.profile(False)
    f.check()
    log(f"[{path}] traced {traced_ms:.3f} ms/step; kernel ms/step: " +
        ", ".join(f"{c} {v[0] / args.steps:.3f} ({v[1] // args.steps} launches)" for c, v in prof.items()))
    acc = error()
    log(f"[{path}] accuracy: {acc}")
    plan = f.plan()
    tiles = [f"step {p['step']}: {p['boxes']} boxes m<={p['mmax']} lq {p['lq']['threads']}t/{p['lq']['lanes_per_row']}l "
             f"{p['lq']['test_slots']}x{p['lq']['sample_slots']}x{p['lq']['col_slots']} chunks {p['lq']['chunks']}"
             + (f" cap {p['lq']['waves_per_simd_cap']}w" if p['lq']['waves_per_simd_cap'] else "")
             + ("" if p["root"] else f", col {p['col']['threads']}t/{p['col']['lanes_per_row']}l "
                f"{p['col']['row_slots']}x{p['col']['col_slots']}"
                + (f" cap {p['col']['waves_per_simd_cap']}w" if p['col']['waves_per_simd_cap'] else "")
                + f", tail_b {p['tail_b']}")
             for p in plan]
    return {"rows_per_s": rows_per_s, "ms_per_step": ms_per_step, "traced_ms_per_step": traced_ms,
            "kernel_ms_per_step": {c: v[0] / args.steps for c, v in prof.items()},
            "lq_launches_per_step": prof["lq"][1] / args.steps, **acc,
            "tiles": {"autotuned": bool(plan and plan[0]["tuned"]), "steps": tiles}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="hbs_exact_batch512")
    ap.add_argument("--path", default="both", choices=["both", "fp64", "split"],
                    help="both: the split-precision path gives `value`, the FP64 path runs beside it")
    ap.add_argument("--truncation", default="qr", choices=["qr", "svd"])
    ap.add_argument("--slices", type=int, default=0, choices=[0, 6, 7, 8],
                    help="split path: 7-bit slices per operand (0: the library's default, 8)")
    ap.add_argument("--n", type=int, default=0,
                    help="single-instance workloads: N other than the workload's own (same k, leaf, s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream-chunks", type=int, default=0,
                    help="log-kernel workloads: also time sampling plus compression with the leaf level "
                         "streamed behind the sampler in this many row ranges")
    ap.add_argument("--cpu-subtree-level", type=int, default=4)
    ap.add_argument("--sampler", default="fp64", choices=["fp64", "bf16"])
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain copy kernel over MIB MiB (reference for HBM byte counters)")
    ap.add_argument("--trace-summary", metavar="RESULTS_DB",
                    help="no GPU run: print a markdown summary of a rocprofv3 --kernel-trace results file of "
                         "bench.py on --workload")
    ap.add_argument("--counter-summary", metavar="COUNTER_CSV",
                    help="no GPU run: print a markdown table of a rocprofv3 --pmc counter file")
    ap.add_argument("--traffic-out", metavar="JSON", default=None,
                    help="with --traffic-from: write the traffic file here instead of profiles/")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn the run_counter_collection.csv files of two rocprofv3 --pmc passes "
                         "(FETCH_SIZE, WRITE_SIZE) of bench.py --copy-probe MIB into the lq_kernel traffic file")
    args = ap.parse_args()
    if args.trace_summary:
        print(trace_summary(args.trace_summary, args.workload))
        return
    if args.counter_summary:
        print(counter_summary(args.counter_summary))
        return
    if args.traffic_from:
        traffic_from_counters(args.traffic_from[0], args.traffic_from[1], args.copy_probe or 512, args.workload,
                              dst=args.traffic_out, args=args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding of the tree is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import inputs
    from paper_2205_02990_amd import hbs

    wl = dict(inputs.WORKLOADS[args.workload])
    if args.n:
        if wl["kind"] == "batch":
            raise SystemExit("--n applies to single-instance workloads")
        wl["n"] = args.n
    if args.slices:
        os.environ["HBS_SPLIT_SLICES"] = str(args.slices)  # read when a factor set or batch is created
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    hbs.load()
    if args.copy_probe:
        # plain elementwise copy of a known size: reads and writes MIB MiB each
        src = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    setup = {"logkernel": setup_logkernel, "synthetic": setup_synthetic, "batch": setup_batch}[wl["kind"]]
    P = setup(wl, args, hbs, torch, inputs, dev)
    log(f"workload {args.workload}: {P.config}; sampler {P.sampler_ms:.2f} ms; truncation {args.truncation}")
    paths = ["split", "fp64"] if args.path == "both" else [args.path]
    res = {p: run_path(P, p, args, torch) for p in paths}
    streamed = None
    if args.stream_chunks > 1:
        if not hasattr(P, "streamed"):
            raise SystemExit("--stream-chunks applies to the log-kernel workloads")
        streamed = P.streamed(paths[-1], args.stream_chunks, args.steps)
        log(f"streamed: {streamed}")
    head = res[paths[0]]
    for p in paths:
        log(f"[{p}] tiles:\n  " + "\n  ".join(res[p]["tiles"]["steps"]))

    # ---- roofline of the dominant kernel (the QR kernel, FP64 on both paths)
    model = {"lq": 0.0, "col": 0.0, "tail": 0.0, "root": 0.0, "lq_bytes": 0.0, "nominal": 0.0, "nominal_lq": 0.0}
    for leaf_sizes, k, s in P.leaf_sets:
        mdl = sweep_model(leaf_sizes, k, s)
        for c in model:
            model[c] += mdl[c]
    lq_ms, lq_launches = head["kernel_ms_per_step"]["lq"], head["lq_launches_per_step"]
    avg_launch_ms = lq_ms / lq_launches
    per_launch = model["nominal_lq"] / lq_launches
    achieved = per_launch / (avg_launch_ms / 1e3) / 1e12
    own = model["lq"] / lq_launches / (avg_launch_ms / 1e3) / 1e12
    traffic = None
    tfile = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                         f"lq_kernel_{args.workload}_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tr = json.load(fh)
        if tr.get("source_digest") == _side_digest():
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_FP64_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
                "kernel": "lq_kernel", "flop_model": "nominal (literal Algorithm 2, LAPACK counts)",
                "flops_per_launch": per_launch, "avg_launch_ms": avg_launch_ms,
                "own_model_achieved": round(own, 3), "own_model_frac": round(own / PEAK_FP64_TFLOPS, 4),
                "algorithmic_hbm_bytes_per_launch": model["lq_bytes"] / lq_launches}

    def strip(r):
        return {k: v for k, v in r.items() if k not in ("tiles", "lq_launches_per_step")}
    out = {
        "metric": METRIC, "value": head["rows_per_s"], "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+i8-slices" if paths[0] == "split" else "f64", "data": "synthetic",
        "config": {"workload": args.workload + (f" at N = {args.n}" if args.n else ""), **P.config,
                   "path": paths[0], "truncation": args.truncation,
                   "slices": (args.slices or 8) if "split" in paths else None},
        "roofline": roofline,
        "rel_apply_err": head["rel_apply_err"], "power_rel_err": head["power_rel_err"],
        "paths": {p: strip(res[p]) for p in paths},
        "sampler_ms": P.sampler_ms,
        **({"streamed": streamed} if streamed else {}),
        "sweep_tflops_nominal": model["nominal"] / (head["ms_per_step"] / 1e3) / 1e12,
        "tiles": res[paths[0]]["tiles"],
    }
    if len(paths) == 2:
        out["mixed_vs_fp64_speedup"] = res["fp64"]["ms_per_step"] / res["split"]["ms_per_step"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = P.cpu()
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


def lq_launch_roots(workload):
    """Whether each QR-kernel launch of one sweep is a root launch, in launch
    order (host arithmetic on the trees, no GPU): one launch per aligned
    level and (k, s) class, the roots last."""
    import inputs

    from paper_2205_02990_amd import hbs

    wl = inputs_workloads()[workload]
    if wl["kind"] != "batch":
        return [False] * hbs.Tree(wl["n"], wl["leaf_max"]).levels + [True]
    spec = inputs.batch_instances(wl["id"], wl["count"], wl["n_lo"], wl["n_hi"], wl["ks"])
    L = [hbs.Tree(x["n"], x["leaf_max"]).levels for x in spec]
    classes = sorted({(x["k"], x["s"]) for x in spec})
    maxL = max(L)
    roots = []
    for j in range(maxL + 1):
        for c in classes:
            if j == maxL or any(Li > j for Li, x in zip(L, spec) if (x["k"], x["s"]) == c):
                roots.append(j == maxL)
    return roots


def traffic_from_counters(fetch_csv, write_csv, mib, workload, dst=None, args=None):
    """HBM bytes per lq_kernel launch from two rocprofv3 --pmc passes of
    `bench.py --copy-probe MIB` (FETCH_SIZE, then WRITE_SIZE, in KiB per
    dispatch).  Each counter is scaled by what it reads for the plain MIB MiB
    copy of the same run; the bytes average the last six sweeps (after the
    autotuner's timing launches), each sweep's root launches left out,
    matching the launches the roofline's time covers.  Written, with the
    digest of the QR kernel's source, to the profiles file bench.py reads."""
    import csv

    roots = lq_launch_roots(workload)
    per = len(roots)
    res = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        with open(path) as fh:
            rows = [r for r in csv.DictReader(fh) if r["Counter_Name"] == name]
        copy = [float(r["Counter_Value"]) for r in rows if "MulFunctor" in r["Kernel_Name"]]
        if not copy:
            raise SystemExit(f"{path}: no copy-probe dispatch (run bench.py with --copy-probe)")
        scale = mib * 1024.0 / (sum(copy) / len(copy))
        lq = [r for r in rows if "lq_kernel" in r["Kernel_Name"]][-6 * per:]
        sweeps = [lq[i:i + per] for i in range(0, len(lq) - len(lq) % per, per)]
        vals = [[float(r["Counter_Value"]) * scale * 1024 for r, root in zip(sw, roots) if not root]
                for sw in sweeps]
        nl = len(vals[0])
        res[name] = dict(scale=scale, copy_kib=copy[0],
                         per_launch=[sum(v[i] for v in vals) / len(vals) for i in range(nl)])
    fetch, write = res["FETCH_SIZE"]["per_launch"], res["WRITE_SIZE"]["per_launch"]
    extra = ""
    if args is not None:
        extra = (f" --workload {workload} --path {args.path} --truncation {args.truncation}")
    out = {"kernel": "lq_kernel", "workload": workload,
           "bytes_per_launch": (sum(fetch) + sum(write)) / len(fetch),
           "fetch_bytes_per_level": fetch, "write_bytes_per_level": write,
           "fetch_scale": res["FETCH_SIZE"]["scale"], "write_scale": res["WRITE_SIZE"]["scale"],
           "calibration": f"elementwise copy of {mib} MiB: FETCH_SIZE reads {res['FETCH_SIZE']['copy_kib']:.0f} KiB, "
                          f"WRITE_SIZE {res['WRITE_SIZE']['copy_kib']:.0f} KiB per dispatch",
           "source_digest": _side_digest(),
           "command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -f csv -d <dir> -o run -- python3 -u bench.py "
                      f"--steps 3 --warmup 1 --no-cpu-baseline --copy-probe {mib}" + extra}
    if dst is None:
        dst = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"lq_kernel_{workload}_traffic.json")
    with open(dst, "w") as fh:
        json.dump(out, fh, indent=1)
    log(f"wrote {dst}: {out['bytes_per_launch'] / 1e6:.1f} MB per lq launch")
    return out


def trace_summary(db_path, workload, sweeps=3):
    """Markdown summary of a rocprofv3 kernel trace (its SQLite results
    file) of bench.py on `workload`: kernel statistics of the whole run, and
    the steady-state QR kernel launches (non-root launches of the last
    `sweeps` sweeps, the launches bench.py's `roofline` time covers)."""
    import collections
    import re
    import sqlite3

    con = sqlite3.connect(db_path)
    rows = con.execute("select name, duration, grid_x, grid_y, grid_z, workgroup_x from kernels order by start").fetchall()
    tot = collections.OrderedDict()
    for name, dur, *_ in rows:
        short = name.replace("(anonymous namespace)::", "").replace("hbs::", "").split("(")[0][:90]
        c, t = tot.get(short, (0, 0))
        tot[short] = (c + 1, t + dur)
    allns = sum(t for _, t in tot.values())
    out = ["| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for name, (c, t) in sorted(tot.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| {name} | {c} | {t / c / 1e3:.1f} | {t / 1e6:.2f} | {100 * t / allns:.1f} |")
    roots = lq_launch_roots(workload)
    lq = [r for r in rows if "lq_kernel" in r[0]][-sweeps * len(roots):]
    steady = [r[1] for i, r in enumerate(lq) if not roots[i % len(roots)]]
    out.append("")
    out.append(f"Steady-state `lq_kernel`: {len(steady)} non-root launches of the last {sweeps} sweeps, "
               f"average {sum(steady) / len(steady) / 1e3:.1f} us, {sum(steady) / sweeps / 1e6:.3f} ms per sweep.")
    # every sweep kernel of the last `sweeps` sweeps, by step of the sweep
    # (a step starts at its QR-kernel launch)
    kinds = ("lq_kernel", "col_kernel", "tail_a", "tail_b", "tail_c")  # tail_b has two kernels
    sw = [r for r in rows if any(k in r[0] for k in kinds)]
    first = next(i for i in range(len(sw)) if sw[i] is lq[0])
    per_step = collections.defaultdict(lambda: collections.defaultdict(list))
    boxes = {}
    step = -1
    for name, dur, gx, gy, gz, wx in sw[first:]:
        kind = next(k for k in kinds if k in name)
        if kind == "lq_kernel":
            step += 1
        if step >= sweeps * len(roots):
            break
        st = step % len(roots)
        if kind == "lq_kernel":
            boxes[st] = gx // max(wx, 1)
        targs = re.search(r"col_kernel<([^>]*)>", name)
        if targs and targs.group(1).replace(" ", "").split(",")[-1] == "2":
            kind = "col_kernel (Jacobi)"
        per_step[st][kind].append(dur)
    cols = ["lq_kernel", "col_kernel", "col_kernel (Jacobi)", "tail_a", "tail_b", "tail_c"]
    cols = [c for c in cols if any(c in d for d in per_step.values())]
    out.append("")
    out.append(f"Per step of the sweep (average over the last {sweeps} sweeps, us; a step is one aligned level "
               f"of one (k, s) class; boxes from the QR kernel's grid):")
    out.append("")
    out.append("| step | boxes | root | " + " | ".join(c.replace("_kernel", "") for c in cols) + " | sum |")
    out.append("|---|---|---|" + "---|" * (len(cols) + 1))
    tot = collections.defaultdict(float)
    for st in sorted(per_step):
        d = per_step[st]
        vals = [sum(d[c]) / sweeps / 1e3 if c in d else 0.0 for c in cols]
        for c, v in zip(cols, vals):
            tot[c] += v
        out.append(f"| {st} | {boxes.get(st, '')} | {'yes' if roots[st] else ''} | "
                   + " | ".join(f"{v:.1f}" if v else "" for v in vals) + f" | {sum(vals):.1f} |")
    out.append("| all | | | " + " | ".join(f"{tot[c]:.1f}" for c in cols) + f" | {sum(tot.values()):.1f} |")
    return "\n".join(out)


def counter_summary(csv_path):
    """Markdown table of a rocprofv3 --pmc counter file: per kernel name,
    dispatches and the mean of each counter per dispatch."""
    import collections
    import csv

    acc = collections.OrderedDict()
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            kname = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("hbs::", "")
            key = (kname.split("(")[0][:80], r["Counter_Name"])
            n, v, ids = acc.get(key, (0, 0.0, set()))
            ids.add(r["Dispatch_Id"])
            acc[key] = (n + 1, v + float(r["Counter_Value"]), ids)
    names = sorted({k[1] for k in acc})
    kern = list(dict.fromkeys(k[0] for k in acc))
    out = ["| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for kname in kern:
        cells, nd = [], 0
        for c in names:
            n, v, ids = acc.get((kname, c), (0, 0.0, set()))
            nd = max(nd, len(ids))
            cells.append(f"{v / max(len(ids), 1):.4g}" if ids else "")
        out.append(f"| {kname} | {nd} | " + " | ".join(cells) + " |")
    return "\n".join(out)


def inputs_workloads():
    import inputs
    return inputs.WORKLOADS


def _side_digest():
    """Digest of the QR kernel's source: hbs_side.hip up to the column
    kernel's section (the shared helpers, LqCore and lq_kernel), so that a
    change to the column kernel alone keeps the traffic file valid."""
    import hashlib
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2205_02990_amd", "csrc", "hbs_side.hip")
    with open(p, "rb") as fh:
        text = fh.read()
    end = text.find(b"// col kernel:")
    return hashlib.sha256(text if end < 0 else text[:end]).hexdigest()[:16]


if __name__ == "__main__":
    main()
