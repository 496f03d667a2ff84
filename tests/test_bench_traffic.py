"""Host logic of bench.py's counter summary (--traffic-from): the copy-probe
calibration, the per-level averaging over the last six sweeps and the
exclusion of each sweep's root launch, on synthetic counter files."""
import csv
import json
import os

import pytest

import bench


@pytest.fixture(autouse=True)
def _library():
    # the workload's level count comes from the library's own tree (host code)
    from paper_2205_02990_amd import hbs
    if not os.path.exists(hbs.LIB_PATH):
        pytest.skip("libhbs.so not built (run python -m paper_2205_02990_amd.build)")

FIELDS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_counters(path, name, copy_kib, sweeps, per, value):
    """One copy-probe dispatch, then `sweeps` sweeps of `per` lq launches
    (levels, then the root) whose counter reads value(sweep, launch) KiB."""
    rows = [dict(Kernel_Name="void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<double>>",
                 Counter_Name=name, Counter_Value=copy_kib)]
    rows.append(dict(Kernel_Name="other_kernel", Counter_Name=name, Counter_Value=12345.0))
    for sw in range(sweeps):
        for j in range(per):
            rows.append(dict(Kernel_Name=f"void hbs::lq_kernel<256, 4, 1, 1, 16, 0>(hbs::SweepArgs)",
                             Counter_Name=name, Counter_Value=value(sw, j)))
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, r in enumerate(rows):
            w.writerow(dict(Correlation_Id=i, Dispatch_Id=i, **r))


@pytest.mark.parametrize("mib", [512, 64])
def test_traffic_summary(tmp_path, mib):
    wl = "hbs_exact_n1024_k16"  # 5 levels below the root: 6 lq launches per sweep
    per = 6
    # FETCH reads half the copy's bytes (scale 2), WRITE all of them (scale 1)
    f_csv, w_csv = tmp_path / "fetch.csv", tmp_path / "write.csv"
    # 8 sweeps: the first two (tuning, warm-up) must not count
    write_counters(f_csv, "FETCH_SIZE", mib * 1024 / 2, 8, per,
                   lambda sw, j: 1e9 if sw < 2 else 100.0 * (j + 1) + (999.0 if j == per - 1 else 0.0))
    write_counters(w_csv, "WRITE_SIZE", mib * 1024, 8, per,
                   lambda sw, j: 1e9 if sw < 2 else 10.0 * (j + 1) + sw)
    dst = tmp_path / "traffic.json"
    out = bench.traffic_from_counters(str(f_csv), str(w_csv), mib, wl, dst=str(dst))
    assert json.loads(dst.read_text()) == out
    assert out["fetch_scale"] == pytest.approx(2.0) and out["write_scale"] == pytest.approx(1.0)
    fetch = [2 * 100.0 * (j + 1) * 1024 for j in range(per - 1)]
    mean_sw = sum(range(2, 8)) / 6
    write = [(10.0 * (j + 1) + mean_sw) * 1024 for j in range(per - 1)]
    assert out["fetch_bytes_per_level"] == pytest.approx(fetch)
    assert out["write_bytes_per_level"] == pytest.approx(write)
    assert out["bytes_per_launch"] == pytest.approx((sum(fetch) + sum(write)) / (per - 1))
    assert out["source_digest"] == bench._side_digest()


def test_traffic_summary_needs_the_copy_probe(tmp_path):
    f_csv = tmp_path / "f.csv"
    with open(f_csv, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        w.writerow(dict(Correlation_Id=0, Dispatch_Id=0, Kernel_Name="void hbs::lq_kernel<>", Counter_Name="FETCH_SIZE",
                        Counter_Value=1.0))
    with pytest.raises(SystemExit):
        bench.traffic_from_counters(str(f_csv), str(f_csv), 512, "hbs_exact_n1024_k16", dst=str(tmp_path / "t.json"))


def test_trace_summary_per_step(tmp_path):
    """bench.py --trace-summary on a synthetic rocpd kernels table: the
    per-step table of the last sweeps averages each kernel's duration by step
    of the sweep, tells the Jacobi pass of col apart, and leaves out the
    tuning launches and everything after the last sweep."""
    import sqlite3

    wl = "hbs_exact_n1024_k16"  # 5 levels below the root, then the root
    per = 6
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration int, grid_x int, grid_y int, grid_z int, "
                "workgroup_x int, start int)")
    rows = []

    def launch(name, dur, boxes=1):
        rows.append((name, dur, boxes * 256, 2, 1, 256, len(rows)))

    lq = "void hbs::(anonymous namespace)::lq_kernel<256, 4, 1, 1, 16, 0>(hbs::SweepArgs)"
    col1 = "void hbs::(anonymous namespace)::col_kernel<256, 4, 1, 8, 0, 1>(hbs::SweepArgs)"
    col2 = "void hbs::(anonymous namespace)::col_kernel<256, 4, 1, 8, 0, 2>(hbs::SweepArgs)"
    for sw in range(5):  # sweeps 0 and 1 are tuning / warm-up with other durations
        for j in range(per):
            scale = 1000 if sw < 2 else 1
            launch(lq, scale * (1000 * (j + 1) + 1000 * sw), boxes=2 ** (per - 1 - j))
            if j == per - 1:
                break
            launch(col1, scale * 2000)
            launch(col2, scale * 300)
            for t in ("tail_a_kernel", "tail_b_small_kernel", "tail_c_kernel<0, 2>"):
                launch(f"void hbs::(anonymous namespace)::{t}(hbs::SweepArgs)", scale * 500)
    launch("apply_up_kernel", 10 ** 9)  # after the sweeps: not part of any step
    con.executemany("insert into kernels values (?, ?, ?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    md = bench.trace_summary(str(db), wl, sweeps=3)
    table = md.split("Per step of the sweep")[1].splitlines()
    head = [c.strip() for c in table[2].split("|")[1:-1]]
    assert head == ["step", "boxes", "root", "lq", "col", "col (Jacobi)", "tail_a", "tail_b", "tail_c", "sum"]
    body = [[c.strip() for c in ln.split("|")[1:-1]] for ln in table[4:4 + per]]
    for j, r in enumerate(body):
        assert int(r[0]) == j and int(r[1]) == 2 ** (per - 1 - j)
        assert (r[2] == "yes") == (j == per - 1)
        assert float(r[3]) == pytest.approx((1000 * (j + 1) + 1000 * 3) / 1e3)  # mean of sweeps 2, 3, 4
        if j < per - 1:
            assert [float(x) for x in r[4:9]] == pytest.approx([2.0, 0.3, 0.5, 0.5, 0.5])
        else:
            assert r[4:9] == [""] * 5


def test_counter_summary_means_per_dispatch(tmp_path):
    """bench.py --counter-summary: per kernel name (template arguments kept,
    namespaces dropped), the number of dispatches and the mean of each counter
    per dispatch."""
    path = tmp_path / "counters.csv"
    rows = []
    for d, (kern, vals) in enumerate([
            ("void hbs::(anonymous namespace)::tail_c_kernel<8, 1>(hbs::SweepArgs)", {"SQ_INSTS_VALU": 10.0, "SQ_BUSY_CU_CYCLES": 4.0}),
            ("void hbs::(anonymous namespace)::tail_c_kernel<8, 1>(hbs::SweepArgs)", {"SQ_INSTS_VALU": 30.0, "SQ_BUSY_CU_CYCLES": 8.0}),
            ("hbs::(anonymous namespace)::tail_a_kernel(hbs::SweepArgs)", {"SQ_INSTS_VALU": 5.0})]):
        for name, v in vals.items():
            rows.append(dict(Correlation_Id=d, Dispatch_Id=d, Kernel_Name=kern, Counter_Name=name, Counter_Value=v))
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        w.writerows(rows)
    md = bench.counter_summary(str(path)).splitlines()
    assert md[0] == "| kernel | dispatches | SQ_BUSY_CU_CYCLES | SQ_INSTS_VALU |"
    body = {ln.split("|")[1].strip(): [c.strip() for c in ln.split("|")[2:-1]] for ln in md[2:]}
    assert body["void tail_c_kernel<8, 1>"] == ["2", "6", "20"]
    assert body["tail_a_kernel"] == ["1", "", "5"]


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says why,
    before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
