"""The counter/trace summariser of bench.py (--profile-summary) on synthetic
rocprofv3 CSV output: what it reads from kernel names and launch sizes, the
copy-kernel scaling of FETCH_SIZE / WRITE_SIZE, and the table rows that the
benchmark's traffic lookup parses.  No GPU."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

DIMS = (8, 8, 8, 8)
VH = 8 ** 4 // 2
RLOOP = ("void wd::dslash16_rloop_kernel<false, false, 0, 1, false, wd::SF16>(wd::DslashGeom, char const*, "
         "wd::FieldView, wd::FieldView, wd::FieldView, wd::FieldView, float, int, int const*, double*, wd::EncView)")
FP64_RES = ("void wd::dslash_kernel<wd::SF64, false, true, 5, 3, 12, false, 1, wd::SF16>(wd::DslashGeom, char const*, "
            "wd::FieldView, wd::FieldView, wd::FieldView, wd::FieldView, wd::SF64::real, int, int const*, double*, "
            "wd::EncView)")
COPY = "void at::native::elementwise_kernel<128, 4, direct_copy_kernel_cuda>(int)"


def test_launch_description_from_template_arguments():
    d = bench.dslash_launch(RLOOP, 2048, 256, VH, True)
    assert (d["prec"], d["form"], d["basis"], d["kind"], d["nrhs"], d["lds"]) == \
        ("f16", "D", "UKQCD", "rhs loop", None, False)
    # FP64 three-slot x + aD with the re-encoded residual, 4 RHS groups of 256-thread blocks
    per_group = 8 * -(-(VH // 8) // 256) * 256
    d = bench.dslash_launch(FP64_RES, 4 * per_group, 256, VH, True)
    assert (d["prec"], d["xpay"], d["dot"], d["kind"], d["groups"], d["nrhs"]) == ("fp64", True, 5, "3 slots", 4, 12)
    assert d["form"] == "x + a D res->enc"
    assert bench.dslash_launch(COPY, 1024, 256, VH, True) is None


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


@pytest.fixture()
def runs(tmp_path):
    copy_bytes = 4_000_000_000
    per_group = 8 * -(-(VH // 8) // 256) * 256
    trace, fetch, write = [], [], []
    did = 0
    for name, grid, f_kib, w_kib, us in [(COPY, 1 << 20, copy_bytes / 2 / 1024, copy_bytes / 1024, 900.0)] + \
            [(RLOOP, per_group, 1000.0, 400.0, 50.0 + k) for k in range(5)] + \
            [(FP64_RES, 4 * per_group, 9000.0, 800.0, 300.0)]:
        did += 1
        trace.append({"Dispatch_Id": did, "Kernel_Name": name, "Start_Timestamp": 0,
                      "End_Timestamp": int(us * 1000), "Workgroup_Size_X": 256, "Grid_Size_X": grid})
        for rows, c, v in ((fetch, "FETCH_SIZE", f_kib), (write, "WRITE_SIZE", w_kib)):
            rows.append({"Dispatch_Id": did, "Kernel_Name": name, "Grid_Size": grid, "Workgroup_Size": 256,
                         "Counter_Name": c, "Counter_Value": v})
    _write(str(tmp_path / "trace" / "run_kernel_trace.csv"), trace)
    _write(str(tmp_path / "trace" / "run_kernel_stats.csv"),
           [{"Name": RLOOP, "Calls": 5, "TotalDurationNs": 260000, "AverageNs": 52000}])
    _write(str(tmp_path / "FETCH_SIZE" / "run_counter_collection.csv"), fetch)
    _write(str(tmp_path / "WRITE_SIZE" / "run_counter_collection.csv"), write)
    return tmp_path


def _summary(path, part):
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--profile-summary", str(path),
                          "--copy-probe-gb", "4", "--dims", "x".join(map(str, DIMS)), "--profile-part", part,
                          "--dslash-reps", "3"], capture_output=True, text=True, check=True)
    return out.stdout


def test_traffic_table_scales_by_the_copy_and_labels_the_plain_batch(runs):
    text = _summary(runs, "traffic")
    assert "FETCH_SIZE x 2.000, WRITE_SIZE x 1.000" in text
    rows = [[c.strip() for c in l.strip().strip("|").split("|")] for l in text.splitlines() if l.startswith("| ")]
    body = {r[7] + " " + r[8]: r for r in rows[1:] if len(r) > 8}
    rl = body["f16 rhs loop, 256 threads D (UKQCD)"]
    assert rl[0] == "dslash_f16_12rhs"                       # the label the benchmark looks up
    assert float(rl[1]) == pytest.approx(1000.0 * 1024 * 2)  # FETCH in KiB x 1024 x copy scale
    assert float(rl[2]) == pytest.approx(400.0 * 1024)
    assert rl[3] == bench.kernel_source_hash() and rl[4] == "5"
    assert float(rl[6]) == pytest.approx(53.0)               # mean of the last 3 launches (52, 53, 54 us)
    fp = body["fp64 3 slots, 256 threads x + a D res->enc (UKQCD)"]
    assert fp[0] == "" and fp[9] == "12"                     # not a lookup label; 4 groups x 3 slots
    # reads of the re-encoding residual launch: links + input + xpay source + y
    assert float(fp[10]) == pytest.approx(VH * (8 * 96 + 12 * 192 * 3), rel=1e-4)  # printed to 5 digits


def test_trace_part_reports_the_timed_launches(runs):
    text = _summary(runs, "trace")
    line = next(l for l in text.splitlines() if l.startswith("| dslash_f16_12rhs"))
    cells = [c.strip() for c in line.strip().strip("|").split("|")]
    assert cells[4] == "3" and float(cells[5]) == pytest.approx(53.0)
    assert "Kernels by total time" in text


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True)
    assert out.returncode == 2
    line = out.stdout.strip().splitlines()[-1]
    assert "exactly one GPU" in line and '"n_gpus": 2' in line


def test_traffic_is_read_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    """bench's traffic lookup takes FETCH + WRITE of the labelled row, and
    nothing when the table was taken on another kernel source."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "dslash_traffic_48x48x48x96.md").write_text(
        "| dslash_f16_12rhs | 1.0000e+10 | 3.0000e+09 | 0000000000000000 | 5 | 1.0 | 1.0 | k | D | 12 | 4.0e9 | 2.5 |\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "1111111111111111")
    assert bench.profiled_traffic("dslash_f16_12rhs", (48, 48, 48, 96)) is None  # another source
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.profiled_traffic("dslash_f16_12rhs", (48, 48, 48, 96)) == pytest.approx(1.3e10)
    assert bench.profiled_traffic("dslash_fp64_1rhs", (48, 48, 48, 96)) is None  # no such row
