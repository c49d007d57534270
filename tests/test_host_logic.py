"""Host-side logic of the benchmark and of the profile summaries (no GPU).

* the algorithmic work per absorption move that the benchmark's headline
  divides by: W = 5 chi^2 d^4 + 3 chi^3 d^3 + 8 chi^3 d^2 + 6 chi^3 d
  multiply-adds, 1.995e11 flop at D = 6, chi = 72 (d = 36);
* the traffic reader, which must hand out the stored HBM bytes only while the
  kernel source still hashes to the value recorded with them;
* the counter scaling of the traffic summary on a synthetic counter file;
* the refusal of a multi-GPU run.
"""
import csv
import io
import os
import subprocess
import sys
from contextlib import redirect_stdout

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1906_02220_amd import profsummary  # noqa: E402


def test_algorithmic_work_per_move():
    chi, d = 72, 36
    w = 5 * chi**2 * d**4 + 3 * chi**3 * d**3 + 8 * chi**3 * d**2 + 6 * chi**3 * d
    assert bench.move_macs(chi, d) == pytest.approx(w, rel=0, abs=0.5)
    assert 2.0 * bench.move_macs(chi, d) == pytest.approx(1.995e11, rel=1e-3)


def test_traffic_is_reported_only_for_the_recorded_kernel_source(tmp_path, monkeypatch):
    src_dir = tmp_path / "paper_1906_02220_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (src_dir / "gemm_f64.hip").write_text("kernel source, version 1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.kernel_source_hash("gemm_f64.hip")
    (tmp_path / "profiles" / "traffic_dgemm_rr_cut_D6_chi72.txt").write_text(
        "# comment: with a colon\nkernel: dgemm_rr\nhbm_bytes_per_launch: 474028539\n"
        "gemm_source_sha256_16: %s\n" % h)
    assert bench.read_traffic(0) == 474028539
    assert bench.read_traffic(1) is None  # no summary for the FP32 mode
    (src_dir / "gemm_f64.hip").write_text("kernel source, version 2\n")
    assert bench.read_traffic(0) is None


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scales_counters_by_the_copy(tmp_path):
    copy_bytes = 1 << 20
    # the copy kernel's counter reads half the true bytes for FETCH, all of
    # them for WRITE; a smaller copy grid must be ignored
    _counter_csv(tmp_path / "cf.csv", [
        {"Kernel_Name": "copyBuffer", "Grid_Size": 4096, "Counter_Value": 512.0},
        {"Kernel_Name": "copyBuffer", "Grid_Size": 64, "Counter_Value": 1.0}])
    _counter_csv(tmp_path / "cw.csv", [
        {"Kernel_Name": "copyBuffer", "Grid_Size": 4096, "Counter_Value": 1024.0}])
    _counter_csv(tmp_path / "f.csv", [
        {"Kernel_Name": "gemm_x<3>", "Grid_Size": 1, "Counter_Value": v} for v in (100.0, 300.0, 200.0)]
        + [{"Kernel_Name": "other", "Grid_Size": 1, "Counter_Value": 9e9}])
    _counter_csv(tmp_path / "w.csv", [
        {"Kernel_Name": "gemm_x<3>", "Grid_Size": 1, "Counter_Value": 50.0}])
    src = tmp_path / "k.hip"
    src.write_text("x")
    buf = io.StringIO()
    with redirect_stdout(buf):
        profsummary.main(["traffic", "--kernel", "gemm_x", "--fetch", str(tmp_path / "f.csv"),
                          "--write", str(tmp_path / "w.csv"), "--copy-fetch", str(tmp_path / "cf.csv"),
                          "--copy-write", str(tmp_path / "cw.csv"), "--copy-bytes", str(copy_bytes),
                          "--source", str(src)])
    kv = dict(line.split(": ", 1) for line in buf.getvalue().splitlines())
    assert float(kv["fetch_scale"]) == pytest.approx(2.0)
    assert float(kv["write_scale"]) == pytest.approx(1.0)
    assert kv["dispatches"] == "3 fetch, 1 write"
    assert float(kv["hbm_fetch_bytes_per_launch"]) == pytest.approx(200.0 * 1024 * 2.0)
    assert float(kv["hbm_bytes_per_launch"]) == pytest.approx(200.0 * 1024 * 2.0 + 50.0 * 1024)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_runs_the_moves_it_divides_by(monkeypatch):
    """The oracle sample runs exactly `moves` moves, cycling L, R, U, D, and
    the rate divides the work of those moves (not of more) by their time."""
    from oracle import ctmrg as O
    calls = []
    real = O.left_move

    def counted(env, arot, k, chi, *a, **kw):
        calls.append(k)
        return real(env, arot, k, chi, *a, **kw)

    monkeypatch.setattr(O, "left_move", counted)
    assert bench.cpu_baseline_order(6) == [0, 2, 1, 3, 0, 2]
    res = bench.cpu_baseline(2, 4, 1, moves=10)
    assert calls == [0, 2, 1, 3, 0, 2, 1, 3, 0, 2]
    assert res["moves"] == 10 and res["sample"].startswith("10 absorption moves")
    rate = 10 * 2.0 * bench.move_macs(4, 4) / res["seconds"] / 1e9
    assert res["value"] == pytest.approx(rate, rel=0.02)


def test_headline_needs_the_bound_on_both_workloads():
    """A mode heads the line only if kappa stays within the bound on the
    random and the structured workload and <H_bond> on the random one."""
    def r(ms, ek, ee):
        return {"ms_per_move": ms, "err_kappa_vs_fp64": ek, "err_energy_vs_fp64": ee}
    runs = {0: r(6.0, 0.0, 0.0), 1: r(5.0, 1e-11, 3e-8), 3: r(4.0, 1e-12, 2e-9),
            4: r(4.5, 1e-12, 3e-9)}
    st = {"_errs": {0: (0.0, 0.0), 1: (2e-10, 2e-6), 3: (2e-12, 5e-6), 4: (1e-12, 8e-8)}}
    assert bench.select_headline(runs, st)[:2] == (3, 1e-8)
    st["_errs"][3] = (2e-8, 5e-6)          # bf16x3 kappa off on the structured case
    assert bench.select_headline(runs, st)[:2] == (4, 1e-8)
    runs[4]["err_energy_vs_fp64"] = 5e-8   # bf16x4 <H> off on the random case
    assert bench.select_headline(runs, st)[:2] == (3, 1e-7)
    assert bench.select_headline(runs, None)[:2] == (3, 1e-8)
    for m in (1, 3, 4):
        runs[m]["err_kappa_vs_fp64"] = 1e-6
    assert bench.select_headline(runs, st)[:2] == (0, 0.0)


def test_mfma_summary_from_counters(tmp_path):
    """Busy fraction = busy / ((gui_active / xcds) x simds) and 512 flop per
    MOPS unit, medians over the dispatches of the named kernel only."""
    path = tmp_path / "c.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for disp, busy, gui, mops in ((1, 512.0, 8.0, 100.0), (2, 256.0, 8.0, 300.0), (3, 768.0, 8.0, 200.0)):
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": "gemm_x<3>", "Counter_Name": "SQ_VALU_MFMA_BUSY_CYCLES", "Counter_Value": busy})
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": "gemm_x<3>", "Counter_Name": "GRBM_GUI_ACTIVE", "Counter_Value": gui})
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": "gemm_x<3>", "Counter_Name": "SQ_INSTS_VALU_MFMA_MOPS_BF16", "Counter_Value": mops})
        w.writerow({"Dispatch_Id": 9, "Kernel_Name": "other", "Counter_Name": "SQ_VALU_MFMA_BUSY_CYCLES", "Counter_Value": 1e9})
    buf = io.StringIO()
    with redirect_stdout(buf):
        profsummary.main(["mfma", "--kernel", "gemm_x", "--counters", str(path), "--simds", "1024", "--xcds", "8",
                          "--us", "2.0"])
    kv = dict(line.split(": ", 1) for line in buf.getvalue().splitlines())
    assert kv["dispatches"] == "3"
    assert float(kv["mfma_busy_fraction"]) == pytest.approx(0.5)
    assert float(kv["mfma_flop_per_dispatch_BF16"]) == pytest.approx(200.0 * 512)
    assert float(kv["mfma_tflops_BF16"]) == pytest.approx(200.0 * 512 / 2e-6 / 1e12)


def test_per_move_table_is_the_difference_of_two_traces(tmp_path):
    import sqlite3
    def db(path, rows):
        c = sqlite3.connect(path)
        c.execute("create table kernels (name text, start integer, end integer)")
        c.executemany("insert into kernels values (?, ?, ?)", rows)
        c.commit()
        c.close()
    # the short run: 2 x k1 (1 us each), 1 x setup; the long run adds 4 moves
    # with 2 x k1 (1 us) and 1 x k2 (3 us) each
    db(tmp_path / "a.db", [("k1(int)", 0, 1000), ("k1(int)", 0, 1000), ("setup(int)", 0, 50000)])
    db(tmp_path / "b.db", [("k1(int)", 0, 1000)] * 10 + [("k2(int)", 0, 3000)] * 4 + [("setup(int)", 0, 50000)])
    buf = io.StringIO()
    with redirect_stdout(buf):
        profsummary.main(["permove", str(tmp_path / "a.db"), str(tmp_path / "b.db"), "4"])
    lines = {l.split("|")[1].strip(): l.split("|")[2:4] for l in buf.getvalue().splitlines()[2:]}
    assert float(lines["k2"][0]) == pytest.approx(1.0) and float(lines["k2"][1]) == pytest.approx(3.0)
    assert float(lines["k1"][0]) == pytest.approx(2.0) and float(lines["k1"][1]) == pytest.approx(2.0)
    assert "setup" not in lines
    assert float(lines["total"][1]) == pytest.approx(5.0)


def test_small_per_mode_figures_keep_their_digits():
    """Errors and self-changes far below 1e-6 are reported to 4 significant
    digits, not rounded to 0 by a fixed number of decimals."""
    assert bench._fmt("self_change_kappa", 2.1e-13) == pytest.approx(2.1e-13)
    assert bench._fmt("err_energy_vs_fp64", 2.716777e-09) == 2.717e-09
    assert bench._fmt("ms_per_move", 3.45292412) == 3.452924
    assert bench._fmt("kappa", 15.547744270432997) == 15.547744270432997
    assert bench._fmt("launches", 120) == 120
