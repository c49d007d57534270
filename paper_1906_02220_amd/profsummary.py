"""Summaries of rocprofv3 output for the kernel-time and HBM-traffic tables.

    python -m paper_1906_02220_amd.profsummary kernels RUN_results.db [TOP]
        Kernel-time table from a `rocprofv3 --kernel-trace --stats` database
        (name, calls, total ms, average us, share of GPU time).

    python -m paper_1906_02220_amd.profsummary permove SHORT.db LONG.db MOVES [TOP]
        Steady-state cost per move: per kernel, the calls and GPU time of the
        LONG trace minus those of the SHORT one (two runs that differ only in
        the number of sweeps), divided by the MOVES the LONG run adds.

    python -m paper_1906_02220_amd.profsummary traffic --kernel SUBSTR \\
            --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \\
            --copy-bytes N --source FILE
        HBM bytes per launch of the kernels whose name contains SUBSTR, from
        two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs (KiB per
        dispatch, CSV output).  Each counter is scaled by the ratio of the
        true size of a plain device copy (N bytes read and written) to what
        the same counter reads for that copy.  Prints 'key: value' lines,
        including a hash of the kernel source so that a reader can tell
        whether the figures still apply.

    python -m paper_1906_02220_amd.profsummary mfma --kernel SUBSTR \
            --counters C1.csv [C2.csv ...] [--simds 1024] [--xcds 8] [--us US]
        Matrix-core use of the kernels whose name contains SUBSTR, from
        `rocprofv3 --pmc` runs (CSV output) holding SQ_VALU_MFMA_BUSY_CYCLES,
        GRBM_GUI_ACTIVE and SQ_INSTS_VALU_MFMA_MOPS_<type>: per dispatch, the
        busy fraction busy / ((gui_active / xcds) x simds) (GRBM_GUI_ACTIVE is
        summed over the XCDs, the busy cycles over every SIMD of the chip:
        1024 on MI355X) and the MFMA work the
        hardware counted (512 flop per MOPS unit); with --us (the kernel's
        average duration from a kernel trace) also the rate of that work.
        Prints 'key: value' lines of the medians over the dispatches.
"""
import argparse
import csv
import hashlib
import sqlite3
import statistics
import sys


def kernels(db, top=25):
    c = sqlite3.connect(db)
    rows = c.execute("select name, total_calls, total_duration, average, percentage "
                     "from top_kernels limit ?", (top,)).fetchall()
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows:
        short = name.replace("(anonymous namespace)::", "").split("(")[0]
        print("| %s | %d | %.2f | %.2f | %.2f |" % (short, calls, tot / 1e3, avg, pct))


def _per_kernel(db):
    c = sqlite3.connect(db)
    return {name: (calls, ns) for name, calls, ns in
            c.execute("select name, count(*), sum(end - start) from kernels group by name")}


def permove(short_db, long_db, moves, top=25):
    a, b = _per_kernel(short_db), _per_kernel(long_db)
    rows = []
    for name, (cb, tb) in b.items():
        ca, ta = a.get(name, (0, 0))
        if cb > ca:
            rows.append(((tb - ta) / moves / 1e3, (cb - ca) / moves, name))
    rows.sort(reverse=True)
    total = sum(r[0] for r in rows)
    print("| kernel | calls per move | us per move | % |")
    print("|---|---|---|---|")
    for us, calls, name in rows[:top]:
        short = name.replace("(anonymous namespace)::", "").split("(")[0]
        print("| %s | %.2f | %.1f | %.1f |" % (short, calls, us, 100.0 * us / total))
    print("| total | | %.1f | 100.0 |" % total)


def _values(path, substr=None, largest_grid=False):
    rows = list(csv.DictReader(open(path)))
    if substr is not None:
        rows = [r for r in rows if substr in r["Kernel_Name"]]
    if largest_grid:
        rows = [r for r in rows if "copy" in r["Kernel_Name"].lower()]
        g = max(int(r["Grid_Size"]) for r in rows)
        rows = [r for r in rows if int(r["Grid_Size"]) == g]
    return [float(r["Counter_Value"]) for r in rows]


def traffic(a):
    kib = 1024.0
    cf = statistics.median(_values(a.copy_fetch, largest_grid=True))
    cw = statistics.median(_values(a.copy_write, largest_grid=True))
    f_fetch = a.copy_bytes / (cf * kib)
    f_write = a.copy_bytes / (cw * kib)
    fv = _values(a.fetch, a.kernel)
    wv = _values(a.write, a.kernel)
    fetch_b = statistics.median(fv) * kib * f_fetch
    write_b = statistics.median(wv) * kib * f_write
    with open(a.source, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    print("kernel: %s" % a.kernel)
    print("dispatches: %d fetch, %d write" % (len(fv), len(wv)))
    print("copy_fetch_kib: %.1f" % cf)
    print("copy_write_kib: %.1f" % cw)
    print("fetch_scale: %.5f" % f_fetch)
    print("write_scale: %.5f" % f_write)
    print("fetch_kib_median_raw: %.1f" % statistics.median(fv))
    print("write_kib_median_raw: %.1f" % statistics.median(wv))
    print("hbm_fetch_bytes_per_launch: %.0f" % fetch_b)
    print("hbm_write_bytes_per_launch: %.0f" % write_b)
    print("hbm_bytes_per_launch: %.0f" % (fetch_b + write_b))
    print("gemm_source_sha256_16: %s" % h)


def mfma(a):
    per = {}  # (file, dispatch) -> {counter: value}
    for fi, path in enumerate(a.counters):
        for r in csv.DictReader(open(path)):
            if a.kernel not in r["Kernel_Name"]:
                continue
            key = (fi, r.get("Dispatch_Id") or r.get("Correlation_Id"))
            per.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    names = sorted({n for d in per.values() for n in d})
    print("kernel: %s" % a.kernel)
    print("dispatches: %d" % len(per))
    for n in names:
        vals = [d[n] for d in per.values() if n in d]
        print("%s_median: %.6g" % (n, statistics.median(vals)))
    busy = [d["SQ_VALU_MFMA_BUSY_CYCLES"] / (d["GRBM_GUI_ACTIVE"] / a.xcds * a.simds)
            for d in per.values()
            if "SQ_VALU_MFMA_BUSY_CYCLES" in d and d.get("GRBM_GUI_ACTIVE", 0) > 0]
    if busy:
        print("mfma_busy_fraction: %.4f" % statistics.median(busy))
    for n in names:
        if n.startswith("SQ_INSTS_VALU_MFMA_MOPS_"):
            flops = statistics.median([d[n] for d in per.values() if n in d]) * 512.0
            if flops <= 0:
                continue
            t = n[len("SQ_INSTS_VALU_MFMA_MOPS_"):]
            print("mfma_flop_per_dispatch_%s: %.6g" % (t, flops))
            if a.us:
                print("mfma_tflops_%s: %.5g" % (t, flops / (a.us * 1e-6) / 1e12))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("top", nargs="?", type=int, default=25)
    pm = sub.add_parser("permove")
    pm.add_argument("short_db")
    pm.add_argument("long_db")
    pm.add_argument("moves", type=int)
    pm.add_argument("top", nargs="?", type=int, default=25)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--source", required=True)
    m = sub.add_parser("mfma")
    m.add_argument("--kernel", required=True)
    m.add_argument("--counters", nargs="+", required=True)
    m.add_argument("--simds", type=int, default=1024)
    m.add_argument("--xcds", type=int, default=8)
    m.add_argument("--us", type=float, default=0.0)
    a = ap.parse_args(argv)
    if a.cmd == "kernels":
        kernels(a.db, a.top)
    elif a.cmd == "permove":
        permove(a.short_db, a.long_db, a.moves, a.top)
    elif a.cmd == "traffic":
        traffic(a)
    else:
        mfma(a)


if __name__ == "__main__":
    main(sys.argv[1:])
