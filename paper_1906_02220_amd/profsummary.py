"""Summaries of rocprofv3 output for the kernel-time and HBM-traffic tables.

    python -m paper_1906_02220_amd.profsummary kernels RUN_results.db [TOP]
        Kernel-time table from a `rocprofv3 --kernel-trace --stats` database
        (name, calls, total ms, average us, share of GPU time).

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


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("top", nargs="?", type=int, default=25)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--source", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "kernels":
        kernels(a.db, a.top)
    else:
        traffic(a)


if __name__ == "__main__":
    main(sys.argv[1:])
