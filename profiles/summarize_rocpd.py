"""Print a kernel-time table from a rocprofv3 results database (rocpd SQLite).

Usage: python profiles/summarize_rocpd.py <run_results.db> [top]
Reads the `top_kernels` view that rocprofv3 writes and prints name, calls,
total duration (ms), average duration (us) and share of GPU time.
"""
import sqlite3
import sys


def main(path, top=25):
    c = sqlite3.connect(path)
    rows = c.execute("select name, total_calls, total_duration, average, percentage "
                     "from top_kernels limit ?", (top,)).fetchall()
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows:
        short = name.replace("(anonymous namespace)::", "").split("(")[0]
        print("| %s | %d | %.2f | %.2f | %.2f |" % (short, calls, tot / 1e3, avg, pct))


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 25)
