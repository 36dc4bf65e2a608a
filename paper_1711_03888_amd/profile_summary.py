"""Summarise a rocprofv3 results database (kernel trace or counters) as text.

Usage: python -m paper_1711_03888_amd.profile_summary RESULTS_DB [COMMAND...]
Prints per-kernel launch counts and average durations from the kernel
trace, and per-kernel averages of any collected counters.
"""
import collections
import sqlite3
import sys


def summarize(path, command=""):
    db = sqlite3.connect(path)
    cur = db.cursor()
    lines = ["# rocprofv3 summary of %s" % path.split("/")[-1]]
    if command:
        lines.append("# command: %s" % command)
    tables = {r[0] for r in cur.execute("select name from sqlite_master where type in ('table','view')")}
    if "top_kernels" in tables:
        rows = cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
        if rows:
            lines.append("%-28s %6s %12s %12s %7s" % ("kernel", "calls", "total_ms", "avg_ms", "pct"))
            for name, calls, tot, avg, pct in rows:
                short = name.split("(")[0].replace("void ", "").replace("sznb::", "")
                if "at::native" in short:
                    short = "torch:" + short.split("<")[0].split("::")[-1]
                lines.append("%-28s %6d %12.4f %12.4f %7.2f" % (short[:28], calls, tot / 1e3, avg / 1e3, pct))
    if "counters_collection" in tables:
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        disp = collections.defaultdict(set)
        for k, c, v, d in cur.execute("select kernel_name, counter_name, value, dispatch_id from counters_collection"):
            short = k.split("(")[0].replace("void ", "").replace("sznb::", "")
            agg[short][c] += v
            disp[short].add(d)
        for k in sorted(agg):
            n = len(disp[k])
            lines.append("%s (%d dispatches): %s" % (k, n, ", ".join("%s=%.0f" % (c, v / n) for c, v in sorted(agg[k].items()))))
    return "\n".join(lines)


if __name__ == "__main__":
    print(summarize(sys.argv[1], " ".join(sys.argv[2:])))
