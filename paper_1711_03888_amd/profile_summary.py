"""Summarise rocprofv3 results databases as text, and turn HBM counter
passes into per-launch traffic.

  python -m paper_1711_03888_amd.profile_summary RESULTS_DB [COMMAND...]
      per-kernel launch counts and average durations from a kernel trace,
      per-kernel averages of any collected counters;
  python -m paper_1711_03888_amd.profile_summary --copy-probe BYTES
      a plain device-to-device copy of BYTES bytes (three launches), the
      calibration run of the FETCH_SIZE / WRITE_SIZE counters;
  python -m paper_1711_03888_amd.profile_summary --traffic FETCH_DB WRITE_DB
      COPY_FETCH_DB COPY_WRITE_DB COPY_BYTES OUT_JSON
      HBM bytes read and written per launch of every kernel: the counters
      (KiB per dispatch) scaled by bytes-per-count of the copy kernel, stamped
      with the hash of the library sources they were taken on.
"""
import collections
import glob
import hashlib
import json
import os
import sqlite3
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def source_hash():
    """sha256 over the HIP sources and headers of the library."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _short(name):
    short = name.split("(")[0].replace("void ", "").replace("sznb::", "")
    if "at::native" in short:
        short = "torch:" + short.split("<")[0].split("::")[-1]
    return short


def counter_per_dispatch(path, counter):
    """{kernel: [value per dispatch]} of one counter."""
    db = sqlite3.connect(path)
    acc = collections.defaultdict(float)
    names = {}
    for k, c, v, d in db.execute("select kernel_name, counter_name, value, dispatch_id from counters_collection"):
        if c == counter:
            acc[d] += v
            names[d] = _short(k)
    out = collections.defaultdict(list)
    for d in sorted(acc):
        out[names[d]].append(acc[d])
    return out


def traffic(fetch_db, write_db, copy_fetch_db, copy_write_db, copy_bytes):
    cf = counter_per_dispatch(copy_fetch_db, "FETCH_SIZE")
    cw = counter_per_dispatch(copy_write_db, "WRITE_SIZE")
    ck = max(cf, key=lambda k: sum(cf[k]))  # the copy kernel
    f_scale = copy_bytes / (sum(cf[ck]) / len(cf[ck]))
    w_scale = copy_bytes / (sum(cw[ck]) / len(cw[ck]))
    fe = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    wr = counter_per_dispatch(write_db, "WRITE_SIZE")
    kern = {}
    for k in sorted(set(fe) | set(wr)):
        r = sum(fe.get(k, [0])) / max(1, len(fe.get(k, [])))
        w = sum(wr.get(k, [0])) / max(1, len(wr.get(k, [])))
        kern[k] = {"read_bytes": r * f_scale, "write_bytes": w * w_scale, "bytes": r * f_scale + w * w_scale,
                   "dispatches": len(fe.get(k, []))}
    return {"source_sha256": source_hash(), "copy_kernel": ck, "copy_bytes": copy_bytes,
            "fetch_bytes_per_count": f_scale, "write_bytes_per_count": w_scale, "kernels": kern}


def copy_probe(nbytes):
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes three times" % nbytes)


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
                short = _short(name)
                lines.append("%-28s %6d %12.4f %12.4f %7.2f" % (short[:28], calls, tot / 1e3, avg / 1e3, pct))
    if "counters_collection" in tables:
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        disp = collections.defaultdict(set)
        for k, c, v, d in cur.execute("select kernel_name, counter_name, value, dispatch_id from counters_collection"):
            short = _short(k)
            agg[short][c] += v
            disp[short].add(d)
        for k in sorted(agg):
            n = len(disp[k])
            lines.append("%s (%d dispatches): %s" % (k, n, ", ".join("%s=%.0f" % (c, v / n) for c, v in sorted(agg[k].items()))))
    return "\n".join(lines)


if __name__ == "__main__":
    if sys.argv[1] == "--copy-probe":
        copy_probe(int(sys.argv[2]))
    elif sys.argv[1] == "--traffic":
        t = traffic(*sys.argv[2:6], int(sys.argv[6]))
        with open(sys.argv[7], "w") as f:
            json.dump(t, f, indent=1, sort_keys=True)
        for k, v in t["kernels"].items():
            print("%-24s read %14.0f  write %14.0f bytes per launch" % (k, v["read_bytes"], v["write_bytes"]))
    else:
        print(summarize(sys.argv[1], " ".join(sys.argv[2:])))
