"""rocprofv3 output -> the short text summaries kept under profiles/.

    python -m paper_1807_10727_amd.profiling trace  <run_results.db> <out.md> "<command>"
    python -m paper_1807_10727_amd.profiling traffic <fetch.db> <write.db> <out.json> "<command>"

`trace` summarises a `--kernel-trace --stats` run: calls, total and average duration per
kernel symbol.  `traffic` combines a `--pmc FETCH_SIZE` run and a `--pmc WRITE_SIZE` run: the
counters (KiB per dispatch) of every kernel, scaled by what the same counters read for the
plain 1 GiB device copy that bench.py performs before its timed steps, give HBM bytes per
launch.  The JSON also records a hash of the kernel sources, so a figure is dropped as soon as
a kernel changes.
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30      # the calibration copy in bench.py
COPY_SYMBOL = "__amd_rocclr_copyBuffer"


def source_hash() -> str:
    """Hash of the sources that hold device code (host-only files do not change what a
    kernel moves)."""
    h = hashlib.sha1()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        with open(p, "rb") as f:
            text = f.read()
        if b"__global__" not in text and b"__device__" not in text:
            continue
        h.update(os.path.basename(p).encode())
        h.update(text)
    return h.hexdigest()


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def kernel_stats(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration) from kernels group by name "
                       "order by sum(duration) desc").fetchall()
    return [(short(n), int(c), float(t) / 1e3, float(a) / 1e3) for (n, c, t, a) in rows]


def write_trace_md(db: str, out: str, command: str, top: int = 25):
    st = kernel_stats(db)
    total = sum(t for _, _, t, _ in st)
    lines = ["# rocprofv3 kernel trace", "", "Command (from the repository root, on one MI355X):", "",
             "    " + command, "", "| kernel | calls | total us | avg us | share |", "|---|---|---|---|---|"]
    for (n, c, t, a) in st[:top]:
        lines.append("| `%s` | %d | %.1f | %.2f | %.1f%% |" % (n, c, t, a, 100 * t / total))
    lines.append("")
    lines.append("Sum of kernel time: %.1f us over %d dispatches." % (total, sum(c for _, c, _, _ in st)))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _pmc_rows(db: str, counter: str):
    """(kernel symbol, value in KiB) for every dispatch that recorded `counter`."""
    con = sqlite3.connect(db)
    tabs = [r[0] for r in con.execute("select name from sqlite_master where type in ('table','view')")]
    if "counters_collection" in tabs:
        rows = con.execute("select kernel_name, value from counters_collection where counter_name = ?",
                           (counter,)).fetchall()
    else:   # older layout: one pmc view joined to dispatches
        rows = con.execute("select k.name, p.value from pmc_events p join kernels k "
                           "on p.dispatch_id = k.dispatch_id where p.counter_name = ?", (counter,)).fetchall()
    return [(short(n), float(v)) for (n, v) in rows]


def _pmc(db: str, counter: str):
    """Per kernel symbol: (average KiB per dispatch, dispatches), and the calibration copy's
    reading (the largest dispatch of the runtime's copy kernel: small copies of a few bytes
    run beside it)."""
    acc = {}
    copy = 0.0
    for n, v in _pmc_rows(db, counter):
        t = acc.setdefault(n, [0.0, 0])
        t[0] += v
        t[1] += 1
        if n == COPY_SYMBOL:
            copy = max(copy, v)
    return {n: (t[0] / t[1], t[1]) for n, t in acc.items()}, copy


def write_traffic(fetch_db: str, write_db: str, out: str, command: str):
    fetch, cf = _pmc(fetch_db, "FETCH_SIZE")
    write, cw = _pmc(write_db, "WRITE_SIZE")
    if cf <= 0 or cw <= 0:
        raise SystemExit("no calibration copy (%s) in the counter runs" % COPY_SYMBOL)
    f_scale = COPY_BYTES / (cf * 1024.0)
    w_scale = COPY_BYTES / (cw * 1024.0)
    kernels = {}
    for name in sorted(set(fetch) & set(write)):
        kernels[name] = {"fetch_bytes_per_launch": fetch[name][0] * 1024.0 * f_scale,
                         "write_bytes_per_launch": write[name][0] * 1024.0 * w_scale,
                         "dispatches": fetch[name][1]}
    data = {"command": command, "source_sha1": source_hash(),
            "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": cf, "write_kib": cw,
                                 "fetch_scale": f_scale, "write_scale": w_scale},
            "kernels": kernels}
    with open(out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load_traffic(path: str, symbol_prefix: str):
    """Scaled HBM bytes per launch of the kernel whose symbol starts with symbol_prefix, if the
    figures were taken from the current kernel sources; else None."""
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("source_sha1") != source_hash():
        return None
    for name, k in data.get("kernels", {}).items():
        if name.startswith(symbol_prefix):
            return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
    return None


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        write_trace_md(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        write_traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    else:
        raise SystemExit(__doc__)
