"""Summaries of rocprofv3 result databases for the profiles directory.

``--stats DB``: per-kernel dispatch counts and durations (kernel trace).
``--fetch DB --write DB``: HBM traffic of one kernel from two counter runs
(FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled by what the
same counter reads for a device-to-device copy of known size in the same run
(the largest copy dispatch; the benchmark issues one of ``--calib-bytes``).

The output is a short ``key: value`` text file that records the command lines,
the kernel and the SHA-256 of the device-code sources it was measured on.
"""

from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources the device code is compiled from
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("pmf_kernels.hip", "pmf_border.h", "pmf_internal.h")]


def source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_stats(db: str):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
                     "from kernels group by name order by sum(duration) desc").fetchall()
    return rows


def counter_per_kernel(db: str, counter: str):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, count(*), avg(value), max(value) from counters_collection "
                     "where counter_name = ? group by kernel_name", (counter,)).fetchall()
    return {r[0]: (r[1], r[2], r[3]) for r in rows}


def calib_kib(db: str, counter: str) -> float:
    """Counter reading (KiB) of the largest copy dispatch of the run."""
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, value from counters_collection where counter_name = ? and "
                     "lower(kernel_name) like '%copy%' order by value desc limit 1", (counter,)).fetchall()
    if not rows:
        raise SystemExit("no copy dispatch with %s in %s" % (counter, db))
    return float(rows[0][1])


def match(name: str, prefix: str) -> bool:
    return name.replace(" ", "").startswith(prefix.replace(" ", ""))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--stats")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", default="void pmf::k_step<4, 32, 32, false, true>")
    ap.add_argument("--calib-bytes", type=int, default=1 << 30)
    ap.add_argument("--command", action="append", default=[], help="command line that produced a database")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    lines = ["# rocprofv3 summary", "kernel_source_sha256: %s" % source_hash()]
    for cmd in a.command:
        lines.append("command: %s" % cmd)
    if a.stats:
        lines.append("## kernel trace (durations in microseconds)")
        lines.append("kernel | calls | total_us | avg_us | min_us | max_us")
        for name, n, tot, avg, mn, mx in kernel_stats(a.stats):
            lines.append("%s | %d | %.1f | %.3f | %.3f | %.3f" % (name, n, tot / 1e3, avg / 1e3, mn / 1e3, mx / 1e3))
            if match(name, a.kernel):
                lines.append("stats_kernel: %s" % name)
                lines.append("stats_avg_us: %.3f" % (avg / 1e3))
                lines.append("stats_calls: %d" % n)
    if a.fetch and a.write:
        fk = counter_per_kernel(a.fetch, "FETCH_SIZE")
        wk = counter_per_kernel(a.write, "WRITE_SIZE")
        cf = calib_kib(a.fetch, "FETCH_SIZE")
        cw = calib_kib(a.write, "WRITE_SIZE")
        f_scale = a.calib_bytes / (cf * 1024.0)
        w_scale = a.calib_bytes / (cw * 1024.0)
        lines.append("## HBM traffic from FETCH_SIZE / WRITE_SIZE (KiB per dispatch)")
        lines.append("calib_copy_bytes: %d" % a.calib_bytes)
        lines.append("calib_fetch_kib: %.1f" % cf)
        lines.append("calib_write_kib: %.1f" % cw)
        lines.append("fetch_scale: %.4f" % f_scale)
        lines.append("write_scale: %.4f" % w_scale)
        for name in sorted(set(fk) | set(wk)):
            if "copy" in name.lower() or "fill" in name.lower():
                continue
            nf, af, _ = fk.get(name, (0, 0.0, 0.0))
            nw, aw, _ = wk.get(name, (0, 0.0, 0.0))
            lines.append("%s | dispatches %d/%d | fetch_kib_avg %.1f | write_kib_avg %.1f" % (name, nf, nw, af, aw))
            if match(name, a.kernel):
                tb = af * 1024.0 * f_scale + aw * 1024.0 * w_scale
                lines.append("traffic_kernel: %s" % name)
                lines.append("traffic_fetch_bytes_per_launch: %.0f" % (af * 1024.0 * f_scale))
                lines.append("traffic_write_bytes_per_launch: %.0f" % (aw * 1024.0 * w_scale))
                lines.append("traffic_bytes_per_launch: %.0f" % tb)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_summary(path: str) -> dict:
    out = {}
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            if ": " in line and not line.startswith("#") and "|" not in line:
                k, v = line.rstrip("\n").split(": ", 1)
                out.setdefault(k, v)
    return out


if __name__ == "__main__":
    sys.exit(main())
