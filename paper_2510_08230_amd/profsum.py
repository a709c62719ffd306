"""Summaries of rocprofv3 CSV output for the profiles/ directory.

  python -m paper_2510_08230_amd.profsum stats  KERNEL_STATS_CSV [--trace KERNEL_TRACE_CSV] --cmd "..."
  python -m paper_2510_08230_amd.profsum traffic FETCH_CSV WRITE_CSV --kernel SUBSTR --copy-bytes B [--last N]
      [--logs FETCH_LOG WRITE_LOG] --cmd "..."
  python -m paper_2510_08230_amd.profsum traffic-total FETCH_CSV WRITE_CSV --kernel SUBSTR --copy-bytes B
      --algorithmic BYTES --cmd "..."

``stats`` renders the per-kernel duration table.  ``traffic`` reports the
median FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the dispatches of one
kernel, scaled by what the same counters read for the library's plain copy
kernel (k_copy16) of known size, plus the digest of the sources the CG
SpMV kernel is built from (the benchmark drops the figures once those
sources change).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/spk_kernels.hip", "csrc/spk_spmv.h", "csrc/spk_device.h", "csrc/spk_internal.h",
                  "csrc/spk_fcg.h"]


def kernel_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stats_md(path: str, cmd: str, top: int = 15) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# rocprofv3 kernel statistics", "", "Command (repository root):", "", "    " + cmd, "",
           "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].replace("(anonymous namespace)::", "").replace("|", "/")
        if len(name) > 110:
            name = name[:107] + "..."
        out.append("| %s | %s | %.1f | %.1f | %.1f | %.1f |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    return "\n".join(out) + "\n"


def working_launches_md(trace_csv: str, top: int = 8) -> str:
    """Per kernel: launches that did work (duration >= 20% of the kernel's
    longest; launches enqueued past convergence return at once), with their
    mean and median duration, from a --kernel-trace CSV."""
    durs = {}
    for r in csv.DictReader(open(trace_csv)):
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        durs.setdefault(r["Kernel_Name"], []).append(d)
    rows = []
    for name, v in durs.items():
        top_d = max(v)
        w = [x for x in v if x >= 0.2 * top_d]
        rows.append((sum(w), name, len(w), len(v), statistics.mean(w), statistics.median(w)))
    rows.sort(reverse=True)
    out = ["", "Launches that did work (duration >= 20% of the kernel's longest launch; launches enqueued",
           "after convergence return at once and are left out):", "",
           "| kernel | working / all launches | mean us | median us |", "|---|---|---|---|"]
    for _, name, nw, na, mean, med in rows[:top]:
        name = name.replace("(anonymous namespace)::", "").replace("|", "/")
        if len(name) > 110:
            name = name[:107] + "..."
        out.append("| %s | %d / %d | %.1f | %.1f |" % (name, nw, na, mean, med))
    return "\n".join(out) + "\n"


def _per_kernel(path: str, counter: str):
    """Kernel name -> counter values in dispatch order."""
    rows = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    vals = {}
    for _, name, v in rows:
        vals.setdefault(name, []).append(v)
    return vals


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, last: int = 20) -> dict:
    """Median counter value of the last `last` working dispatches of the kernel
    whose name contains `kernel` (the timed loop's, after any tuning runs),
    scaled by the copy kernel's reading of a known size."""
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")

    def pick(d, sub, tail=last):
        got = [v for k, v in d.items() if sub in k]
        if not got:
            raise SystemExit("no dispatch of %r in the counter CSV" % sub)
        if len(got) > 1:
            raise SystemExit("%r matches %d kernels; name one" % (sub, len(got)))
        vals = got[0]
        work = [x for x in vals if x > 0.01 * max(vals)]   # drop launches that returned at once
        return statistics.median(work[-tail:] if tail else work)

    copy_f = pick(f, "k_copy16", 0)
    copy_w = pick(w, "k_copy16", 0)
    scale_f = copy_bytes / (copy_f * 1024.0)
    scale_w = copy_bytes / (copy_w * 1024.0)
    kf = pick(f, kernel)
    kw = pick(w, kernel)
    return {"kernel": kernel, "fetch_kib": kf, "write_kib": kw, "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
            "copy_bytes_each_way": copy_bytes, "fetch_scale": scale_f, "write_scale": scale_w,
            "read_bytes": kf * 1024.0 * scale_f, "write_bytes": kw * 1024.0 * scale_w,
            "traffic_bytes": kf * 1024.0 * scale_f + kw * 1024.0 * scale_w, "kernel_digest": kernel_digest()}


def traffic_total(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, algorithmic: float) -> dict:
    """Counter totals over every dispatch of a kernel whose work differs from
    dispatch to dispatch (the serving tick's SpMV), copy-scaled, against the
    algorithmic bytes of the whole run."""
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")

    def one(d, sub):
        got = [v for k, v in d.items() if sub in k]
        if len(got) != 1:
            raise SystemExit("%r matches %d kernels" % (sub, len(got)))
        return got[0]

    copy_f = statistics.median(one(f, "k_copy16"))
    copy_w = statistics.median(one(w, "k_copy16"))
    kf, kw = one(f, kernel), one(w, kernel)
    rb = sum(kf) * 1024.0 * copy_bytes / (copy_f * 1024.0)
    wb = sum(kw) * 1024.0 * copy_bytes / (copy_w * 1024.0)
    return {"kernel": kernel, "dispatches": [len(kf), len(kw)], "fetch_kib_total": sum(kf),
            "write_kib_total": sum(kw), "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
            "copy_bytes_each_way": copy_bytes, "read_bytes": rb, "write_bytes": wb, "traffic_bytes": rb + wb,
            "algorithmic_bytes": algorithmic, "traffic_over_algorithmic": (rb + wb) / algorithmic,
            "kernel_digest": kernel_digest()}


TILING_KEYS = ("spmv_kernel", "lanes", "grid", "xcd_remap", "col_codes")


def bench_tiling(log_path: str) -> dict:
    """The SpMV launch shape a benchmark run reported (its JSON line)."""
    for line in reversed(open(log_path).read().splitlines()):
        if line.startswith("{"):
            t = json.loads(line)["config"]["spmv_tiling"]
            return {k: t[k] for k in TILING_KEYS}
    raise SystemExit("no benchmark JSON line in %s" % log_path)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--trace", help="kernel-trace CSV of the same run: adds the working-launch table")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--last", type=int, default=20, help="use the kernel's last N working dispatches")
    t.add_argument("--cmd", required=True)
    t.add_argument("--logs", nargs=2, metavar=("FETCH_LOG", "WRITE_LOG"),
                   help="the two runs' benchmark output: their SpMV tiling (which must agree) is recorded")
    u = sub.add_parser("traffic-total")
    u.add_argument("fetch_csv")
    u.add_argument("write_csv")
    u.add_argument("--kernel", required=True)
    u.add_argument("--copy-bytes", type=int, required=True)
    u.add_argument("--algorithmic", type=float, required=True, help="algorithmic bytes of all dispatches")
    u.add_argument("--cmd", required=True)
    a = ap.parse_args()
    if a.what == "traffic-total":
        d = traffic_total(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, a.algorithmic)
        d["command"] = a.cmd
        print(json.dumps(d, indent=1))
        return
    if a.what == "stats":
        print(stats_md(a.csv, a.cmd), end="")
        if a.trace:
            print(working_launches_md(a.trace), end="")
    else:
        d = traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, a.last)
        if a.logs:
            tilings = [bench_tiling(p) for p in a.logs]
            if tilings[0] != tilings[1]:
                raise SystemExit("the two runs chose different SpMV tilings: %s vs %s" % tuple(tilings))
            d["tiling"] = tilings[0]
        d["command"] = a.cmd
        print(json.dumps(d, indent=1))


if __name__ == "__main__":
    main()
