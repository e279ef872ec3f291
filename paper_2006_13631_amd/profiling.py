"""Summaries of rocprofv3 CSV output (kernel statistics and HBM counters).

    python -m paper_2006_13631_amd.profiling stats KERNEL_STATS_CSV --out FILE --command CMD \
        [--trace KERNEL_TRACE_CSV --kernel NAME --windows A:B,C:D]
    python -m paper_2006_13631_amd.profiling traffic --fetch PMC_CSV --write PMC_CSV \
        --kernel k_stream_collide --copy-bytes N --out FILE --command CMD [--skip N]

`traffic` turns the FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch) of
a kernel into bytes per launch, each scaled by what the same counter reads
for a plain device copy of known size recorded in the same run, and stores
the SHA-256 of the kernel source so a later benchmark can tell whether the
counters still describe the kernel it runs.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import re
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")
COPY_KERNEL = "copyBuffer"


def source_sha256(path: str = KERNEL_SOURCE) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def _short(name: str) -> str:
    name = name.replace("mghlbm::(anonymous namespace)::", "")
    return name.split("(")[0].replace("void ", "")


def stats_table(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = [f"{'kernel':46s} {'calls':>7s} {'avg_us':>10s} {'min_us':>9s} {'max_us':>9s} {'pct':>7s}"]
    for r in rows:
        lines.append(f"{_short(r['Name'])[:46]:46s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.3f} "
                     f"{float(r['MinNs']) / 1e3:9.3f} {float(r['MaxNs']) / 1e3:9.3f} {float(r['Percentage']):7.2f}")
    return "\n".join(lines)


def window_table(trace: str, kernel: str, windows: str) -> str:
    """Mean duration of a kernel's launches in index windows [a, b) of the
    trace (launches in the order they ran)."""
    rows = [r for r in csv.DictReader(open(trace)) if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]
    out = [f"{kernel}: mean duration by launch window (launch index, in order)"]
    for w in windows.split(","):
        a, b = (int(x) for x in w.split(":"))
        seg = d[a:b]
        if seg:
            out.append(f"  launches {a:6d}..{b - 1:6d}: {len(seg):5d} launches, avg {sum(seg) / len(seg):9.3f} us")
    return "\n".join(out)


def _per_dispatch(path: str, counter: str):
    """{kernel: [value per dispatch]} for one counter (summed over its
    instances within a dispatch)."""
    rows = list(csv.DictReader(open(path)))
    acc = collections.defaultdict(float)
    names = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        d = r.get("Dispatch_Id") or r.get("Correlation_Id")
        acc[d] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    out = collections.defaultdict(list)
    for d in sorted(acc, key=lambda x: int(x) if str(x).isdigit() else x):  # in dispatch order
        out[names[d]].append(acc[d])
    return out


def kernel_file(kernel: str) -> str:
    """File-name form of a kernel name (template arguments joined by '_')."""
    return re.sub(r"[^A-Za-z0-9_]+", "_", kernel).strip("_")


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, skip: int = 0) -> dict:
    """skip: leave out the kernel's first `skip` dispatches of each run (in
    dispatch order), e.g. launches in a configuration the benchmark does
    not time."""
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = _per_dispatch(path, counter)
        # the kernel, not a longer name; with template arguments, that instance only
        match = (lambda n: kernel + "(" in n) if "<" in kernel else (lambda n: kernel + "<" in n)
        kv = [v for n, vs in per.items() if match(n) for v in vs][skip:]
        cv = [v for n, vs in per.items() if COPY_KERNEL in n for v in vs]
        if not kv or not cv:
            raise SystemExit(f"{counter}: no dispatch of {kernel!r} or of the copy kernel in {path}")
        copy_kib = max(cv)  # the calibration copy is the largest copy of the run
        scale = (copy_bytes / 1024.0) / copy_kib
        res[counter] = {"kernel_kib_per_dispatch": sum(kv) / len(kv), "dispatches": len(kv), "skipped": skip,
                        "copy_kib": copy_kib, "copy_scale": scale,
                        "bytes_per_launch": sum(kv) / len(kv) * 1024.0 * scale}
    res["bytes_per_launch"] = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    return res


def counters(path: str, kernels: list) -> str:
    """Mean per dispatch of every counter in a rocprofv3 --pmc CSV for each
    kernel (a name matches when it contains the given text), and ratios of
    counters whose units cancel."""
    rows = list(csv.DictReader(open(path)))
    names = sorted({r["Counter_Name"] for r in rows})
    out = []
    for k in kernels:
        mean = {}
        for c in names:
            vs = [v for n, lst in _per_dispatch(path, c).items() if k in n for v in lst]
            if vs:
                mean[c] = (sum(vs) / len(vs), len(vs))
        if not mean:
            out.append(f"{k}: no dispatch")
            continue
        out.append(f"{k}  ({max(n for _, n in mean.values())} dispatches)")
        for c, (v, _) in mean.items():
            out.append(f"  {c:<24s} {v:16.1f}")
        g = {c: v for c, (v, _) in mean.items()}
        ratios = [("SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES", "wave cycles waiting on any instruction"),
                  ("SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES", "wave cycles waiting on LDS"),
                  ("SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", "wave cycles issuing VALU"),
                  ("SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS", "bank-conflict cycles per LDS instruction"),
                  ("SQ_INSTS_VALU", "SQ_WAVES", "VALU instructions per wave"),
                  ("SQ_INSTS_LDS", "SQ_WAVES", "LDS instructions per wave")]
        for a, b, label in ratios:
            if a in g and b in g and g[b] > 0:
                out.append(f"  {a} / {b} = {g[a] / g[b]:.3f}  ({label})")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--out", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--trace")
    s.add_argument("--kernel", default="k_stream_collide")
    s.add_argument("--windows")
    s.add_argument("--note", default="")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--kernels", required=True, help="texts a kernel name must contain, separated by ';'")
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--note", default="")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--skip", type=int, default=0, help="leave out the kernel's first N dispatches")
    t.add_argument("--note", default="")
    t.add_argument("--workload", required=True)
    t.add_argument("--storage", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        text = (f"# rocprofv3 counters, mean per dispatch\n# command: {a.command}\n"
                + counters(a.csv, a.kernels.split(";")) + "\n")
        if a.note:
            text += "".join(f"# {line}\n" for line in a.note.split("\n"))
        open(a.out, "w").write(text)
        print(text)
        return
    if a.cmd == "stats":
        text = f"# rocprofv3 kernel statistics\n# command: {a.command}\n" + stats_table(a.csv) + "\n"
        if a.trace and a.windows:
            text += "\n" + window_table(a.trace, a.kernel, a.windows) + "\n"
        if a.note:
            text += "".join(f"# {line}\n" for line in a.note.split("\n"))
        open(a.out, "w").write(text)
        print(text)
    else:
        res = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.skip)
        res.update({"kernel": a.kernel, "workload": a.workload, "storage": a.storage,
                    "source_sha256": source_sha256(), "command": a.command})
        if a.note:
            res["note"] = a.note
        json.dump(res, open(a.out, "w"), indent=1)
        print(json.dumps(res, indent=1))


if __name__ == "__main__":
    sys.exit(main())
