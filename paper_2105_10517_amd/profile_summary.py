"""Text summaries of rocprofv3 output for ``profiles/``.

    python3 paper_2105_10517_amd/profile_summary.py stats RUN_DIR [--last N] --command "..." --out profiles/NAME.md
    python3 paper_2105_10517_amd/profile_summary.py traffic --fetch DIR --write DIR --copy-fetch DIR \
        --copy-write DIR --copy-mib 512 --command "..." --out profiles/NAME.md
    python3 paper_2105_10517_amd/profile_summary.py counters DIR [DIR ...] [--match RE] [--last N] \
        --command "..." --out profiles/NAME.md

``stats`` condenses ``*_kernel_stats.csv`` of a ``--kernel-trace --stats``
run (calls, mean / min / max duration per kernel).  ``traffic`` turns
``FETCH_SIZE`` and ``WRITE_SIZE`` passes (KiB per dispatch) into bytes per
launch of every SSCN kernel, scaled by what the same counters read for a
plain device copy of known size, and records a hash of the kernel sources so
that a reader (``bench.py``) can tell whether the numbers still describe the
kernels it runs.  ``counters`` tabulates other ``--pmc`` passes (SQ, TA, TCP,
TCC groups) per kernel, with per-wave instruction counts and a few ratios.
"""
import argparse
import csv
import glob
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def kernel_source_hash() -> str:
    """sha256 over the device and launch sources of the library."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp")) and f != "gp_runtime.hip":
            h.update(f.encode())
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    n = re.sub(r"\(.*", "", name)
    n = re.sub(r"^void ", "", n)
    return n


def find(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def counters(d: str, counter: str, last: int = 0) -> dict:
    """Mean value per dispatch of one counter, per kernel; with last > 0 over
    each kernel's last `last` dispatches only (the timed steps of a run whose
    launch shapes were tuned first, not the tuner's candidates)."""
    acc = {}
    for row in csv.DictReader(open(find(d, "counter_collection.csv"))):
        if row["Counter_Name"] != counter:
            continue
        acc.setdefault(short(row["Kernel_Name"]), []).append((int(row["Dispatch_Id"]), float(row["Counter_Value"])))
    out = {}
    for k, v in acc.items():
        v = [x for _, x in sorted(v)]
        if last > 0:
            v = v[-last:]
        out[k] = sum(v) / len(v)
    return out


def last_means(d: str, last: int) -> dict:
    """Per kernel, from the kernel trace: the launch shape (grid size) that
    took the most time in total (one workload's timed steps: tuning candidates
    and other, smaller workloads launch other shapes), that shape's dispatch
    count, and the mean duration in us of its last `last` dispatches."""
    acc = {}
    for row in csv.DictReader(open(find(d, "kernel_trace.csv"))):
        acc.setdefault(short(row["Kernel_Name"]), {}).setdefault(int(row["Grid_Size_X"]), []).append(
            (int(row["Dispatch_Id"]), int(row["End_Timestamp"]) - int(row["Start_Timestamp"])))
    out = {}
    for k, shapes in acc.items():
        grid, v = max(shapes.items(), key=lambda kv: sum(x for _, x in kv[1]))
        t = [x for _, x in sorted(v)][-last:]
        out[k] = (grid, len(v), sum(t) / len(t) / 1e3)
    return out


def cmd_stats(a):
    rows = list(csv.DictReader(open(find(a.run_dir, "kernel_stats.csv"))))
    tail = last_means(a.run_dir, a.last) if a.last else {}
    lines = [f"# Kernel durations: {a.title}", "", "Command:", "", "```", a.command, "```", "",
             f"Kernel sources: `{kernel_source_hash()}`", ""]
    if a.last:
        lines += [f"Last columns: each kernel's launch shape (grid size in work-items) with the largest total "
                  f"time, its dispatches, and their mean over the last {a.last} (one workload's timed steps; "
                  f"tuning candidates and other workloads launch other shapes).", ""]
    lines += ["| kernel | calls | mean us | min us | max us | share |" + (
              f" main grid | its calls | its last {a.last} mean us |" if a.last else ""),
              "|---|---:|---:|---:|---:|---:|" + ("---:|---:|---:|" if a.last else "")]
    for r in rows:
        k = short(r["Name"])
        extra = ""
        if a.last:
            extra = f" {tail[k][0]} | {tail[k][1]} | {tail[k][2]:.2f} |" if k in tail else " | | |"
        lines.append(f"| `{k}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f}% |"
                     + extra)
    open(a.out, "w").write("\n".join(lines) + "\n")


def cmd_traffic(a):
    copy_bytes = a.copy_mib * (1 << 20)
    cf = counters(a.copy_fetch, "FETCH_SIZE")
    cw = counters(a.copy_write, "WRITE_SIZE")
    ck = max(cf, key=cf.get)  # the copy kernel reads the most
    f_scale = copy_bytes / (cf[ck] * 1024.0)
    w_scale = copy_bytes / (cw[max(cw, key=cw.get)] * 1024.0)
    fetch = counters(a.fetch, "FETCH_SIZE", a.last)
    write = counters(a.write, "WRITE_SIZE", a.last)
    s = 16 if a.precision == "fp64" else 8
    algo = 3 * s * a.points  # read or write of one sweep kernel, bytes per launch
    lines = [f"# HBM traffic per launch: {a.title}", "", "Commands (one counter per pass):", "", "```",
             a.command, "```", "",
             f"Kernel sources: `{kernel_source_hash()}`", "",
             f"Calibration: a plain copy of {a.copy_mib} MiB reads FETCH_SIZE = {cf[ck]:.0f} KiB and "
             f"WRITE_SIZE = {cw[max(cw, key=cw.get)]:.0f} KiB per dispatch: fetch factor {f_scale:.3f}, "
             f"write factor {w_scale:.3f}.", "",
             f"Algorithmic bytes per sweep launch: read {algo} B + write {algo} B "
             f"(3 complex values of {s} B per point, {a.points} points)."
             + (f"  Per kernel, the mean over its last {a.last} dispatches (the timed steps after"
                f" the launch shapes were tuned)." if a.last else ""), "",
             "| kernel | fetch B | write B | traffic B | fetch / algo | write / algo |",
             "|---|---:|---:|---:|---:|---:|"]
    for k in sorted(set(fetch) & set(write)):
        if "k_x_" not in k and "k_y_" not in k:
            continue
        fb = fetch[k] * 1024.0 * f_scale
        wb = write[k] * 1024.0 * w_scale
        lines.append(f"| `{k}` | {fb:.4g} | {wb:.4g} | {fb + wb:.4g} | {fb / algo:.3f} | {wb / algo:.3f} |")
    open(a.out, "w").write("\n".join(lines) + "\n")


def all_counters(d: str, last: int = 0) -> dict:
    """kernel -> counter -> mean value per dispatch (over the last `last`
    dispatches of each kernel when last > 0)."""
    acc = {}
    for row in csv.DictReader(open(find(d, "counter_collection.csv"))):
        k = short(row["Kernel_Name"])
        c = acc.setdefault(k, {}).setdefault(row["Counter_Name"], {})
        did = int(row["Dispatch_Id"])
        c[did] = c.get(did, 0.0) + float(row["Counter_Value"])
    out = {}
    for k, cs in acc.items():
        out[k] = {}
        for c, v in cs.items():
            vals = [v[i] for i in sorted(v)]
            if last > 0:
                vals = vals[-last:]
            out[k][c] = sum(vals) / len(vals)
    return out


# Ratios worth reading off the counters (name, numerator, denominator).
DERIVED = (
    ("VALU instr / wave", "SQ_INSTS_VALU", "SQ_WAVES"),
    ("FP64 FMA / wave", "SQ_INSTS_VALU_FMA_F64", "SQ_WAVES"),
    ("FP64 MUL / wave", "SQ_INSTS_VALU_MUL_F64", "SQ_WAVES"),
    ("FP64 ADD / wave", "SQ_INSTS_VALU_ADD_F64", "SQ_WAVES"),
    ("FP32 FMA / wave", "SQ_INSTS_VALU_FMA_F32", "SQ_WAVES"),
    ("SALU instr / wave", "SQ_INSTS_SALU", "SQ_WAVES"),
    ("LDS instr / wave", "SQ_INSTS_LDS", "SQ_WAVES"),
    ("vector loads / wave", "SQ_INSTS_VMEM_RD", "SQ_WAVES"),
    ("vector stores / wave", "SQ_INSTS_VMEM_WR", "SQ_WAVES"),
    ("wave cycles / busy cycle", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES"),
    ("waiting / issuing (any instr)", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY"),
    ("VALU share of issue", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_ANY"),
    ("L2 hit rate", "TCC_HIT_sum", ("TCC_HIT_sum", "TCC_MISS_sum")),
)


def cmd_counters(a):
    merged = {}
    for d in a.runs:
        for k, cs in all_counters(d, a.last).items():
            merged.setdefault(k, {}).update(cs)
    keep = [k for k in sorted(merged) if any(re.search(m, k) for m in a.match)] if a.match else sorted(merged)
    names = sorted({c for k in keep for c in merged[k]})
    lines = [f"# Counters per dispatch: {a.title}", "", "Commands (one counter group per pass):", "", "```",
             a.command, "```", "", f"Kernel sources: `{kernel_source_hash()}`", "",
             "Mean value per dispatch" + (f" over each kernel's last {a.last} dispatches" if a.last else "")
             + ", summed over the hardware instances of each counter.", ""]
    lines += ["| ratio | " + " | ".join(f"`{k}`" for k in keep) + " |", "|---|" + "---:|" * len(keep)]
    for label, num, den in DERIVED:
        row = []
        for k in keep:
            c = merged[k]
            dv = sum(c.get(x, 0.0) for x in den) if isinstance(den, tuple) else c.get(den, 0.0)
            row.append(f"{c[num] / dv:.3g}" if num in c and dv else "")
        if any(row):
            lines.append(f"| {label} | " + " | ".join(row) + " |")
    lines += ["", "| counter | " + " | ".join(f"`{k}`" for k in keep) + " |", "|---|" + "---:|" * len(keep)]
    for c in names:
        lines.append(f"| {c} | " + " | ".join(f"{merged[k][c]:.4g}" if c in merged[k] else "" for k in keep) + " |")
    open(a.out, "w").write("\n".join(lines) + "\n")


def read_traffic(path: str) -> dict:
    """Kernel -> traffic bytes per launch from a summary written by ``traffic``,
    or {} when the kernel sources have changed since."""
    if not os.path.exists(path):
        return {}
    txt = open(path).read()
    m = re.search(r"Kernel sources: `([0-9a-f]+)`", txt)
    if not m or m.group(1) != kernel_source_hash():
        return {}
    out = {}
    for line in txt.splitlines():
        mm = re.match(r"\| `([^`]+)` \| ([0-9.e+]+) \| ([0-9.e+]+) \| ([0-9.e+]+) \|", line)
        if mm:
            out[mm.group(1)] = float(mm.group(4))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("run_dir")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--last", type=int, default=0, help="add each kernel's main launch shape and its mean over its last N dispatches")
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--points", type=int, required=True, help="grid points nx ny of the workload")
    t.add_argument("--precision", choices=("fp64", "fp32"), required=True)
    t.add_argument("--last", type=int, default=0, help="use each kernel's last N dispatches only")
    t.add_argument("--command", required=True)
    t.add_argument("--title", default="")
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("runs", nargs="+", help="rocprofv3 --pmc output directories (one counter group each)")
    c.add_argument("--match", action="append", default=[], help="keep kernels whose name matches (regex; repeatable)")
    c.add_argument("--last", type=int, default=0, help="use each kernel's last N dispatches only")
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="")
    c.add_argument("--out", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters}[a.cmd](a)


if __name__ == "__main__":
    main()
