"""Turn rocprofv3 output into the short summaries kept under profiles/.

    python -m paper_1110_0899_amd.profiling stats <rocprofv3 dir> <out.md> "<command>"
    python -m paper_1110_0899_amd.profiling counters --kernel team_kernel --workload 2d_L4096 \
        --fetch <dir> --write <dir> --copy-fetch <dir> --copy-write <dir> \
        --last <n dispatches> --added <added spins> --out profiles/counters_<kernel>_<workload>.json \
        --command "<command>"

    python -m paper_1110_0899_amd.profiling pmc --kernel lds_kernel --dir <dir> --last <n> \
        --added <added spins> --out profiles/<name>.md --command "<command>" [--note ...]

`stats` reads the kernel-trace statistics (csv or rocpd sqlite output) and
writes a markdown table.  `pmc` sums every counter of one `--pmc` run over
the last n dispatches of a kernel and writes them per dispatch and per added
spin.  `counters` averages FETCH_SIZE / WRITE_SIZE (KiB
per dispatch) over the last n dispatches of a kernel, scales each by what
the same counter reports for the calibration copy (1 GiB read, 1 GiB
written), and records the kernel-source hash, so that bench.py uses the
figure only while the kernels are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


# The device code: the kernels and the headers they include (csrc-relative;
# the public header defines the record layout the kernels write).  The host
# library (wolff_lib.hip) is left out, so a change to its heuristics keeps
# the counter figures of unchanged kernels.
DEVICE_SOURCES = ("wolff_device.h", "wolff_kernels.h", "wolff_kernels.hip", "wolff_lds.hip",
                  "../../include/wolff.h")


def code_tokens(text: str) -> str:
    """C/C++ source with its comments removed and each run of whitespace
    made one space (string and character literals kept as written), so that
    a change to documentation alone leaves the hash of the code as it was."""
    out = []
    i, n = 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_sha() -> str:
    """Hash of the device code (the one bench.py checks counter files
    against): the sources' tokens, comments and layout left out."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in DEVICE_SOURCES:
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode() + b"\0" + code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def kernel_stats(d: str):
    """[(name, calls, total_us, avg_us, pct)] from a rocprofv3 output directory."""
    csvs = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    rows = []
    if csvs:
        for r in csv.DictReader(open(csvs[0])):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                         float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
        return rows
    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if not dbs:
        raise SystemExit("no kernel statistics under %s" % d)
    c = sqlite3.connect(dbs[0])
    for n, calls, tot, avg, pct in c.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        rows.append((n, int(calls), float(tot), float(avg), float(pct)))
    return rows


def write_stats(d: str, out: str, command: str, note: str = ""):
    rows = kernel_stats(d)
    with open(out, "w") as f:
        f.write("# rocprofv3 kernel statistics\n\nCommand (repository at $R, run from a scratch "
                "directory):\n\n    %s\n\n" % command)
        if note:
            f.write(note.strip() + "\n\n")
        f.write("| kernel | calls | total us | average us | % |\n|---|---|---|---|---|\n")
        for n, calls, tot, avg, pct in rows:
            f.write("| `%s` | %d | %.1f | %.3f | %.2f |\n" % (n.split("(")[0], calls, tot, avg, pct))
        f.write("\nKernel sources: %s\n" % kernel_source_sha())


def counter_values(d: str, kernel: str, counter: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    vals = []
    for r in csv.DictReader(open(files[0])):
        if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter:
            vals.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    vals.sort()
    return [v for _, v in vals]


def counters(a):
    f = counter_values(a.fetch, a.kernel, "FETCH_SIZE")[-a.last:]
    w = counter_values(a.write, a.kernel, "WRITE_SIZE")[-a.last:]
    cf = max(counter_values(a.copy_fetch, "copyBuffer", "FETCH_SIZE"))
    cw = max(counter_values(a.copy_write, "copyBuffer", "WRITE_SIZE"))
    gib_kib = float(1 << 20)
    fetch_scale, write_scale = gib_kib / cf, gib_kib / cw
    fetch_b = sum(f) / len(f) * 1024 * fetch_scale
    write_b = sum(w) / len(w) * 1024 * write_scale
    out = {
        "kernel": a.kernel, "workload": a.workload, "kernel_source_sha": kernel_source_sha(),
        "command": a.command, "dispatches": len(f),
        "fetch_kib_per_dispatch_raw": sum(f) / len(f), "write_kib_per_dispatch_raw": sum(w) / len(w),
        "copy_fetch_kib_per_gib": cf, "copy_write_kib_per_gib": cw,
        "fetch_scale": fetch_scale, "write_scale": write_scale,
        "hbm_bytes_per_launch": fetch_b + write_b,
    }
    if a.added:
        out["added_spins_per_launch"] = a.added / len(f)
        out["hbm_bytes_per_added_spin"] = (fetch_b + write_b) / (a.added / len(f))
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def pmc_table(a):
    files = glob.glob(os.path.join(a.dir, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    for r in csv.DictReader(open(files[0])):
        if a.kernel in r["Kernel_Name"]:
            per.setdefault(r["Counter_Name"], []).append((int(r["Dispatch_Id"]),
                                                          float(r["Counter_Value"])))
    name = None
    for r in csv.DictReader(open(files[0])):
        if a.kernel in r["Kernel_Name"]:
            name = r["Kernel_Name"].split("(")[0]
            break
    with open(a.out, "w") as f:
        f.write("# rocprofv3 counters of `%s`\n\nCommand (repository at $R, run from a scratch "
                "directory):\n\n    %s\n\n" % (name, a.command))
        if a.note:
            f.write(a.note.strip() + "\n\n")
        f.write("Summed over the last %d dispatches (%.4g added spins).\n\n" % (a.last, a.added))
        f.write("| counter | per dispatch | per added spin |\n|---|---|---|\n")
        for c in sorted(per):
            v = [x for _, x in sorted(per[c])][-a.last:]
            tot = sum(v)
            f.write("| `%s` | %.4g | %s |\n" % (c, tot / len(v),
                                               "%.4g" % (tot / a.added) if a.added else "-"))
        f.write("\nKernel sources: %s\n" % kernel_source_sha())


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("out")
    s.add_argument("command")
    s.add_argument("--note", default="")
    c = sub.add_parser("counters")
    for k in ("kernel", "workload", "fetch", "write", "copy_fetch", "copy_write", "out", "command"):
        c.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    c.add_argument("--last", type=int, default=1)
    c.add_argument("--added", type=float, default=0.0, help="added spins over the last dispatches")
    m = sub.add_parser("pmc")
    for k in ("kernel", "dir", "out", "command"):
        m.add_argument("--" + k, dest=k, required=True)
    m.add_argument("--last", type=int, default=1)
    m.add_argument("--added", type=float, default=0.0)
    m.add_argument("--note", default="")
    a = ap.parse_args()
    if a.cmd == "stats":
        write_stats(a.dir, a.out, a.command, a.note)
    elif a.cmd == "pmc":
        pmc_table(a)
    else:
        counters(a)


if __name__ == "__main__":
    main()
