"""Summarise rocprofv3 CSV output into the text summaries kept under profiles/.

Usage (after the profiling runs listed in each summary, from the repository
root):

    python -m paper_1809_00845_amd.profile_summary PROF_DIR WORKLOAD NAME [NOTE_FILE]
        [--kt DIR] [--fetch DIR] [--write DIR] [--counters DIR]
    python -m paper_1809_00845_amd.profile_summary --stats-only RUN_DIR NAME [NOTE_FILE]

PROF_DIR holds the rocprofv3 output directories kt/ (--kernel-trace --stats),
fetch/ and write/ (--pmc FETCH_SIZE / WRITE_SIZE of the workload), cfetch/
and cwrite/ (the same counters on bench.py --copy-probe: 5 launches of a
plain kernel that reads and writes 256 MiB); --kt/--fetch/--write name other
subdirectories of PROF_DIR, and --counters one with further --pmc counters
(their mean per dispatch is tabulated).  Writes profiles/NAME.md and
profiles/NAME_counters.json.  Kernel names are reduced to the kernel and its
template arguments.

The counters are scaled by what they read for the copy kernel of known size:
factor = known bytes / (counter KiB * 1024).  The JSON also records a hash of
the sources that define the apply kernels, so that bench.py reports the
measured traffic only while those kernels are unchanged.
"""

from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
APPLY_SOURCES = ["apply_impl.hpp", "fft_device.hpp", "kinds.hpp", "internal.hpp", "apply_l3d.hip", "apply_l2d.hip",
                 "apply_nav.hip", "api.hip"]
COPY_BYTES = 256 * 1024 * 1024


def apply_sources_sha256() -> str:
    h = hashlib.sha256()
    for fn in APPLY_SOURCES:
        h.update(open(os.path.join(HERE, "csrc", fn), "rb").read())
    return h.hexdigest()


def _find(d, suffix):
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def _norm(name):
    """'void bemfft::k_x<float, 2>(bemfft::ApplyArgs)' -> 'k_x<float, 2>'."""
    for pre in ("void ",):
        if name.startswith(pre):
            name = name[len(pre):]
    name = name.replace("bemfft::", "").replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):  # cut the parameter list (first '(' outside template brackets)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def _counter_values(d, counter):
    acc = defaultdict(list)
    with open(_find(d, "counter_collection.csv")) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter:
                acc[_norm(row["Kernel_Name"])].append(float(row["Counter_Value"]))
    return acc


def _all_counters(d):
    """{kernel: {counter: mean per dispatch}} of every counter in a run."""
    acc = defaultdict(lambda: defaultdict(list))
    with open(_find(d, "counter_collection.csv")) as f:
        for row in csv.DictReader(f):
            acc[_norm(row["Kernel_Name"])][row["Counter_Name"]].append(float(row["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def _counter_means(d, counter):
    return {k: (sum(v) / len(v), len(v)) for k, v in _counter_values(d, counter).items()}


def _copy_factor(d, counter):
    # the probe's fill and its five copies share torch's elementwise kernel
    # name; every copy moves 256 MiB each way, so the largest dispatch is one
    kib = max(max(v) for v in _counter_values(d, counter).values())
    return COPY_BYTES / (kib * 1024.0)


def _stats(d):
    stats = []
    with open(_find(d, "kernel_stats.csv")) as f:
        for row in csv.DictReader(f):
            name = _norm(row["Name"])
            # rocprofv3 -T leaves some template kernels mangled; keep the readable core
            for tag in ("k_conv16ILb0", "k_conv16ILb1"):
                if tag in name:
                    name = "k_conv16<" + ("false" if tag.endswith("0") else "true") + ">"
            stats.append((name, int(row["Calls"]), float(row["AverageNs"]) / 1e3, float(row["MinNs"]) / 1e3,
                          float(row["MaxNs"]) / 1e3, float(row["TotalDurationNs"]) / 1e3))
    return sorted(stats, key=lambda r: -r[5])


def stats_only(sub_dir, name, command_note="", top=25):
    """profiles/NAME.md with the kernel-trace statistics of one run."""
    lines = [f"# {name}", "", command_note, "", "| kernel | calls | avg us | min us | max us | total ms |",
             "|---|---|---|---|---|---|"]
    for n, c, a, lo, hi, tot in _stats(sub_dir)[:top]:
        lines.append(f"| {n} | {c} | {a:.1f} | {lo:.1f} | {hi:.1f} | {tot / 1e3:.2f} |")
    with open(os.path.join(ROOT, "profiles", name + ".md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def summarise(prof_dir, workload, name, command_note="", kt="kt", fetch_dir="fetch", write_dir="write",
              counters_dir=None):
    stats = [r[:5] for r in _stats(os.path.join(prof_dir, kt))]
    ff = _copy_factor(os.path.join(prof_dir, "cfetch"), "FETCH_SIZE")
    wf = _copy_factor(os.path.join(prof_dir, "cwrite"), "WRITE_SIZE")
    fetch = _counter_means(os.path.join(prof_dir, fetch_dir), "FETCH_SIZE")
    write = _counter_means(os.path.join(prof_dir, write_dir), "WRITE_SIZE")
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith("k_"):
            continue
        fk, nf = fetch.get(k, (0.0, 0))
        wk, nw = write.get(k, (0.0, 0))
        kernels[k] = {"fetch_kib": fk, "write_kib": wk, "read_bytes": fk * 1024 * ff, "write_bytes": wk * 1024 * wf,
                      "dispatches": max(nf, nw)}
    rec = {"workload": workload, "csrc_sha256": apply_sources_sha256(), "fetch_factor": ff, "write_factor": wf,
           "kernels": kernels}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", name + "_counters.json"), "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# {name}", "", command_note, "", "Kernel trace (rocprofv3 --kernel-trace --stats):", "",
             "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for n, c, a, lo, hi in sorted(stats, key=lambda r: -r[1] * r[2]):
        lines.append(f"| {n} | {c} | {a:.1f} | {lo:.1f} | {hi:.1f} |")
    lines += ["", f"HBM counters per dispatch, calibrated with the copy kernel (fetch factor {ff:.4f}, write "
                  f"factor {wf:.4f}):", "", "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | write MB |",
              "|---|---|---|---|---|"]
    for k, v in kernels.items():
        lines.append(f"| {k} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | {v['read_bytes'] / 1e6:.1f} | "
                     f"{v['write_bytes'] / 1e6:.1f} |")
    if counters_dir:
        cs = {k: v for k, v in _all_counters(os.path.join(prof_dir, counters_dir)).items() if k.startswith("k_")}
        names = sorted({c for v in cs.values() for c in v})
        lines += ["", "Further counters, mean per dispatch:", "", "| kernel | " + " | ".join(names) + " |",
                  "|---|" + "---|" * len(names)]
        for k, v in sorted(cs.items()):
            lines.append(f"| {k} | " + " | ".join(f"{v.get(c, float('nan')):.4g}" for c in names) + " |")
        rec["counters"] = cs
        with open(os.path.join(ROOT, "profiles", name + "_counters.json"), "w") as f:
            json.dump(rec, f, indent=1)
    with open(os.path.join(ROOT, "profiles", name + ".md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return rec


if __name__ == "__main__":
    if sys.argv[1] == "--stats-only":
        stats_only(sys.argv[2], sys.argv[3], open(sys.argv[4]).read() if len(sys.argv) > 4 else "")
    else:
        import argparse

        ap = argparse.ArgumentParser()
        ap.add_argument("prof_dir")
        ap.add_argument("workload")
        ap.add_argument("name")
        ap.add_argument("note", nargs="?")
        ap.add_argument("--kt", default="kt")
        ap.add_argument("--fetch", default="fetch")
        ap.add_argument("--write", default="write")
        ap.add_argument("--counters", default=None)
        a = ap.parse_args()
        summarise(a.prof_dir, a.workload, a.name, open(a.note).read() if a.note else "", a.kt, a.fetch, a.write,
                  a.counters)
