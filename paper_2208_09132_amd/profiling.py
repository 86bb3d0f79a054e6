"""Summaries of rocprofv3 output for the committed profiles.

Three kinds of summary, all markdown with a machine-readable JSON block:

* ``trace``: the ``*_kernel_stats.csv`` of a ``--kernel-trace --stats`` run,
  one row per kernel (calls, average, min, max duration).
* ``pmc``: HBM traffic of one kernel (or the kernels of one phase) from two ``--pmc`` runs, ``FETCH_SIZE``
  then ``WRITE_SIZE`` (KiB per dispatch).  Each counter is scaled by what it
  reads for a plain copy kernel of known size in the same run: the library's
  FP64-to-FP64 distribution copy (``k_to_f64<double>``, n doubles read and n
  written per dispatch).
* ``counters``: per-dispatch means of SQ counters of one kernel, with the
  instruction counters also per update.

The JSON block records a digest of the library's kernel and launch sources
(:func:`source_digest`); the benchmark only reports traffic from a summary
whose digest matches the sources it runs.

    python -m paper_2208_09132_amd.profiling trace <csv_dir> <out.md> --title T --command C
    python -m paper_2208_09132_amd.profiling pmc <fetch_dir> <write_dir> <out.md> --kernel K ...
    python -m paper_2208_09132_amd.profiling counters <csv_dir> <out.md> --kernel K --counter C ...
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# sources that decide what a kernel launch reads and writes
DIGEST_FILES = ["csrc/cdugks_kernels.hip", "csrc/cdugks_device.h", "csrc/cdugks_face_sums.hip",
                "csrc/cdugks_batched.hip", "csrc/cdugks_internal.h", "csrc/cdugks_api.cpp"]
COPY_PATTERN = r"k_to_f64<double>"


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in DIGEST_FILES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _one(pattern: str) -> str:
    found = sorted(glob.glob(pattern))
    if not found:
        raise FileNotFoundError(pattern)
    return found[0]


def kernel_stats(csv_dir: str):
    rows = []
    with open(_one(os.path.join(csv_dir, "*kernel_stats.csv"))) as f:
        for r in csv.DictReader(f):
            rows.append({"kernel": r["Name"], "calls": int(r["Calls"]),
                         "avg_us": float(r["AverageNs"]) / 1e3, "min_us": float(r["MinNs"]) / 1e3,
                         "max_us": float(r["MaxNs"]) / 1e3, "share": float(r["Percentage"])})
    return rows


def counter_means(csv_dir: str, counter: str):
    """Average counter value per dispatch, by kernel name."""
    acc = {}
    with open(_one(os.path.join(csv_dir, "*counter_collection.csv"))) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            s = acc.setdefault(r["Kernel_Name"], [0.0, 0])
            s[0] += float(r["Counter_Value"])
            s[1] += 1
    return {k: v[0] / v[1] for k, v in acc.items()}


def _find(means: dict, pattern: str) -> str:
    hits = [k for k in means if re.search(pattern, k)]
    if len(hits) != 1:
        raise ValueError(f"{pattern!r} matches {hits}")
    return hits[0]


def dispatch_durations(csv_dir: str, pattern: str):
    """Durations (us) of the dispatches of one kernel, in launch order."""
    out = []
    with open(_one(os.path.join(csv_dir, "*kernel_trace.csv"))) as f:
        for r in csv.DictReader(f):
            if re.search(pattern, r["Kernel_Name"]):
                out.append((int(r["Dispatch_Id"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    return [d for _, d in sorted(out)]


def write_trace(csv_dir, out, title, command, note="", tail_kernels=(), tail=10):
    rows = kernel_stats(csv_dir)
    lines = [f"# Kernel trace: {title}", "", "Command (from the repository root; committed files only):", "",
             "    " + command, "", f"Library sources digest: `{source_digest()}`.", ""]
    if note:
        lines += [note, ""]
    lines += ["| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['kernel'][:90]}` | {r['calls']} | {r['avg_us']:.1f} | {r['min_us']:.1f} | "
                     f"{r['max_us']:.1f} | {r['share']:.1f}% |")
    tails = {}
    if tail_kernels:
        lines += ["", f"Mean of the last {tail} dispatches (the benchmark's per-phase timing pass, after the "
                  "clock ramp of the first steps):", ""]
        for pat in tail_kernels:
            d = dispatch_durations(csv_dir, pat)
            if d:
                tails[pat] = sum(d[-tail:]) / len(d[-tail:])
                lines.append(f"* `{pat}`: {tails[pat]:.1f} us (all {len(d)} dispatches: {sum(d) / len(d):.1f} us)")
    lines += ["", "```json", json.dumps({"digest": source_digest(), "kernels": rows, "tail_mean_us": tails},
                                        indent=1), "```", ""]
    with open(out, "w") as f:
        f.write("\n".join(lines))


def write_pmc(fetch_dir, write_dir, out, kernels, title, commands, units_per_launch, algo_bytes_per_unit,
              copy_bytes):
    """HBM traffic of one launch of a phase: the kernels it runs (one
    dispatch each per phase), each counter scaled by the copy kernel's."""
    fm, wm = counter_means(fetch_dir, "FETCH_SIZE"), counter_means(write_dir, "WRITE_SIZE")
    c_f, c_w = _find(fm, COPY_PATTERN), _find(wm, COPY_PATTERN)
    f_fac = copy_bytes / (fm[c_f] * 1024.0)
    w_fac = copy_bytes / (wm[c_w] * 1024.0)
    per = []
    for pat in kernels:
        k_f, k_w = _find(fm, pat), _find(wm, pat)
        per.append({"kernel": k_f, "fetch_kib_raw": fm[k_f], "write_kib_raw": wm[k_w],
                    "fetch_bytes": fm[k_f] * 1024.0 * f_fac, "write_bytes": wm[k_w] * 1024.0 * w_fac})
    fetch = sum(k["fetch_bytes"] for k in per)
    write = sum(k["write_bytes"] for k in per)
    algo = units_per_launch * algo_bytes_per_unit
    rec = {"digest": source_digest(), "kernel": per[0]["kernel"], "kernels": per,
           "fetch_kib_raw": sum(k["fetch_kib_raw"] for k in per), "write_kib_raw": sum(k["write_kib_raw"] for k in per),
           "copy_kernel": c_f, "copy_bytes": copy_bytes, "copy_fetch_kib_raw": fm[c_f],
           "copy_write_kib_raw": wm[c_w],
           "fetch_factor": f_fac, "write_factor": w_fac, "fetch_bytes": fetch, "write_bytes": write,
           "traffic_bytes": fetch + write, "units_per_launch": units_per_launch,
           "algorithmic_bytes": algo}
    lines = [f"# HBM traffic: {title}", "", "Commands (from the repository root; committed files only):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", f"Library sources digest: `{source_digest()}`.", "",
              f"Calibration: the copy kernel `{c_f}` of the same run reads and writes {copy_bytes} bytes per "
              f"dispatch; its FETCH_SIZE reads {fm[c_f]:.0f} KiB (factor {f_fac:.3f}) and its WRITE_SIZE "
              f"{wm[c_w]:.0f} KiB (factor {w_fac:.3f}).", "",
              "| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | fetch (GB) | write (GB) | total (GB) | "
              "algorithmic (GB) |", "|---|---|---|---|---|---|---|"]
    for k in per:
        lines.append(f"| `{k['kernel'][:80]}` | {k['fetch_kib_raw']:.0f} | {k['write_kib_raw']:.0f} | "
                     f"{k['fetch_bytes'] / 1e9:.3f} | {k['write_bytes'] / 1e9:.3f} | "
                     f"{(k['fetch_bytes'] + k['write_bytes']) / 1e9:.3f} | |")
    if len(per) > 1:
        lines.append(f"| phase total | | | {fetch / 1e9:.3f} | {write / 1e9:.3f} | {(fetch + write) / 1e9:.3f} | "
                     f"{algo / 1e9:.3f} |")
    else:
        lines[-1] = lines[-1][:-2] + f"{algo / 1e9:.3f} |"
    lines += ["", "```json", json.dumps(rec, indent=1), "```", ""]
    with open(out, "w") as f:
        f.write("\n".join(lines))


def write_counters(csv_dir, out, kernel, counters, title, command, units_per_launch, wave_size=64):
    """Per-dispatch means of SQ counters for one kernel, and per update
    (units) where the counter counts wave instructions: instructions per
    update = counter / (units / wave size)."""
    means = {c: counter_means(csv_dir, c) for c in counters}
    name = _find(means[counters[0]], kernel)
    vals = {c: means[c][_find(means[c], kernel)] for c in counters}
    waves_per_launch = units_per_launch / wave_size
    rec = {"digest": source_digest(), "kernel": name, "units_per_launch": units_per_launch,
           "per_dispatch": vals,
           "per_update": {c: v / waves_per_launch for c, v in vals.items() if c.startswith("SQ_INSTS")}}
    if "SQ_ACTIVE_INST_VALU" in vals and "SQ_WAVE_CYCLES" in vals and vals["SQ_WAVE_CYCLES"] > 0:
        rec["valu_active_per_wave_cycle"] = vals["SQ_ACTIVE_INST_VALU"] / vals["SQ_WAVE_CYCLES"]
    lines = [f"# SQ counters: {title}", "", "Command (from the repository root; committed files only):", "",
             "    " + command, "", f"Library sources digest: `{source_digest()}`.", "",
             "| counter | per dispatch | per update (instruction counters) |", "|---|---|---|"]
    for c, v in vals.items():
        pu = rec["per_update"].get(c)
        lines.append(f"| {c} | {v:.4g} | {'' if pu is None else f'{pu:.1f}'} |")
    if "valu_active_per_wave_cycle" in rec:
        lines += ["", f"SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES = {rec['valu_active_per_wave_cycle']:.3f}."]
    lines += ["", "```json", json.dumps(rec, indent=1), "```", ""]
    with open(out, "w") as f:
        f.write("\n".join(lines))


def load_record(md_path: str):
    """The JSON block of a summary, or None."""
    try:
        text = open(md_path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv_dir")
    t.add_argument("out")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--note", default="")
    t.add_argument("--tail-kernel", action="append", default=[], help="regex; report its last dispatches")
    t.add_argument("--tail", type=int, default=10)
    p = sub.add_parser("pmc")
    p.add_argument("fetch_dir")
    p.add_argument("write_dir")
    p.add_argument("out")
    p.add_argument("--kernel", action="append", required=True,
                   help="regex selecting one kernel name; repeat for a phase of several kernels")
    p.add_argument("--title", required=True)
    p.add_argument("--command", action="append", required=True)
    p.add_argument("--units", type=float, required=True, help="updates per launch")
    p.add_argument("--algo-bytes", type=float, required=True, help="algorithmic bytes per update")
    p.add_argument("--copy-bytes", type=float, required=True, help="bytes read (and written) per copy dispatch")
    c = sub.add_parser("counters")
    c.add_argument("csv_dir")
    c.add_argument("out")
    c.add_argument("--kernel", required=True, help="regex selecting one kernel name")
    c.add_argument("--counter", action="append", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--units", type=float, required=True, help="updates per launch")
    a = ap.parse_args()
    if a.mode == "counters":
        write_counters(a.csv_dir, a.out, a.kernel, a.counter, a.title, a.command, a.units)
        return
    if a.mode == "trace":
        write_trace(a.csv_dir, a.out, a.title, a.command, a.note, a.tail_kernel, a.tail)
    else:
        write_pmc(a.fetch_dir, a.write_dir, a.out, a.kernel, a.title, a.command, a.units, a.algo_bytes,
                  a.copy_bytes)


if __name__ == "__main__":
    main()
