"""Turn rocprofv3 CSV output into the short text summaries kept with the code.

  python -m paper_2506_03905_amd.profile_summary stats KERNEL_STATS_CSV --cmd "..." > out.md
      per-kernel calls / average / share table of a ``--kernel-trace --stats`` run.

  python -m paper_2506_03905_amd.profile_summary traffic --kernel k_step \
      --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --copy-bytes N \
      --algorithmic-bytes B --cmd "..." > out.md
      HBM bytes per launch of one kernel from two ``--pmc`` runs (FETCH_SIZE,
      then WRITE_SIZE, both in KiB per dispatch), each scaled by what the same
      counter reads for a plain device copy of N bytes (it reads and writes N
      bytes), next to the kernel's algorithmic bytes B per launch.

  python -m paper_2506_03905_amd.profile_summary valu --kernel k_step --pmc DIR \
      --stats KERNEL_STATS_CSV --cells N --cmd "..." > out.md
      VALU instructions per cell update of each matching kernel from one
      ``--pmc SQ_INSTS_VALU SQ_WAVES`` run (one wave of 64 lanes updates 64
      cells), and the share of the kernel's duration (from a kernel-trace run
      of the same workload) the VALU issue alone needs on MI355X: 256 CUs x 4
      SIMDs, one wave64 VALU instruction per SIMD every 4 cycles, 2.4 GHz.

The traffic summary ends with a JSON block (fields ``fetch_bytes``,
``write_bytes``, ``traffic_bytes``, ``source_sha256``) that ``bench.py``
reads; ``source_sha256`` is the hash of the kernel sources' code (comments and
spacing left out) the counters were taken with, so a later change of the
kernels voids the figure.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import shutil
import statistics
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/lbm.hip", "csrc/lbm_device.hpp")


def _code_only(text: str) -> str:
    """C++ source without comments and blank space, so that an edit of a
    comment does not void the recorded counters (string literals are kept)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_sha256() -> str:
    """Hash of the kernel sources' code (comments and spacing excluded)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()


def _demangle(name: str) -> str:
    if not name.startswith("_Z") or not shutil.which("c++filt"):
        return name
    # binutils' c++filt predates the _Float16 mangling DF16_: spell it as half
    out = subprocess.run(["c++filt", name.replace("DF16_", "Dh")], capture_output=True,
                         text=True).stdout.strip()
    return out.replace("half", "_Float16") if out and not out.startswith("_Z") else name


def _short(name: str) -> str:
    name = _demangle(name)
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    cut = name.find("(lbmd::KP")
    return name[:cut] if cut > 0 else name[:90]


def stats(path: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", cmd, "```", "",
           "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.2f}% |")
    return "\n".join(out) + "\n"


def _counter(dirpath: str, counter: str, match: str) -> list:
    files = glob.glob(os.path.join(dirpath, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {dirpath}")
    vals = []
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter and match in r["Kernel_Name"]:
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} rows for kernels matching {match!r} in {dirpath}")
    return vals


def traffic(a) -> str:
    copy_f = statistics.mean(_counter(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)) * 1024.0
    copy_w = statistics.mean(_counter(a.copy_write, "WRITE_SIZE", a.copy_kernel)) * 1024.0
    kf = _counter(a.fetch, "FETCH_SIZE", a.kernel)
    kw = _counter(a.write, "WRITE_SIZE", a.kernel)
    scale_f = a.copy_bytes / copy_f
    scale_w = a.copy_bytes / copy_w
    fetch = statistics.mean(kf) * 1024.0 * scale_f
    write = statistics.mean(kw) * 1024.0 * scale_w
    res = {"kernel": a.kernel, "fetch_bytes": fetch, "write_bytes": write,
           "traffic_bytes": fetch + write, "algorithmic_bytes": a.algorithmic_bytes,
           "traffic_over_algorithmic": (fetch + write) / a.algorithmic_bytes,
           "fetch_scale": scale_f, "write_scale": scale_w, "dispatches": [len(kf), len(kw)],
           "source_sha256": source_sha256()}
    out = [f"# HBM traffic of `{a.kernel}`", "", "Commands:", "", "```", a.cmd, "```", "",
           f"Calibration: a plain device copy of {a.copy_bytes} bytes reads "
           f"{copy_f / 1024:.0f} KiB on FETCH_SIZE and {copy_w / 1024:.0f} KiB on WRITE_SIZE, "
           f"so FETCH_SIZE is scaled by {scale_f:.3f} and WRITE_SIZE by {scale_w:.3f}.", "",
           "| per launch | bytes |", "|---|---:|",
           f"| fetched (scaled) | {fetch:.4e} |", f"| written (scaled) | {write:.4e} |",
           f"| total | {fetch + write:.4e} |", f"| algorithmic | {a.algorithmic_bytes:.4e} |",
           f"| total / algorithmic | {res['traffic_over_algorithmic']:.3f} |", "",
           f"Kernel launches counted: {len(kf)} (FETCH_SIZE), {len(kw)} (WRITE_SIZE).", "",
           "```json", json.dumps(res, indent=1), "```"]
    return "\n".join(out) + "\n"


def _rows(dirpath: str) -> list:
    files = glob.glob(os.path.join(dirpath, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {dirpath}")
    return [r for f in files for r in csv.DictReader(open(f))]


def valu(a) -> str:
    per = {}
    for r in _rows(a.pmc):
        if a.kernel not in r["Kernel_Name"]:
            continue
        per.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    dur = {}
    for r in csv.DictReader(open(a.stats)):
        dur[r["Name"]] = float(r["AverageNs"]) * 1e-9
    out = ["# VALU instructions per cell update", "", "Commands:", "", "```", a.cmd, "```", "",
           f"Lattice of {a.cells} cells; one wave of 64 lanes per 64 cells, so VALU instructions "
           "per wave = per cell update.  Issue time = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x "
           "2.4 GHz) (one wave64 VALU instruction per SIMD every 4 cycles, no packed math).", "",
           "| kernel | launches | SQ_INSTS_VALU | SQ_WAVES | VALU per cell | kernel time (us) | VALU issue time (us) | share |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for name, c in sorted(per.items()):
        v = statistics.mean(c["SQ_INSTS_VALU"])
        w = statistics.mean(c["SQ_WAVES"])
        t_issue = v * 4 / (1024 * 2.4e9)
        short = _short(name)
        t = dur.get(name)
        share = f"{t_issue / t:.0%}" if t else "n/a"
        out.append(f"| `{short}` | {len(c['SQ_INSTS_VALU'])} | {v:.4e} | {w:.0f} | {v / w:.0f} | "
                   f"{t * 1e6 if t else float('nan'):.1f} | {t_issue * 1e6:.1f} | {share} |")
    return "\n".join(out) + "\n"


def read_traffic(path: str):
    """The JSON block of a traffic summary, or None if it is missing or was
    taken with other kernel sources."""
    try:
        text = open(path).read()
    except OSError:
        return None
    i = text.find("```json")
    if i < 0:
        return None
    j = text.find("```", i + 7)
    res = json.loads(text[i + 7:j])
    return res if res.get("source_sha256") == source_sha256() else None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--algorithmic-bytes", type=float, required=True)
    t.add_argument("--cmd", required=True)
    v = sub.add_parser("valu")
    v.add_argument("--kernel", required=True)
    v.add_argument("--pmc", required=True)
    v.add_argument("--stats", required=True)
    v.add_argument("--cells", type=int, required=True)
    v.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    sys.stdout.write({"stats": lambda: stats(a.csv, a.cmd), "traffic": lambda: traffic(a),
                      "valu": lambda: valu(a)}[a.mode]())


if __name__ == "__main__":
    main()
