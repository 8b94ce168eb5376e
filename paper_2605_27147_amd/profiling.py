"""Summaries of rocprofv3 runs for the profiles/ directory.

    python -m paper_2605_27147_amd.profiling stats   DIR OUT.txt --title T --command C
    python -m paper_2605_27147_amd.profiling traffic FETCH_DIR WRITE_DIR OUT.json --kind K --copy-bytes N
        [--command C ...] [--calibrate FETCH_DIR2 WRITE_DIR2]

`stats` turns a `rocprofv3 --kernel-trace --stats --output-format csv` output
directory into a short text table (kernel, calls, total ms, average us, %).

`counters` turns `rocprofv3 --pmc <SQ counters>` runs into the average per
launch of every counter for one kernel kind (instruction counts, LDS bytes
in 64-byte units, cycle counts), with the kernel's source hashes.

`traffic` turns two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
the same command into HBM bytes per launch of one kernel kind.  Both counters
are scaled by what they report for a device copy of known size in the same
run (the runtime's copy kernel): the copy reads and writes N bytes each.  The
JSON records the SHA-256 of the kernel's source files, so a reader can tell
whether the kernel has changed since the counters were taken.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# kernel kind (as traced by the library) -> (kernel name pattern, source files)
KINDS = {
    "tilesort": (r"k_tilesort<", ["tilesort.hip", "merge_tile.hpp", "vmps_internal.hpp"]),
    "level_merge": (r"k_level_merge<", ["merge.hip", "merge_tile.hpp", "vmps_internal.hpp"]),
    "level_partition": (r"k_level_partition<", ["merge.hip", "vmps_internal.hpp"]),
    "scatter": (r"k_part_scatter[12]<", ["learned.hip", "vmps_internal.hpp"]),
    "histogram": (r"k_part_hist1<", ["learned.hip", "vmps_internal.hpp"]),
    "train": (r"k_cdf_step<", ["learned.hip", "vmps_internal.hpp"]),
    "vm_round": (r"k_vm_round<", ["vm.hip", "merge_tile.hpp", "vmps_internal.hpp"]),
    "vm_copy": (r"k_vm_copy_move<", ["vm.hip", "vmps_internal.hpp"]),
    "rec_gather": (r"k_rec_gather<", ["records.hip", "vmps_internal.hpp"]),
}
COPY_PATTERN = r"copyBuffer"


def source_hashes(kind: str) -> dict:
    out = {}
    for f in KINDS[kind][1]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            out[f] = hashlib.sha256(fh.read()).hexdigest()
    return out


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def _short(name: str) -> str:
    name = re.sub(r"\(.*", "", name).replace("void ", "")
    return name.replace("unsigned long", "u64").replace("unsigned int", "u32")


def stats(directory: str, out: str, title: str, command: str) -> None:
    path = _one(os.path.join(directory, "**", "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    lines = [f"# rocprofv3 kernel stats: {title}", f"# command (repo root): {command}",
             "# kernel | calls | total_ms | average_us | percent"]
    for r in rows[:40]:
        lines.append(f"{_short(r['Name'])[:110]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _all_counters(directory: str) -> dict:
    """counter -> list of per-dispatch records (summed over the counter's
    hardware instances)."""
    path = _one(os.path.join(directory, "**", "*counter_collection.csv"))
    per = {}
    for r in csv.DictReader(open(path)):
        d = per.setdefault((r["Counter_Name"], r["Dispatch_Id"]),
                           {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"]), "value": 0.0})
        d["value"] += float(r["Counter_Value"])
    out = {}
    for (c, _), rec in per.items():
        out.setdefault(c, []).append(rec)
    return out


def counters(dirs: list, out: str, kind: str, commands: list) -> dict:
    pat = re.compile(KINDS[kind][0])
    per_launch, launches = {}, {}
    for d in dirs:
        for c, recs in _all_counters(d).items():
            v = [r["value"] for r in recs if pat.search(r["name"])]
            if v:
                per_launch[c] = sum(v) / len(v)
                launches[c] = len(v)
    if not per_launch:
        raise ValueError(f"no dispatch matches {KINDS[kind][0]}")
    res = {"kind": kind, "kernel_pattern": KINDS[kind][0], "per_launch": per_launch, "launches_counted": launches,
           "sources": source_hashes(kind), "commands": commands}
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    return res


def _counters(directory: str, counter: str) -> list:
    path = _one(os.path.join(directory, "**", "*counter_collection.csv"))
    per = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = per.setdefault(r["Dispatch_Id"], {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"]), "kib": 0.0})
        d["kib"] += float(r["Counter_Value"])
    return list(per.values())


def _largest_copies(recs: list) -> list:
    """The runtime's copy dispatches of the largest grid: the known-size
    copies (small readbacks also use the copy kernel)."""
    copies = [r for r in recs if re.search(COPY_PATTERN, r["name"])]
    if not copies:
        raise ValueError("no copy dispatch to calibrate against")
    g = max(r["grid"] for r in copies)
    return [r for r in copies if r["grid"] == g]


def traffic(fetch_dir: str, write_dir: str, out: str, kind: str, copy_bytes: int, commands: list,
            calibrate: list = None) -> dict:
    """calibrate: (fetch_dir, write_dir) of another run whose largest copies
    are all of copy_bytes (when this run's copies differ in size)."""
    pat = re.compile(KINDS[kind][0])
    fetch = _counters(fetch_dir, "FETCH_SIZE")
    write = _counters(write_dir, "WRITE_SIZE")
    cal_f = _counters(calibrate[0], "FETCH_SIZE") if calibrate else fetch
    cal_w = _counters(calibrate[1], "WRITE_SIZE") if calibrate else write

    def avg(recs, p):
        v = [r["kib"] * 1024.0 for r in recs if p.search(r["name"])]
        if not v:
            raise ValueError(f"no dispatch matches {p.pattern}")
        return sum(v) / len(v), len(v)

    anything = re.compile(".")
    cf, _ = avg(_largest_copies(cal_f), anything)
    cw, _ = avg(_largest_copies(cal_w), anything)
    sf, sw = copy_bytes / cf, copy_bytes / cw
    f, nf = avg(fetch, pat)
    w, nw = avg(write, pat)
    res = {
        "kind": kind,
        "kernel_pattern": KINDS[kind][0],
        "launches_counted": [nf, nw],
        "fetch_bytes_per_launch": f * sf,
        "write_bytes_per_launch": w * sw,
        "traffic_bytes_per_launch": f * sf + w * sw,
        "scale_fetch": sf,
        "scale_write": sw,
        "calibration": f"device copy of {copy_bytes} bytes: FETCH_SIZE x{sf:.3f}, WRITE_SIZE x{sw:.3f}"
                       + (f" (copies of the runs in {calibrate[0]}, {calibrate[1]})" if calibrate else ""),
        "sources": source_hashes(kind),
        "commands": commands,
    }
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    return res


def load_traffic(path: str):
    """Bytes per launch from a traffic JSON, or None when the kernel's source
    has changed since the counters were taken (or the file is missing)."""
    try:
        with open(path) as fh:
            t = json.load(fh)
        if t["sources"] != source_hashes(t["kind"]):
            return None
        return t
    except (OSError, KeyError, ValueError):
        return None


def load_counters(path: str):
    """Per-launch SQ counters from a counters JSON, or None when the
    kernel's source has changed since they were taken (or it is missing)."""
    return load_traffic(path)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2605_27147_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("out")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kind", required=True, choices=sorted(KINDS))
    c.add_argument("--command", action="append", default=[])
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("out")
    t.add_argument("--kind", required=True, choices=sorted(KINDS))
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--calibrate", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        stats(a.dir, a.out, a.title, a.command)
    elif a.cmd == "counters":
        r = counters(a.dirs, a.out, a.kind, a.command)
        print(json.dumps(r["per_launch"]))
    else:
        r = traffic(a.fetch_dir, a.write_dir, a.out, a.kind, a.copy_bytes, a.command, a.calibrate)
        print(json.dumps({k: r[k] for k in ("kind", "traffic_bytes_per_launch", "calibration")}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
