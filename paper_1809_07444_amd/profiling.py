"""Counter summaries for the benchmark's roofline entry.

Turns the CSV output of two `rocprofv3 --pmc` runs of `bench.py
--traffic-probe` (one with FETCH_SIZE, one with WRITE_SIZE) into a short text
summary of the bytes beyond L2 per dispatch of each heap kernel, scaled by
what the same counters read for the calibration kernel of known size that
`--traffic-probe` launches (an elementwise add over 64 Mi int32: 256 MiB read,
256 MiB written).  The summary records a hash of the device sources; the
benchmark reports the traffic only while the sources still hash the same.

    python -m paper_1809_07444_amd.profiling --workload gol \\
        --fetch out/pmc_fetch/gol_counter_collection.csv \\
        --write out/pmc_write/gol_counter_collection.csv \\
        --command "<the rocprofv3 commands>" --out profiles/traffic_gol.txt
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CAL_BYTES_KIB = 256 * 1024  # the calibration add reads and writes 256 MiB

# do-all method struct -> the kernel kind the heap's timing reports
METHOD_KIND = {
    "AlivePrep": "gol_alive_prep", "CandPrep": "gol_cand_prep", "AliveUpdate": "gol_alive_update",
    "CandUpdate": "gol_cand_update", "MicroUpdate": "micro_update", "MicroCull": "micro_cull",
    "Choose": "sugar_choose", "Move": "sugar_move", "Eat": "sugar_eat", "Request": "sugar_request",
    "Birth": "sugar_birth", "VisitCount": "visit_count", "DeleteIfMod": "delete_if_mod",
    "FieldGather": "gather", "GolDeleteWorld": "gol_delete_world", "SugarDeleteWorld": "sugar_delete_world",
    "Decide": "traffic_decide", "Drive": "traffic_drive", "BodyForce": "collide_force", "BodyMove": "collide_move",
    "BodyRoot": "collide_root", "BodyTarget": "collide_target", "BodyMerge": "collide_merge",
    "BodyRemove": "collide_remove", "FishDecide": "wator_fish_decide", "FishMove": "wator_fish_move",
    "SharkDecide": "wator_shark_decide", "SharkMove": "wator_shark_move", "FishEaten": "wator_fish_eaten",
    "FishRead": "wator_fish_read", "SharkRead": "wator_shark_read",
}


# two-list do-alls (both methods in one launch) -> kind
METHOD2_KIND = {("AliveUpdate", "CandUpdate"): "gol_update"}


# Kernels outside the do-alls that carry a timing kind: (function name, a
# substring of the argument list that tells same-named kernels apart).
PLAIN_KIND = [
    ("micro_create_kernel", "", "micro_create"), ("gol_init_kernel", "", "gol_init"),
    ("gol_admit_kernel", "", "gol_admit"), ("regrow_kernel", "", "sugar_regrow"),
    ("sugar_admit_kernel", "", "sugar_admit"), ("entry_kernel", "", "traffic_entry"),
    ("traffic_init_kernel", "", "traffic_init"),
    ("collide_init_kernel", "", "collide_init"), ("wator_init_kernel", "", "wator_init"),
    ("tick_kernel", "Sea", "wator_tick"),
]


def kernel_kind(name: str) -> str | None:
    """Kernel kind of a rocprofv3 kernel name, 'calibration' for the add, or None."""
    # Kernels that touch the bitmaps are instantiated per container width: a
    # trailing template argument such as ", 6u" follows the methods, and
    # do-alls may add ", true" / ", false" (the large-heap variant).
    tail = r"(?:,\s*\d+u)?(?:,\s*(?:true|false))?>"
    m2 = re.search(r"doall2_kernel<(?:[\w:]*::|\(anonymous namespace\)::)*(\w+),\s*"
                   r"(?:[\w:]*::|\(anonymous namespace\)::)*(\w+)" + tail, name)
    if m2:
        return METHOD2_KIND.get((m2.group(1), m2.group(2)))
    m = re.search(r"doall_kernel<(?:[\w:]*::|\(anonymous namespace\)::)*(\w+)" + tail, name)
    if m:
        return METHOD_KIND.get(m.group(1))
    if "enumerate_kernel" in name:
        return "enumerate"
    m = re.search(r"(\w+)(?:<[^()]*>)?\((.*)\)\s*$", name)
    if m:
        for fn, arg, kind in PLAIN_KIND:
            if m.group(1) == fn and arg in m.group(2):
                return kind
    if "elementwise" in name and "add" in name.lower():
        return "calibration"
    return None


def source_hash(root: str = ROOT) -> str:
    """SHA-256 over the device sources and the ABI header, in a fixed order."""
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_1809_07444_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".hpp")))
    files.append(os.path.join(root, "include", "dsoar.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _averages(path: str) -> dict:
    tot = collections.defaultdict(lambda: [0, 0.0])
    with open(path) as fh:
        for r in csv.DictReader(fh):
            k = kernel_kind(r["Kernel_Name"])
            if k is None:
                continue
            tot[k][0] += 1
            tot[k][1] += float(r["Counter_Value"])
    return {k: (n, v / n) for k, (n, v) in tot.items()}


def summarize(fetch_csv: str, write_csv: str) -> dict:
    f, w = _averages(fetch_csv), _averages(write_csv)
    if "calibration" not in f or "calibration" not in w:
        raise ValueError("no calibration kernel in the counter files (run bench.py with --traffic-probe)")
    ff = CAL_BYTES_KIB / f["calibration"][1]
    fw = CAL_BYTES_KIB / w["calibration"][1]
    kernels = {}
    for k in sorted(set(f) & set(w) - {"calibration"}):
        kernels[k] = {"dispatches": f[k][0], "fetch_kib": f[k][1], "write_kib": w[k][1],
                      "bytes": (f[k][1] * ff + w[k][1] * fw) * 1024}
    return {"fetch_factor": ff, "write_factor": fw, "kernels": kernels}


def write_summary(path: str, workload: str, s: dict, command: str, src_hash: str) -> None:
    with open(path, "w") as fh:
        fh.write(f"# bytes beyond L2 per dispatch, {workload}\n")
        fh.write(f"# commands: {command}\n")
        fh.write(f"# source-hash {src_hash}\n")
        fh.write(f"# fetch-factor {s['fetch_factor']:.4f} write-factor {s['write_factor']:.4f} "
                 f"(calibration: elementwise add, 256 MiB read + 256 MiB written)\n")
        fh.write("# kernel dispatches fetch_kib write_kib scaled_bytes\n")
        for k, v in s["kernels"].items():
            fh.write(f"{k} {v['dispatches']} {v['fetch_kib']:.1f} {v['write_kib']:.1f} {v['bytes']:.0f}\n")


def read_summary(path: str) -> dict | None:
    """{'source_hash': str, 'kernels': {kind: scaled bytes per dispatch}} or None."""
    if not os.path.exists(path):
        return None
    out = {"source_hash": None, "kernels": {}}
    with open(path) as fh:
        for line in fh:
            if line.startswith("# source-hash "):
                out["source_hash"] = line.split()[2]
            elif line.strip() and not line.startswith("#"):
                parts = line.split()
                out["kernels"][parts[0]] = float(parts[4])
    return out


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--workload", required=True)
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--command", required=True)
    p.add_argument("--out", required=True)
    a = p.parse_args()
    s = summarize(a.fetch, a.write)
    write_summary(a.out, a.workload, s, a.command, source_hash())
    print(open(a.out).read())


if __name__ == "__main__":
    main()
