"""HBM traffic of the CG-iteration kernels from rocprofv3 counter runs.

Two `rocprofv3 --pmc` runs of the same bench command, one with FETCH_SIZE and
one with WRITE_SIZE (KiB per dispatch), each begin with an elementwise copy of
known size (`bench.py --copy-probe MIB`: MIB MiB read and MIB MiB written per
launch).  What the counters report for that copy, against its known bytes,
gives one scale factor per counter; the per-dispatch means of every hot kernel
are scaled by it.  The record is written into a short text summary under
profiles/ together with a fingerprint of the kernel sources, and bench.py
reports the traffic of its dominant kernel only while the sources still
match that fingerprint.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
KERNEL_SOURCES = ["fft_device.hpp", "fft_static.hpp", "kernel_bodies.hpp", "kernels.hpp",
                  "kernels.hip", "static_table.hpp", "kernels_static_f32.hip",
                  "kernels_static_f64.hip"]
RECORD_TAG = "traffic-record:"

# slot -> (kernel name prefixes, suffix or None) of the FP32 CG iteration;
# a slot may list several such pairs
SLOTS = {
    "expand0": (("hom::k_col_expand<float", "hom::k_col_expand_r2<float"), None),
    "inv1": (("hom::k_col_plain<float", "hom::k_col_reg2<float", "hom::k_col_mid2<float"), ", 1>"),
    "row": [(("hom::k_row<float",), ", 0>"), (("hom::k_row_multi<float",), None)],
    "fwd1": (("hom::k_col_plain<float", "hom::k_col_reg2<float", "hom::k_col_mid2<float"), ", -1>"),
    "project0": (("hom::k_col_project<float", "hom::k_col_project_r2<float"), None),
    "update": (("hom::k_cg_update<float>",), None),
    "direction": (("hom::k_cg_direction<float>",), None),
}


def fingerprint() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _slot_of(name: str):
    head = name[5:] if name.startswith("void ") else name
    head = head.split("(")[0].rstrip()
    for slot, rule in SLOTS.items():
        for prefixes, suffix in (rule if isinstance(rule, list) else [rule]):
            if head.startswith(prefixes) and (suffix is None or head.endswith(suffix)):
                return slot
    return None


def _per_kernel(path: str):
    out = {}
    for r in csv.DictReader(open(path)):
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def summarize(fetch_csv: str, write_csv: str, copy_mib: int) -> dict:
    """Per-slot median FETCH/WRITE KiB per dispatch, the copy-probe scale
    factors and the scaled HBM bytes per launch."""
    fe, wr = _per_kernel(fetch_csv), _per_kernel(write_csv)
    probe = [k for k in fe if "neg_kernel" in k]
    if not probe:
        raise ValueError("no copy-probe kernel in the FETCH_SIZE run")
    known_kib = copy_mib * 1024.0
    f_scale = known_kib / statistics.median(fe[probe[0]])
    w_scale = known_kib / statistics.median(wr[[k for k in wr if "neg_kernel" in k][0]])
    slots = {}
    for name in fe:
        slot = _slot_of(name)
        if slot is None or name not in wr:
            continue
        # median over dispatches: launches in which some items had already
        # stopped move less data and would bias a mean low
        f, w = statistics.median(fe[name]), statistics.median(wr[name])
        slots[slot] = {"kernel": name.split("(")[0][:160], "fetch_kib": f, "write_kib": w,
                       "dispatches": len(fe[name]),
                       "bytes": 1024.0 * (f * f_scale + w * w_scale)}
    return {"fetch_scale": f_scale, "write_scale": w_scale, "copy_probe_mib": copy_mib,
            "slots": slots, "fingerprint": fingerprint()}


def write_summary(rec: dict, path: str, workload: str, command: str) -> None:
    rec = dict(rec, workload=workload)
    lines = [f"# HBM traffic per launch, {workload} (FP32 CG iteration kernels)", "",
             "Commands (one counter per run; the copy probe calibrates each counter):", "",
             f"    {command.replace('COUNTER', 'FETCH_SIZE')}",
             f"    {command.replace('COUNTER', 'WRITE_SIZE')}", "",
             f"Copy probe ({rec['copy_probe_mib']} MiB read + written per launch): FETCH_SIZE scale "
             f"{rec['fetch_scale']:.3f}, WRITE_SIZE scale {rec['write_scale']:.3f}.", "",
             "| slot | kernel | FETCH KiB | WRITE KiB | scaled MB per launch |",
             "|---|---|---|---|---|"]
    for slot, v in rec["slots"].items():
        lines.append(f"| {slot} | `{v['kernel'][:90]}` | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} "
                     f"| {v['bytes'] / 1e6:.2f} |")
    lines += ["", f"Kernel source fingerprint: {rec['fingerprint']}", "",
              RECORD_TAG + " " + json.dumps(rec), ""]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


def load(path: str):
    """The record of a summary, or None when absent or taken from other
    kernel sources."""
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith(RECORD_TAG):
            rec = json.loads(line[len(RECORD_TAG):])
            return rec if rec.get("fingerprint") == fingerprint() else None
    return None


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="write the traffic summary of a workload")
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--workload", required=True, help="e.g. pixels-1023x1023_mixed")
    ap.add_argument("--command", required=True, help="the profiled command, COUNTER for the counter")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    write_summary(summarize(a.fetch_csv, a.write_csv, a.copy_mib), a.out, a.workload, a.command)
    print(f"wrote {a.out}")
