"""Hardware-counter probe of the hot-path launches.

Dispatches, in order: a plain device copy of 2^26 float64 (512 MiB read,
512 MiB written; the runtime's copy kernel) that calibrates the byte
counters, then one launch of each entry in LAUNCHES on the benchmark's
inputs.  Run once per counter set, e.g.

    rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_WAVES \\
        SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_SALU GRBM_GUI_ACTIVE \\
        -d <dir> -o valu --output-format csv -- python -m paper_2409_08729_amd.counter_probe
    rocprofv3 --pmc FETCH_SIZE -d <dir> -o fetch --output-format csv -- python -m ...
    rocprofv3 --pmc WRITE_SIZE -d <dir> -o write --output-format csv -- python -m ...

then

    python -m paper_2409_08729_amd.counter_probe --reduce <valu csv> <fetch csv> <write csv> <out.json>

writes, per launch, the VALU busy fraction, the active-lane fraction, VALU
instructions per wave and the HBM bytes read and written (scaled by the
copy's calibration), with the sha256 of the kernel sources the counters were
taken on (the benchmark reports traffic only while the sources match).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ["paper_2409_08729_amd/csrc/lbessel_device.hpp",
           "paper_2409_08729_amd/csrc/lbessel_kernels.hip",
           "paper_2409_08729_amd/csrc/lbessel_fastmath.hpp",
           "paper_2409_08729_amd/csrc/lbessel_tables.h"]
COPY_BYTES = (1 << 26) * 8
XCDS = 8
SIMDS = 1024
# (label, kind, precision, input set, variant): input set "stress" is the
# 2^26-pair grid, "order10" the 20M-pair set at v = 2^10, "order0" at v = 1
LAUNCHES = [
    ("log_kv_f64_stress", "K", 64, "stress", "default"),
    ("log_iv_f64_stress", "I", 64, "stress", "default"),
    ("log_kv_f64_order0", "K", 64, "order0", "default"),
    ("log_iv_f64_order0", "I", 64, "order0", "default"),
    ("log_kv_f64_order10", "K", 64, "order10", "default"),
    ("log_iv_f64_order10", "I", 64, "order10", "default"),
    ("log_kv_f32_stress", "K", 32, "stress", "default"),
    ("log_iv_f32_stress", "I", 32, "stress", "default"),
    ("log_kv_f64_stress_u_integral", "K", 64, "stress", "u_integral"),
]
LIB_KERNELS = ("k_grouped", "k_ungrouped")


def source_sha256() -> str:
    h = hashlib.sha256()
    for src in SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def _dispatches(csv_path: str):
    """{dispatch id: (kernel name, {counter: value})} of one counter run."""
    out: dict = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            d = int(row.get("Dispatch_Id") or row.get("Correlation_Id") or 0)
            name = row["Kernel_Name"]
            out.setdefault(d, (name, {}))[1][row["Counter_Name"]] = float(row["Counter_Value"])
    return out


def _split(csv_path: str):
    """(copy counters, [counters of each library launch in dispatch order])."""
    disp = _dispatches(csv_path)
    copy, lib = None, []
    for d in sorted(disp):
        name, c = disp[d]
        if "copyBuffer" in name and copy is None:
            copy = c
        elif any(k in name for k in LIB_KERNELS):
            lib.append((name, c))
    if copy is None or len(lib) != len(LAUNCHES):
        raise SystemExit(f"{csv_path}: expected the copy and {len(LAUNCHES)} library launches, "
                         f"found copy={copy is not None} and {len(lib)}")
    return copy, lib


def reduce(valu_csv: str, fetch_csv: str, write_csv: str, out_json: str) -> dict:
    _, lv = _split(valu_csv)
    cf, lf = _split(fetch_csv)
    cw, lw = _split(write_csv)
    ff = COPY_BYTES / (cf["FETCH_SIZE"] * 1024.0)
    fw = COPY_BYTES / (cw["WRITE_SIZE"] * 1024.0)
    rec = {"source_sha256": source_sha256(), "sources": SOURCES,
           "copy_fetch_kib": cf["FETCH_SIZE"], "copy_write_kib": cw["WRITE_SIZE"],
           "copy_bytes_each_way": COPY_BYTES, "fetch_factor": ff, "write_factor": fw,
           "launches": {}}
    for (label, kind, prec, inputs, var), (name, c), (_, f), (_, w) in zip(LAUNCHES, lv, lf, lw):
        n = (1 << 26) if inputs == "stress" else 20_000_000
        busy = c["SQ_ACTIVE_INST_VALU"] * 4.0 / (c["GRBM_GUI_ACTIVE"] / XCDS * SIMDS)
        lanes = c["SQ_THREAD_CYCLES_VALU"] / (64.0 * c["SQ_ACTIVE_INST_VALU"])
        rd = f["FETCH_SIZE"] * 1024.0 * ff
        wr = w["WRITE_SIZE"] * 1024.0 * fw
        alg = n * (24 if prec == 64 else 12)
        rec["launches"][label] = {
            "kernel": name, "kind": kind, "precision": prec, "inputs": inputs, "variant": var,
            "pairs": n, "counters": c, "fetch_kib": f["FETCH_SIZE"], "write_kib": w["WRITE_SIZE"],
            "valu_busy": busy, "active_lanes": lanes,
            "valu_per_wave": c["SQ_INSTS_VALU"] / c["SQ_WAVES"],
            "hbm_read_bytes": rd, "hbm_write_bytes": wr, "hbm_bytes": rd + wr,
            "algorithmic_bytes": alg, "traffic_over_algorithmic": (rd + wr) / alg}
    with open(out_json, "w") as fo:
        json.dump(rec, fo, indent=1)
    return rec


def main() -> None:
    import torch

    import paper_2409_08729_amd as lb
    from paper_2409_08729_amd import workloads as wl
    n = 1 << 26
    # the calibration copy comes first: its kernel is the first copyBuffer
    a = torch.empty(n, dtype=torch.float64, device="cuda:0").uniform_()
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy: {n * 8} bytes read, {n * 8} bytes written", flush=True)
    del a, b
    inputs = {}
    v, x = wl.m3()
    inputs[("stress", 64)] = (torch.from_numpy(v).to("cuda:0"), torch.from_numpy(x).to("cuda:0"))
    for k in (0, 10):
        v, x = wl.m2_order(k)
        inputs[(f"order{k}", 64)] = (torch.from_numpy(v).to("cuda:0"),
                                     torch.from_numpy(x).to("cuda:0"))
    inputs[("stress", 32)] = tuple(t.float() for t in inputs[("stress", 64)])
    for label, kind, prec, which, var in LAUNCHES:
        dv, dx = inputs[(which, prec)]
        torch.cuda.synchronize()
        if var == "default":
            (lb.log_iv if kind == "I" else lb.log_kv)(dv, dx)
        else:
            lb.eval_variant(kind, var, "grouped", dv, dx)
        torch.cuda.synchronize()
        print(f"{label}: {dv.numel()} pairs", flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--reduce":
        print(json.dumps(reduce(*sys.argv[2:6]), indent=1))
    else:
        main()
