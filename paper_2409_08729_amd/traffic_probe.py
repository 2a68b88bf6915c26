"""HBM traffic probe for counter runs.

Dispatches, in order: (1) a plain device copy of 2^26 float64 (512 MiB read,
512 MiB written; torch's copy kernel), then (2) one lbessel_log_kv_f64 launch
on the 2^26-pair stress grid (algorithmic traffic 24 B per pair = 1.5 GiB).
Run once per counter, e.g.

    rocprofv3 --pmc FETCH_SIZE -d <dir> -o fetch --output-format csv \
        -- python -m paper_2409_08729_amd.traffic_probe

The copy's reading calibrates the counter (bytes it reports per byte moved).
After both runs,

    python -m paper_2409_08729_amd.traffic_probe --reduce <fetch csv> <write csv> <out.json>

writes the per-launch HBM bytes with the sha256 of the kernel sources they
were taken on (the benchmark reports them only while the sources match).
"""
import hashlib
import json
import re
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ["paper_2409_08729_amd/csrc/lbessel_device.hpp",
           "paper_2409_08729_amd/csrc/lbessel_kernels.hip",
           "paper_2409_08729_amd/csrc/lbessel_fastmath.hpp",
           "paper_2409_08729_amd/csrc/lbessel_tables.h"]
COPY_BYTES = (1 << 26) * 8


def source_sha256() -> str:
    h = hashlib.sha256()
    for src in SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def _read(csv_path: str, counter: str):
    import csv
    copy, launch = None, None
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            name, val = row["Kernel_Name"], float(row["Counter_Value"])
            if "copyBuffer" in name:             # the runtime's device-to-device copy
                copy = val
            elif re.search(r"k_grouped<double, 1, 0(, 0)?>", name):
                launch = val
    if copy is None or launch is None:
        raise SystemExit(f"{csv_path}: copy or log K dispatch not found for {counter}")
    return copy, launch


def reduce(fetch_csv: str, write_csv: str, out_json: str) -> dict:
    cf, lf = _read(fetch_csv, "FETCH_SIZE")
    cw, lw = _read(write_csv, "WRITE_SIZE")
    ff = COPY_BYTES / (cf * 1024.0)
    fw = COPY_BYTES / (cw * 1024.0)
    n = 1 << 26
    rec = {"kernel": "k_grouped<double, K, log> (lbessel_log_kv_f64)",
           "launch": "2^26-pair stress grid", "source_sha256": source_sha256(),
           "sources": SOURCES, "fetch_kib": lf, "write_kib": lw, "copy_fetch_kib": cf,
           "copy_write_kib": cw, "copy_bytes_each_way": COPY_BYTES, "fetch_factor": ff,
           "write_factor": fw, "hbm_bytes_per_launch": lf * 1024.0 * ff + lw * 1024.0 * fw,
           "hbm_read_bytes_per_launch": lf * 1024.0 * ff,
           "hbm_write_bytes_per_launch": lw * 1024.0 * fw,
           "algorithmic_bytes_per_launch": 24 * n}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def main() -> None:
    import torch

    import paper_2409_08729_amd as lb
    from paper_2409_08729_amd import workloads as wl
    n = 1 << 26
    a = torch.empty(n, dtype=torch.float64, device="cuda:0").uniform_()
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy: {n * 8} bytes read, {n * 8} bytes written", flush=True)
    del a, b
    v, x = wl.m3()
    dv = torch.from_numpy(v).to("cuda:0")
    dx = torch.from_numpy(x).to("cuda:0")
    torch.cuda.synchronize()
    lb.log_kv(dv, dx)
    torch.cuda.synchronize()
    print(f"log_kv_f64: {dv.numel()} pairs, algorithmic {24 * dv.numel()} bytes", flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--reduce":
        print(json.dumps(reduce(*sys.argv[2:5]), indent=1))
    else:
        main()
