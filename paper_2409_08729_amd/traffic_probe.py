"""HBM traffic probe for counter runs.

Dispatches, in order: (1) a plain device copy of 2^26 float64 (512 MiB read,
512 MiB written; torch's copy kernel), then (2) one lbessel_log_kv_f64 launch
on the 2^26-pair stress grid (algorithmic traffic 24 B per pair = 1.5 GiB).
Run once per counter, e.g.

    rocprofv3 --pmc FETCH_SIZE -d <dir> -o fetch --output-format csv \
        -- python -m paper_2409_08729_amd.traffic_probe

The copy's reading calibrates the counter (bytes it reports per byte moved).
"""
import torch

import paper_2409_08729_amd as lb
from paper_2409_08729_amd import workloads as wl


def main() -> None:
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
    main()
