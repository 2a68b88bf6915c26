"""Per-branch VALU instruction counts for the roofline op model.

Probe (GPU): every branch of log I and log K (f64) on 2^18 identical
elements, one dispatch per branch, so that an instruction-counter run

    rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES -d <dir> -o opcount --output-format csv \
        -- python -m paper_2409_08729_amd.opcount

reports the VALU instructions one evaluation issues with no divergence
(per element = SQ_INSTS_VALU / SQ_WAVES: all 64 lanes of every wave run the
same branch on the same input).  Dispatch order: I mu20, I u13, I series,
K mu20, K u13, K integral.

Reduce (host):

    python -m paper_2409_08729_amd.opcount --reduce <counter_collection.csv>

writes paper_2409_08729_amd/opmodel.json.  The series branch of I is probed
at one point (its trip count varies with (v, x)); the integral branch of K,
which dominates every K launch, has a fixed trip count (600 nodes).
"""
from __future__ import annotations

import csv
import json
import os
import sys

POINTS = [  # (kind, branch, v, x): well inside each branch's region
    ("I", 0, 3.0, 40.0), ("I", 1, 40.0, 10.0), ("I", 2, 3.0, 5.0),
    ("K", 0, 3.0, 40.0), ("K", 1, 40.0, 10.0), ("K", 2, 3.0, 5.0),
]
NAMES = {0: "mu20", 1: "u13", 2: "fallback"}
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "opmodel.json")


def probe(n: int = 1 << 18) -> None:
    import torch
    import paper_2409_08729_amd as lb
    for kind, b, v0, x0 in POINTS:
        v = torch.full((n,), v0, dtype=torch.float64, device="cuda:0")
        x = torch.full((n,), x0, dtype=torch.float64, device="cuda:0")
        lb.eval_branch(kind, b, v, x)
        torch.cuda.synchronize()
        print(f"{kind} branch {b} at v={v0} x={x0}: {n} elements", flush=True)


def reduce(path: str) -> dict:
    rows = list(csv.DictReader(open(path)))
    disp: dict = {}
    for r in rows:
        name = r.get("Kernel_Name", "")
        if "k_branch" not in name:
            continue
        d = int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0)
        disp.setdefault(d, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    ids = sorted(disp)
    if len(ids) != len(POINTS):
        raise SystemExit(f"expected {len(POINTS)} k_branch dispatches, found {len(ids)}")
    model = {"_doc": "VALU instructions per evaluation of each branch (binary64, no "
                     "divergence): SQ_INSTS_VALU / SQ_WAVES of the probe dispatches of "
                     "paper_2409_08729_amd/opcount.py.",
             "I_f64": {}, "K_f64": {}}
    for d, (kind, b, v0, x0) in zip(ids, POINTS):
        c = disp[d]
        model[f"{kind}_f64"][NAMES[b]] = c["SQ_INSTS_VALU"] / c["SQ_WAVES"]
    with open(OUT, "w") as f:
        json.dump(model, f, indent=1)
    return model


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--reduce":
        print(json.dumps(reduce(sys.argv[2]), indent=1))
    else:
        probe()
