"""Per-branch VALU instruction counts for the roofline op model.

Probe (GPU): every branch of log I and log K (f64) on 2^18 identical
elements, one dispatch per probe point, so that an instruction-counter run

    rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES -d <dir> -o opcount --output-format csv \
        -- python -m paper_2409_08729_amd.opcount <dir>/opcount_points.json

reports the VALU instructions one evaluation issues with no divergence
(per element = SQ_INSTS_VALU / SQ_WAVES: all 64 lanes of every wave run the
same branch on the same input).  The probe writes the integrand node count of
each K fallback point (lbessel_k_nodes) to the JSON file.

Reduce (host):

    python -m paper_2409_08729_amd.opcount --reduce <counter_collection.csv> <points.json>

writes paper_2409_08729_amd/opmodel.json.  The I series branch is probed at
one point (its trip count varies mildly with (v, x)).  The K fallback's cost
is setup + per_node x nodes, fitted by least squares over three points with
different node counts (the fit residual is recorded); a launch's algorithmic
ops then use each element's own node count.
"""
from __future__ import annotations

import csv
import json
import os
import sys

POINTS = [  # (kind, branch, v, x): well inside each branch's region; the Debye
    # branch at one order per term-count tier (U_13, U_9, U_6, U_4)
    ("I", 0, 3.0, 40.0), ("I", 1, 20.0, 10.0), ("I", 1, 40.0, 10.0), ("I", 1, 100.0, 10.0),
    ("I", 1, 400.0, 10.0), ("I", 2, 3.0, 5.0),
    ("K", 0, 3.0, 40.0), ("K", 1, 20.0, 10.0), ("K", 1, 40.0, 10.0), ("K", 1, 100.0, 10.0),
    ("K", 1, 400.0, 10.0),
    ("K", 2, 3.0, 5.0), ("K", 2, 0.5, 1e-4), ("K", 2, 12.0, 0.01),
]
U_TIER_NAMES = {20.0: "u13", 40.0: "u9", 100.0: "u6", 400.0: "u4"}
NAMES = {0: "mu20", 2: "fallback"}
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "opmodel.json")


def probe(points_json: str | None, n: int = 1 << 18) -> None:
    import torch
    import paper_2409_08729_amd as lb
    nodes = []
    for kind, b, v0, x0 in POINTS:
        v = torch.full((n,), v0, dtype=torch.float64, device="cuda:0")
        x = torch.full((n,), x0, dtype=torch.float64, device="cuda:0")
        lb.eval_branch(kind, b, v, x)
        torch.cuda.synchronize()
        c = int(lb.k_nodes(v[:1], x[:1]).item()) if (kind, b) == ("K", 2) else 0
        nodes.append(c)
        print(f"{kind} branch {b} at v={v0} x={x0}: {n} elements, {c} nodes", flush=True)
    if points_json:
        with open(points_json, "w") as f:
            json.dump({"points": POINTS, "nodes": nodes}, f)


def reduce(path: str, points_json: str) -> dict:
    import numpy as np
    nodes = json.load(open(points_json))["nodes"]
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
                     "paper_2409_08729_amd/opcount.py.  K fallback: setup + per_node x "
                     "nodes (least squares over the probe points).",
             "I_f64": {}, "K_f64": {}}
    fb = []
    for d, (kind, b, v0, x0), c in zip(ids, POINTS, nodes):
        per = disp[d]["SQ_INSTS_VALU"] / disp[d]["SQ_WAVES"]
        if (kind, b) == ("K", 2):
            fb.append((c, per, v0, x0))
        elif b == 1:
            model[f"{kind}_f64"][U_TIER_NAMES[v0]] = per
        else:
            model[f"{kind}_f64"][NAMES[b]] = per
    A = np.array([[1.0, c] for c, _, _, _ in fb])
    y = np.array([p for _, p, _, _ in fb])
    (setup, per_node), *_ = np.linalg.lstsq(A, y, rcond=None)
    model["K_f64"]["fallback_setup"] = float(setup)
    model["K_f64"]["fallback_per_node"] = float(per_node)
    model["K_f64"]["fallback_probes"] = [
        {"v": v0, "x": x0, "nodes": c, "valu": p, "fit": float(setup + per_node * c)}
        for c, p, v0, x0 in fb]
    with open(OUT, "w") as f:
        json.dump(model, f, indent=1)
    return model


if __name__ == "__main__":
    if len(sys.argv) > 3 and sys.argv[1] == "--reduce":
        print(json.dumps(reduce(sys.argv[2], sys.argv[3]), indent=1))
    else:
        probe(sys.argv[1] if len(sys.argv) > 1 else None)
