"""Per-branch VALU instruction counts for the roofline op model.

Probe (GPU): every branch of log I and log K, binary64 and binary32, on 2^18
identical elements, one dispatch per probe point, so that an
instruction-counter run

    rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES -d <dir> -o opcount --output-format csv \
        -- python -m paper_2409_08729_amd.opcount <dir>/opcount_points.json f64,f32,quad

reports the VALU instructions one evaluation issues with no divergence
(per element = SQ_INSTS_VALU / SQ_WAVES: all 64 lanes of every wave run the
same branch on the same input).  The probe writes the integrand node count of
each K fallback point (lbessel_k_nodes) to the JSON file.  The set "quad"
probes the paper's own 600-node integral (the u_integral variant); the set
"int" the integer-order path of the K fallback (orders 0..14, one point with
x <= 2 and one above, where the order-0/1 expansions switch form); the set
"temme" the K fallback's Temme series (x <= 1.25), whose cost is
fitted as setup + per_term x terms + per_step x order steps (terms from
lbessel_k_terms, steps = max(rint(v) - 1, 0)).

Reduce (host):

    python -m paper_2409_08729_amd.opcount --reduce <counter_collection.csv> <points.json>

merges the probed sets into paper_2409_08729_amd/opmodel.json.  The I series
branch is probed at one point (its trip count varies mildly with (v, x)).
The K fallback's integral costs setup + per_node x nodes, fitted by least
squares over eight (binary32) or ten (binary64) points with different node
counts; Temme's series setup + per_term x terms + per_step x order steps,
fitted the same way over its probe points; the fit residuals are recorded.
A launch's algorithmic ops then use each element's own node and term count.
"""
from __future__ import annotations

import csv
import json
import os
import sys

# (precision, kind, branch, v, x): well inside each branch's region; the Debye
# branch at one order per term-count tier (U_13, U_9, U_6, U_4); the K
# fallback at points with different node counts (non-integer orders, x > 1.25:
# integer orders up to 14 take the integer-order path and x <= 1.25 the
# Temme series, both probed apart).
_FB_K64 = [(3.3, 5.0), (0.5, 1.5), (12.3, 1.3), (1.1, 2.5), (6.2, 2.0), (0.1, 3.0),
           (13.7, 10.0), (2.2, 15.0), (9.5, 1.4), (14.4, 4.0)]
# Temme points: term counts ~2..11 (x) times order steps 0..13 (v)
_TM_K64 = [(0.3, 1e-4), (0.3, 0.01), (0.3, 0.3), (0.3, 1.2), (4.4, 1e-3), (4.4, 0.1),
           (4.4, 1.0), (9.7, 1e-4), (9.7, 0.05), (9.7, 1.2), (14.3, 1e-3), (14.3, 0.5),
           (1.6, 0.02), (7.2, 0.7)]
# binary32: orders up to 9 (the binary32 fallback region)
_TM_K32 = [(0.3, 1e-4), (0.3, 0.01), (0.3, 0.3), (0.3, 1.2), (4.4, 1e-3), (4.4, 0.1),
           (4.4, 1.0), (8.7, 1e-4), (8.7, 0.05), (8.7, 1.2), (1.6, 0.02), (7.2, 0.7)]
_FB_K32 = [(3.3, 5.0), (0.5, 1.5), (8.1, 1.3), (1.1, 2.5), (6.2, 2.0), (0.1, 3.0),
           (8.5, 5.0), (2.2, 6.5)]
# integer orders of the K fallback region: 0..14 in binary64, 0..9 in binary32
# (above 9 the binary32 classifier takes the Debye branch at every x)
INT_X = (1.0, 5.0)
INT_MAX = {64: 14, 32: 9}
SETS = {
    "f64": [(64, k, b, v, x) for k in ("I", "K") for b, v, x in
            [(0, 3.0, 40.0), (1, 20.0, 10.0), (1, 40.0, 10.0), (1, 100.0, 10.0),
             (1, 400.0, 10.0)]]
           + [(64, "I", 2, 3.0, 5.0)] + [(64, "K", 2, v, x) for v, x in _FB_K64],
    "f32": [(32, k, b, v, x) for k in ("I", "K") for b, v, x in
            [(0, 3.0, 40.0), (1, 20.0, 10.0), (1, 40.0, 10.0), (1, 100.0, 10.0),
             (1, 400.0, 10.0)]]
           + [(32, "I", 2, 3.0, 5.0)] + [(32, "K", 2, v, x) for v, x in _FB_K32],
    # the paper's integral (eq. log Kv integral) on its 600 nodes, trapezoid +
    # Gregory weights: the u_integral variant on a uniform fallback array (one
    # element per thread, no grouping); the per-element count is the same at
    # every point of the fallback region (fixed node count)
    "quad": [(64, "K", "u_integral", 3.0, 5.0), (64, "K", "u_integral", 0.5, 1e-4)],
    "int": [(p, "K", 2, float(n), x) for p in (64, 32) for x in INT_X
            for n in range(INT_MAX[p] + 1)],
    "temme": [(64, "K", 2, v, x) for v, x in _TM_K64]
             + [(32, "K", 2, v, x) for v, x in _TM_K32],
}
U_TIER_NAMES = {20.0: "u13", 40.0: "u9", 100.0: "u6", 400.0: "u4"}
NAMES = {0: "mu20", 2: "fallback"}
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "opmodel.json")
PROBE_KERNELS = ("k_branch", "k_ungrouped")


def probe(points_json: str, sets: list[str], n: int = 1 << 18) -> None:
    import torch
    import paper_2409_08729_amd as lb
    pts, nodes, terms = [], [], []
    for name in sets:
        for prec, kind, b, v0, x0 in SETS[name]:
            dt = torch.float64 if prec == 64 else torch.float32
            v = torch.full((n,), v0, dtype=dt, device="cuda:0")
            x = torch.full((n,), x0, dtype=dt, device="cuda:0")
            if isinstance(b, str):
                lb.eval_variant(kind, b, "naive", v, x)
            else:
                lb.eval_branch(kind, b, v, x)
            torch.cuda.synchronize()
            c = int(lb.k_nodes(v[:1], x[:1]).item()) if (kind, b) == ("K", 2) else 0
            tm = int(lb.k_terms(v[:1], x[:1]).item()) if (kind, b) == ("K", 2) else 0
            pts.append([name, prec, kind, b, v0, x0])
            nodes.append(c)
            terms.append(tm)
            print(f"{name}: {kind} branch {b} at v={v0} x={x0}: {n} elements, {c} nodes, "
                  f"{tm} series terms", flush=True)
    with open(points_json, "w") as f:
        json.dump({"points": pts, "nodes": nodes, "terms": terms}, f)


def reduce(path: str, points_json: str) -> dict:
    """Merge the probed sets into opmodel.json (sets not probed are kept)."""
    import numpy as np
    meta = json.load(open(points_json))
    pts, nodes = meta["points"], meta["nodes"]
    terms = meta.get("terms", [0] * len(pts))
    rows = list(csv.DictReader(open(path)))
    disp: dict = {}
    for r in rows:
        name = r.get("Kernel_Name", "")
        if not any(k in name for k in PROBE_KERNELS):
            continue
        d = int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0)
        disp.setdefault(d, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    ids = sorted(disp)
    if len(ids) != len(pts):
        raise SystemExit(f"expected {len(pts)} probe dispatches, found {len(ids)}")
    model = json.load(open(OUT)) if os.path.exists(OUT) else {}
    model["_doc"] = ("VALU instructions per evaluation of each branch (no divergence): "
                     "SQ_INSTS_VALU / SQ_WAVES of the probe dispatches of "
                     "paper_2409_08729_amd/opcount.py.  K fallback: setup + per_node x nodes "
                     "(least squares over the probe points).  quad600_per_eval: the paper's "
                     "600-node integral (u_integral variant), per fallback evaluation.  "
                     "int_le2 / int_gt2: the integer-order path of the K fallback, per order "
                     "0.. (x <= 2 and x > 2).  temme_setup + temme_per_term x terms + "
                     "temme_per_step x max(rint(v) - 1, 0): the binary64 Temme series.")
    fbs: dict = {}
    tms: dict = {}
    for d, (name, prec, kind, b, v0, x0), c, tm in zip(ids, pts, nodes, terms):
        per = disp[d]["SQ_INSTS_VALU"] / disp[d]["SQ_WAVES"]
        key = f"{kind}_f{prec}"
        if name == "quad":
            model.setdefault(key, {}).setdefault("quad600_probes", [])
            model[key]["quad600_probes"] = [q for q in model[key]["quad600_probes"]
                                            if (q["v"], q["x"]) != (v0, x0)]
            model[key]["quad600_probes"].append({"v": v0, "x": x0, "valu": per})
            model[key]["quad600_per_eval"] = float(np.mean(
                [q["valu"] for q in model[key]["quad600_probes"]]))
            continue
        if name == "temme":
            tms.setdefault(key, []).append((tm, max(round(v0) - 1, 0), per, v0, x0))
            continue
        if name == "int":
            lst = model.setdefault(key, {}).setdefault("int_le2" if x0 <= 2.0 else "int_gt2", [])
            lst.extend([None] * (int(v0) + 1 - len(lst)))
            lst[int(v0)] = per
            continue
        if (kind, b) == ("K", 2):
            fbs.setdefault(key, []).append((c, per, v0, x0))
        elif b == 1:
            model.setdefault(key, {})[U_TIER_NAMES[v0]] = per
        else:
            model.setdefault(key, {})[NAMES[b]] = per
    for key, fb in fbs.items():
        A = np.array([[1.0, c] for c, _, _, _ in fb])
        y = np.array([p for _, p, _, _ in fb])
        (setup, per_node), *_ = np.linalg.lstsq(A, y, rcond=None)
        model[key]["fallback_setup"] = float(setup)
        model[key]["fallback_per_node"] = float(per_node)
        model[key]["fallback_probes"] = [
            {"v": v0, "x": x0, "nodes": c, "valu": p, "fit": float(setup + per_node * c)}
            for c, p, v0, x0 in fb]
    for key, tp in tms.items():
        A = np.array([[1.0, t, st] for t, st, _, _, _ in tp])
        y = np.array([p for _, _, p, _, _ in tp])
        (setup, per_term, per_step), *_ = np.linalg.lstsq(A, y, rcond=None)
        model[key]["temme_setup"] = float(setup)
        model[key]["temme_per_term"] = float(per_term)
        model[key]["temme_per_step"] = float(per_step)
        model[key]["temme_probes"] = [
            {"v": v0, "x": x0, "terms": t, "steps": st, "valu": p,
             "fit": float(setup + per_term * t + per_step * st)} for t, st, p, v0, x0 in tp]
    with open(OUT, "w") as f:
        json.dump(model, f, indent=1)
    return model


if __name__ == "__main__":
    if len(sys.argv) > 3 and sys.argv[1] == "--reduce":
        print(json.dumps(reduce(sys.argv[2], sys.argv[3]), indent=1))
    else:
        # python -m paper_2409_08729_amd.opcount <points.json> [f64,f32,quad]
        probe(sys.argv[1], (sys.argv[2] if len(sys.argv) > 2 else "f64,f32,quad").split(","))
