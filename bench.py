"""Throughput of log I_v(x) and log K_v(x) on one MI355X.

One step = one pass of the whole forward path over the f64 workload:
  * per-order set: v = 2^k, k = 0..10, 20,000,000 values of x ~ U[1, 100)
    each (220M pairs), log I and log K;
  * stress grid: 2^26 pairs, log10 v ~ U[-3, 4], log10 x ~ U[-4, 4],
    log I and log K.
value = pairs evaluated per second over the step (both functions), in
G evals/s, with inputs resident in HBM before timing starts.

Also reported: per-kernel times (HIP events on the launch stream), the
roofline of the dominant kernel (log K f64: plain VALU arithmetic), the f32
path on the same inputs rounded to f32, and the binary128 oracle timed on a
bounded sample on the host cores (cpu_baseline).

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline] [--no-f32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
OPMODEL = os.path.join(ROOT, "paper_2409_08729_amd", "opmodel.json")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def make_inputs(torch, dev):
    from paper_2409_08729_amd import workloads as wl
    sets = []
    for k in range(11):
        v, x = wl.m2_order(k)
        sets.append((f"order_2^{k}", torch.from_numpy(v).to(dev), torch.from_numpy(x).to(dev)))
    v, x = wl.m3()
    sets.append(("stress_2^26", torch.from_numpy(v).to(dev), torch.from_numpy(x).to(dev)))
    return sets


def one_step(lb, torch, sets, outs, timers=None):
    for j, (name, v, x) in enumerate(sets):
        for kind, fn in (("I", lb.log_iv), ("K", lb.log_kv)):
            if timers is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
            outs[(j, kind)] = fn(v, x)
            if timers is not None:
                e1.record()
                timers.append((name, kind, e0, e1))


def op_counts(lb, torch, sets):
    """Branch mix of every set (lbessel_classify) for the op model."""
    mix = {}
    for j, (name, v, x) in enumerate(sets):
        for kind in ("I", "K"):
            b = lb.classify(kind, v, x)
            mix[(j, kind)] = torch.bincount(b.to(torch.int64), minlength=4).cpu().tolist()
    return mix


def cpu_baseline(sets_host, seconds_target=15.0):
    from oracle import oracle
    rng = np.random.default_rng(5)
    vs, xs = [], []
    for v, x in sets_host:
        idx = rng.choice(v.size, 96, replace=False)
        vs.append(v[idx])
        xs.append(x[idx])
    v = np.concatenate(vs)
    x = np.concatenate(xs)
    t = time.perf_counter()
    oracle.log_iv(v, x)
    oracle.log_kv(v, x)
    dt = time.perf_counter() - t
    n = 2 * v.size
    return {"value": n / dt / 1e9, "unit": "G evals/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{v.size} pairs (96 per set: 11 orders + stress grid), log I and log K, "
                      f"binary128, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2409_08729_amd as lb
    lb.lib()
    dev = torch.device("cuda:0")
    log("generating inputs")
    sets = make_inputs(torch, dev)
    n_pairs = sum(v.numel() for _, v, _ in sets)
    outs = {}
    log(f"{n_pairs} pairs resident; warmup {args.warmup}")
    for _ in range(args.warmup):
        one_step(lb, torch, sets, outs)
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps")
    timers = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        one_step(lb, torch, sets, outs, timers)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    evals = 2 * n_pairs
    value = evals * args.steps / wall / 1e9

    # per kernel (HIP events on the launch stream)
    per = {}
    for name, kind, e0, e1 in timers:
        per.setdefault((name, kind), []).append(e0.elapsed_time(e1))
    finite = all(torch.isfinite(o).all().item() for o in outs.values())

    # roofline of the dominant kernel: log K f64
    mix = op_counts(lb, torch, sets)
    roof = None
    if os.path.exists(OPMODEL):
        om = json.load(open(OPMODEL))
        ck = om["K_f64"]
        ops = 0.0
        dur = 0.0
        for j, (name, v, x) in enumerate(sets):
            c = mix[(j, "K")]
            ops += c[0] * ck["mu20"] + c[1] * ck["u13"] + c[2] * ck["fallback"]
            dur += np.mean(per[(name, "K")]) * 1e-3
        achieved = ops / dur / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                "kernel": "k_grouped<double, K, log> (lbessel_log_kv_f64)",
                "ops_per_launch_avg": ops / len(sets), "launch_ms_avg": dur * 1e3 / len(sets)}

    kern = {}
    for (name, kind), ts in per.items():
        n = [v.numel() for nm, v, _ in sets if nm == name][0]
        kern[f"{kind}:{name}"] = {"ms": float(np.mean(ts)), "G_evals_s": n / np.mean(ts) / 1e6}
    i_ms = sum(np.mean(ts) for (nm, kd), ts in per.items() if kd == "I")
    k_ms = sum(np.mean(ts) for (nm, kd), ts in per.items() if kd == "K")

    f32 = None
    if not args.no_f32:
        sets32 = [(nm, v.float(), x.float()) for nm, v, x in sets]
        o32 = {}
        one_step(lb, torch, sets32, o32)
        torch.cuda.synchronize()
        t = time.perf_counter()
        one_step(lb, torch, sets32, o32)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        f32 = {"value": evals / dt / 1e9, "unit": "G evals/s", "ms_per_step": dt * 1e3}
        del sets32, o32

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        host = [(v.cpu().numpy(), x.cpu().numpy()) for _, v, x in sets]
        cpu = cpu_baseline(host)

    line = {
        "metric": "G evals/s log I_v & log K_v (f64)",
        "value": value,
        "unit": "G evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "log I_v and log K_v, f64: 20M pairs per order v=2^0..2^10 with "
                               "x~U[1,100) plus 2^26-pair stress grid (log10 v~U[-3,4], "
                               "log10 x~U[-4,4])",
                   "pairs_per_step": n_pairs, "evals_per_step": evals},
        "roofline": roof,
        "cpu_baseline": cpu,
        "all_finite": finite,
        "ms_I_per_step": i_ms,
        "ms_K_per_step": k_ms,
        "f32": f32,
        "kernels": kern,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
