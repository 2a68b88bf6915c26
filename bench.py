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


TRAFFIC = os.path.join(ROOT, "profiles", "traffic_log_kv_f64_stress.json")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def traffic_per_launch():
    """HBM bytes of one stress-grid log K launch from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None if the kernel sources changed
    since those counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC):
        return None
    t = json.load(open(TRAFFIC))
    h = hashlib.sha256()
    for src in t["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != t["source_sha256"]:
        return None
    return t["hbm_bytes_per_launch"]


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


def cpu_baseline(sets_host, seconds_target=12.0):
    """The binary128 oracle on a uniform random sample of the same workload
    (equal share per set, doubling until ~seconds_target of work)."""
    from oracle import oracle
    rng = np.random.default_rng(5)
    per_set, total_pairs, total_t = 64, 0, 0.0
    while total_t < seconds_target and per_set <= 1 << 16:
        vs, xs = [], []
        for v, x in sets_host:
            idx = rng.integers(0, v.size, per_set)
            vs.append(v[idx])
            xs.append(x[idx])
        v = np.concatenate(vs)
        x = np.concatenate(xs)
        t = time.perf_counter()
        oracle.log_iv(v, x)
        oracle.log_kv(v, x)
        total_t += time.perf_counter() - t
        total_pairs += v.size
        per_set *= 2
    n = 2 * total_pairs
    return {"value": n / total_t / 1e9, "unit": "G evals/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{total_pairs} pairs drawn uniformly, equal share from each of the 12 sets "
                      f"(11 orders + stress grid), log I and log K each, binary128, "
                      f"{total_t:.1f} s"}


def vmf_bench(lb, torch, n=50_000, dims=(2048, 8192, 32768)):
    """vMF fit on synthetic features (N rows |g|, g ~ N(mu, 0.5^2 I)): the
    mean-resultant kernels (two HBM passes over X) and the kappa solve."""
    from paper_2409_08729_amd import vmf, workloads as wl
    out = {}
    for p in dims:
        X = wl.vmf_features(n, p, seed=p, device="cuda:0")
        vmf.mean_resultant(X)
        torch.cuda.synchronize()
        reps = 5
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            colsum, sumsq = lb.vmf_colsum(X)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        R = (sumsq.item() ** 0.5) / n
        t = time.perf_counter()
        ks = vmf.kappa_estimates(R, p)
        t_newton = time.perf_counter() - t
        t = time.perf_counter()
        k_lbfgs = vmf.fit_kappa_lbfgs(R, p)
        t_lbfgs = time.perf_counter() - t
        nbytes = 2 * X.numel() * 4          # row-norm pass + column-sum pass
        out[str(p)] = {"N": n, "colsum_ms": ms, "hbm_GBs": nbytes / ms / 1e6,
                       "hbm_frac": nbytes / ms / 1e6 / 8000.0, "R": R,
                       "kappa_0": ks[0], "kappa_1": ks[1], "kappa_2": ks[2] if len(ks) > 2 else None,
                       "kappa": ks[-1], "newton_steps": len(ks) - 1, "newton_s": t_newton,
                       "kappa_lbfgs": k_lbfgs, "lbfgs_s": t_lbfgs}
        del X, colsum, sumsq
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--no-vmf", action="store_true")
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

    # roofline of the dominant kernel: log K f64, on its largest launch (the
    # stress grid); op model = per-branch VALU instructions x branch counts
    mix = op_counts(lb, torch, sets)
    om = json.load(open(OPMODEL))
    ck = om["K_f64"]

    def k_ops(j):
        c = mix[(j, "K")]
        return c[0] * ck["mu20"] + c[1] * ck["u13"] + c[2] * ck["fallback"]

    js = len(sets) - 1
    ops = k_ops(js)
    dur = float(np.mean(per[(sets[js][0], "K")])) * 1e-3
    achieved = ops / dur / 1e12
    all_ops = sum(k_ops(j) for j in range(len(sets)))
    all_dur = sum(float(np.mean(per[(nm, "K")])) for nm, _, _ in sets) * 1e-3
    roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic_per_launch(),
            "kernel": "k_grouped<double, K, log> (lbessel_log_kv_f64)",
            "launch": f"{sets[js][0]}: {sets[js][1].numel()} pairs",
            "ops_per_launch": ops, "launch_ms": dur * 1e3,
            "branch_counts": dict(zip(("mu20", "u13", "fallback", "special"), mix[(js, "K")])),
            "algorithmic_bytes_per_launch": 24 * sets[js][1].numel(),
            "all_K_launches": {"frac": all_ops / all_dur / 1e12 / VALU_PEAK_TOPS,
                               "ms": all_dur * 1e3}}

    kern = {}
    for (name, kind), ts in per.items():
        n = [v.numel() for nm, v, _ in sets if nm == name][0]
        kern[f"{kind}:{name}"] = {"ms": float(np.mean(ts)), "G_evals_s": n / np.mean(ts) / 1e6}
    i_ms = sum(np.mean(ts) for (nm, kd), ts in per.items() if kd == "I")
    k_ms = sum(np.mean(ts) for (nm, kd), ts in per.items() if kd == "K")

    # grouping ablation: the same launches without regrouping by branch
    ablation = {}
    for name, v, x in (sets[0], sets[-1]):
        for kind in ("I", "K"):
            lb.eval_ungrouped(kind, v, x)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            lb.eval_ungrouped(kind, v, x)
            e1.record()
            torch.cuda.synchronize()
            ung = e0.elapsed_time(e1)
            grp = float(np.mean(per[(name, kind)]))
            ablation[f"{kind}:{name}"] = {"grouped_ms": grp, "ungrouped_ms": ung,
                                          "speedup": ung / grp}

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

    vmf_res = None
    if not args.no_vmf:
        vmf_res = vmf_bench(lb, torch)

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
        "grouping_ablation": ablation,
        "vmf": vmf_res,
        "kernels": kern,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
