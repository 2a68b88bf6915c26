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

The serving section replays a seeded Poisson request stream through the
native server (batched vs one launch per request) and reports p50/p99
latency and throughput at several offered loads.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline]
                    [--no-f32] [--no-vmf] [--no-serving]
"""
from __future__ import annotations

import argparse
import gc
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


COUNTERS = os.path.join(ROOT, "profiles", "counters_hot_path.json")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def counters(label: str):
    """Counter record of one launch from the committed probe summary
    (counter_probe.py), or None if the kernel sources changed since the
    counters were taken (or the launch was not probed)."""
    import hashlib
    if not os.path.exists(COUNTERS):
        return None
    t = json.load(open(COUNTERS))
    h = hashlib.sha256()
    for src in t["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != t["source_sha256"]:
        return None
    return t["launches"].get(label)


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
    """One pass of log I and log K over every set; timers, if given, is an
    iterator over pre-created (name, kind, start, end) event records, one per
    launch in this order."""
    for j, (name, v, x) in enumerate(sets):
        for kind, fn in (("I", lb.log_iv), ("K", lb.log_kv)):
            if timers is not None:
                _, _, e0, e1 = next(timers)
                e0.record()
            outs[(j, kind)] = fn(v, x)
            if timers is not None:
                e1.record()


def timed_steps(lb, torch, sets, outs, steps):
    """steps passes between two device synchronisations.  The HIP events of
    every launch are created before the timed region, and the cyclic garbage
    collector is paused inside it (a collection over the bench's objects can
    stall the launching thread for milliseconds).  Returns (wall seconds,
    host seconds to issue the launches, event records)."""
    timers = [(name, kind, torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True))
              for _ in range(steps) for name, _, _ in sets for kind in ("I", "K")]
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = iter(timers)
        for _ in range(steps):
            one_step(lb, torch, sets, outs, it)
        t_issue = time.perf_counter() - t0
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gc.enable()
    return wall, t_issue, timers


# Debye term-count tiers of the library (u_tier in lbessel_device.hpp):
# U_13 up to v = 26, U_9 up to 60, U_6 up to 190, U_4 above
U_TIER_CUTS = (26.0, 60.0, 190.0)


# integer orders of the K fallback that run the integer-order path (x >= 1e-10)
K_INT_ORDER_MAX = 14


def op_counts(lb, torch, sets):
    """Branch mix of every set (lbessel_classify; Debye elements split by
    term-count tier; K fallback elements of integer order 0..14 at x >= 1e-10
    counted per order and side of x = 2) and the total integrand node count of
    the K fallback elements (lbessel_k_nodes) for the op model."""
    mix, nodes = {}, {}
    cuts = torch.tensor(U_TIER_CUTS, dtype=sets[0][1].dtype, device=sets[0][1].device)
    for j, (name, v, x) in enumerate(sets):
        for kind in ("I", "K"):
            b = lb.classify(kind, v, x).to(torch.int64)
            c = torch.bincount(b, minlength=4).cpu().tolist()
            vu = v[b == 1].abs()
            tiers = torch.bucketize(vu, cuts)     # v > cut: 0 = U_13 ... 3 = U_4
            c_u = torch.bincount(tiers, minlength=4).cpu().tolist()
            mix[(j, kind)] = {"mu20": c[0], "u13": c_u[0], "u9": c_u[1], "u6": c_u[2],
                              "u4": c_u[3], "fallback": c[2], "special": c[3]}
            if kind == "K":
                va = v.abs()
                m = (b == 2) & (x >= 1e-10) & (va <= K_INT_ORDER_MAX) & (va == torch.round(va))
                for side, sm in (("int_le2", x <= 2.0), ("int_gt2", x > 2.0)):
                    n_of = va[m & sm].to(torch.int64)
                    mix[(j, kind)][side] = torch.bincount(
                        n_of, minlength=K_INT_ORDER_MAX + 1).cpu().tolist()
                # Temme-series elements: term counts and order steps
                tt = lb.k_terms(v, x).to(torch.int64)
                tm = tt > 0
                steps = (torch.round(va[tm]) - 1).clamp(min=0)
                mix[(j, kind)]["temme"] = int(tm.sum().item())
                mix[(j, kind)]["temme_terms"] = int(tt.sum().item())
                mix[(j, kind)]["temme_steps"] = int(steps.sum().item())
        nodes[j] = int(lb.k_nodes(v, x).to(torch.int64).sum().item())
    return mix, nodes


def k_int_ops(c, ck):
    """Ops and element count of the integer-order K fallback elements of one
    launch (op model entries int_le2 / int_gt2, per order)."""
    ops, cnt = 0.0, 0
    for side in ("int_le2", "int_gt2"):
        per = ck.get(side) or []
        for n, k in enumerate(c.get(side, [])):
            if k:
                if n >= len(per) or per[n] is None:
                    raise SystemExit(f"op model has no {side} entry for order {n}")
                ops += k * per[n]
                cnt += k
    return ops, cnt


def cpu_baseline(sets_host, seconds_target=12.0):
    """The binary128 oracle on a uniform random sample of the same workload
    (equal share per set, doubling until ~seconds_target of work).  Returns
    the baseline record and the sample with its reference values, so the GPU
    outputs of the timed step can be checked on the same points."""
    from oracle import oracle
    rng = np.random.default_rng(5)
    per_set, total_pairs, total_t = 64, 0, 0.0
    sample = []
    while total_t < seconds_target and per_set <= 1 << 16:
        vs, xs, ids = [], [], []
        for j, (v, x) in enumerate(sets_host):
            idx = rng.integers(0, v.size, per_set)
            vs.append(v[idx])
            xs.append(x[idx])
            ids.append((j, idx))
        v = np.concatenate(vs)
        x = np.concatenate(xs)
        t = time.perf_counter()
        ri = oracle.log_iv(v, x)
        rk = oracle.log_kv(v, x)
        total_t += time.perf_counter() - t
        total_pairs += v.size
        sample.append((ids, v, x, ri, rk))
        per_set *= 2
    n = 2 * total_pairs
    rec = {"value": n / total_t / 1e9, "unit": "G evals/s", "cores": oracle.max_threads(),
           "kind": "oracle",
           "sample": f"{total_pairs} pairs drawn uniformly, equal share from each of the 12 sets "
                     f"(11 orders + stress grid), log I and log K each, binary128, "
                     f"{total_t:.1f} s"}
    return rec, sample


def _err_record(v, x, y, hi, lo, tol, kind, deriv=None):
    """Error measures of outputs y against the oracle (hi + lo) at (v, x):
    the parity measure |y - ref| / max(|ref|, 1 + |(v, x)|), the plain relative
    error |y - ref| / |ref| and rel_floor1 = |y - ref| / max(|ref|, 1), with
    decade histograms, and every point whose plain relative error exceeds tol
    listed with |ref|, |(v, x)| and its distance to the nearest zero of the
    log-value in relative x, |ref / (x d ref/dx)| (first order; deriv gives
    the oracle's d/dx at the listed points)."""
    fin = np.isfinite(hi)
    v, x, y, hi, lo = v[fin], x[fin], y[fin], hi[fin], lo[fin]
    d = np.abs((y - hi) - lo)
    cond = d / np.maximum(np.abs(hi), 1.0 + np.hypot(v, x))
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(hi != 0, d / np.abs(hi), 0.0)
    floor1 = d / np.maximum(np.abs(hi), 1.0)
    above = np.nonzero(rel > tol)[0]
    listing = []
    if above.size:
        above = above[np.argsort(-rel[above])]
        dh = deriv(v[above], x[above])[0] if deriv is not None else np.full(above.size, np.nan)
        for k, dk in zip(above, dh):
            listing.append({"v": float(v[k]), "x": float(x[k]), "abs_y": float(abs(hi[k])),
                            "norm_vx": float(np.hypot(v[k], x[k])), "rel_err": float(rel[k]),
                            "cond_err": float(cond[k]), "rel_floor1": float(floor1[k]),
                            "zero_dist_rel_x": float(abs(hi[k] / (x[k] * dk)))})
    return {"kind": kind, "points": int(fin.sum()), "max_cond_err": float(cond.max(initial=0.0)),
            "max_rel_err": float(rel.max(initial=0.0)),
            "max_rel_floor1": float(floor1.max(initial=0.0)),
            "hist_cond_err": histogram(cond), "hist_rel_err": histogram(rel),
            "hist_rel_floor1": histogram(floor1), "rel_err_tol": tol,
            "above_tol": len(listing),
            "above_tol_max_abs_y_over_scale": max(
                (p["abs_y"] / (1.0 + p["norm_vx"]) for p in listing), default=None),
            "above_tol_max_zero_dist_rel_x": max(
                (p["zero_dist_rel_x"] for p in listing), default=None),
            "above_tol_points": listing}


def sample_errors(torch, outs, sample):
    """Errors of the timed step's f64 outputs on the oracle sample, per
    function (_err_record with the binary64 target 4e-15)."""
    from oracle import oracle
    res = {}
    for kind, col in (("I", 3), ("K", 4)):
        vs, xs, ys, his, los = [], [], [], [], []
        for blk in sample:
            ids, v, x = blk[0], blk[1], blk[2]
            hi, lo = blk[col]
            ys.append(np.concatenate([outs[(j, kind)][torch.from_numpy(idx).to(outs[(j, kind)].device)]
                                      .cpu().numpy() for j, idx in ids]))
            vs.append(v)
            xs.append(x)
            his.append(hi)
            los.append(lo)
        res[kind] = _err_record(np.concatenate(vs), np.concatenate(xs), np.concatenate(ys),
                                np.concatenate(his), np.concatenate(los), 4e-15, kind,
                                oracle.dlog_iv if kind == "I" else oracle.dlog_kv)
    return res


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
        lb.vmf_fit(X)
        torch.cuda.synchronize()
        t = time.perf_counter()
        k_dev, _, _, steps_dev = lb.vmf_fit(X)      # column sums + device Newton, result on host
        t_dev = time.perf_counter() - t
        nbytes = 2 * X.numel() * 4          # row-norm pass + column-sum pass
        out[str(p)] = {"N": n, "colsum_ms": ms, "hbm_GBs": nbytes / ms / 1e6,
                       "hbm_frac": nbytes / ms / 1e6 / 8000.0, "R": R,
                       "kappa_0": ks[0], "kappa_1": ks[1], "kappa_2": ks[2] if len(ks) > 2 else None,
                       "kappa": ks[-1], "newton_steps": len(ks) - 1, "newton_s": t_newton,
                       "kappa_lbfgs": k_lbfgs, "lbfgs_s": t_lbfgs,
                       "device_fit": {"kappa": k_dev, "newton_steps": steps_dev,
                                      "ms": t_dev * 1e3}}
        del X, colsum, sumsq
        torch.cuda.empty_cache()
    return out


ABLATIONS = (  # (variant, layout): the paper's own choices put back one at a time
    ("default", "grouped"), ("default", "naive"), ("default", "sorted"),
    ("paper_regimes", "grouped"), ("u_integral", "grouped"), ("simpson", "grouped"),
    ("paper", "grouped"), ("paper", "sorted"), ("paper", "naive"),
    ("seven", "naive"), ("seven", "sorted"),
)


DECADES = [10.0 ** k for k in range(-18, -1)]


def histogram(err):
    """Counts per decade bin of the error: [0, 1e-18), [1e-18, 1e-17), ..., >= 1e-2."""
    edges = np.array(DECADES)
    idx = np.searchsorted(edges, err, side="right")
    counts = np.bincount(idx, minlength=len(edges) + 1)
    labels = ["<1e-18"] + [f"[1e{k},1e{k + 1})" for k in range(-18, -2)] + [">=1e-2"]
    return dict(zip(labels, counts.tolist()))


def f32_errors(torch, sets32, outs32, per_set=1 << 11):
    """Per-result error of the timed binary32 outputs against the oracle at the
    binary32 inputs (widened exactly), on a seeded sample of every set
    (_err_record with the binary32 target 2e-6)."""
    from oracle import oracle
    rng = np.random.default_rng(6)
    res = {}
    for kind in ("I", "K"):
        vs, xs, ys, his, los = [], [], [], [], []
        for j, (name, v, x) in enumerate(sets32):
            idx = torch.from_numpy(rng.integers(0, v.numel(), per_set)).to(v.device)
            hv = v[idx].double().cpu().numpy()
            hx = x[idx].double().cpu().numpy()
            ys.append(outs32[(j, kind)][idx].double().cpu().numpy())
            hi, lo = (oracle.log_iv if kind == "I" else oracle.log_kv)(hv, hx)
            vs.append(hv)
            xs.append(hx)
            his.append(hi)
            los.append(lo)
        res[kind] = _err_record(np.concatenate(vs), np.concatenate(xs), np.concatenate(ys),
                                np.concatenate(his), np.concatenate(los), 2e-6, kind,
                                oracle.dlog_iv if kind == "I" else oracle.dlog_kv)
    return {"sample": f"{per_set} seeded points per set at the binary32 inputs", **res}


def ablation_bench(lb, torch, sets, sample=1 << 13):
    """Time and accuracy of each (variant, layout) on the stress grid and on the
    v = 1 order set, log I and log K (binary64).  Accuracy: largest error on a
    seeded sample of the stress grid against the binary128 oracle."""
    from oracle import oracle
    res = {}
    picks = [sets[0], sets[-1]]
    works = {}
    for name, v, x in picks:
        need = lb.lib().lbessel_eval_variant_workspace(v.numel())
        works[name] = torch.empty(int(need), dtype=torch.uint8, device=v.device)
    rng = np.random.default_rng(11)
    _, vs, xs = sets[-1]
    idx = torch.from_numpy(rng.integers(0, vs.numel(), sample)).to(vs.device)
    sv, sx = vs[idx].contiguous(), xs[idx].contiguous()
    hv, hx = sv.cpu().numpy(), sx.cpu().numpy()
    ref = {"I": oracle.log_iv(hv, hx), "K": oracle.log_kv(hv, hx)}
    den = 1.0 + np.hypot(hv, hx)
    for var, lay in ABLATIONS:
        key = f"{var}/{lay}"
        res[key] = {}
        for kind in ("I", "K"):
            row = {}
            for name, v, x in picks:
                lb.eval_variant(kind, var, lay, v[:4096], x[:4096], works[name])
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                lb.eval_variant(kind, var, lay, v, x, works[name])
                e1.record()
                torch.cuda.synchronize()
                row[f"{name}_ms"] = e0.elapsed_time(e1)
            y = lb.eval_variant(kind, var, lay, sv, sx).cpu().numpy()
            hi, lo = ref[kind]
            fin = np.isfinite(hi)
            d = np.abs((y[fin] - hi[fin]) - lo[fin]) / np.maximum(np.abs(hi[fin]), den[fin])
            row["max_cond_err_stress_sample"] = float(d.max(initial=0.0))
            row["frac_above_4e-15"] = float((d > 4e-15).mean())
            res[key][kind] = row
        log(f"ablation {key} done")
    return {"sample": f"{sample} stress-grid points (seed 11) against the binary128 oracle",
            "results": res}


def order01_bench(lb, torch, n=20_000_000):
    """Orders 0 and 1 (the paper's v = 0, 1 comparisons) and the integer
    orders 2, 4, 8 of the per-order set: the scalar-order path against the
    general path on the same arguments, x ~ U[0, 150) (the paper's Small
    region) and x ~ U[150, 1e4) (Large), binary64."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(20240917)
    res = {}
    for region, lo, hi in (("small", 0.0, 150.0), ("large", 150.0, 1e4)):
        x = torch.rand(n, generator=g, device="cuda:0", dtype=torch.float64) * (hi - lo) + lo
        for v in (0.0, 1.0, 2.0, 4.0, 8.0):
            vv = torch.full_like(x, v)
            for kind in ("I", "K"):
                f_fast = lb.log_iv_order if kind == "I" else lb.log_kv_order
                f_gen = lb.log_iv if kind == "I" else lb.log_kv
                row = {}
                for name, call in (("fast", lambda: f_fast(v, x)), ("general", lambda: f_gen(vv, x))):
                    call()
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(3):
                        call()
                    e1.record()
                    torch.cuda.synchronize()
                    row[f"{name}_ms"] = e0.elapsed_time(e1) / 3
                row["speedup"] = row["general_ms"] / row["fast_ms"]
                row["fast_G_evals_s"] = n / row["fast_ms"] / 1e6
                res[f"{kind}{int(v)}:{region}"] = row
        del x, vv
    return {"n": n, "results": res}


# The paper's own runtime tables (RTX 2080 Ti, binary64; Sec. "Runtime",
# Tables 6 and 7): milliseconds for 10M points per region (Table 6) and 100M
# points at v = 0, 1 (Table 7).  Quoted as context beside this GPU's times on
# the same workloads.
PAPER_TABLE6_MS = {("I", "small"): 50.41, ("I", "large"): 39.68,
                   ("K", "small"): 430.60, ("K", "large"): 39.96}
PAPER_TABLE7_MS = {("I", 0, "small"): 433.00, ("I", 0, "large"): 187.14,
                   ("I", 1, "small"): 336.44, ("I", 1, "large"): 175.59}


def paper_tables_bench(lb, torch):
    """The paper's runtime workloads on this GPU (binary64, inputs resident):
    Table 6: 10M (v, x) pairs uniform in the Small [0,150]^2 and Large
    [150,1e4]^2 ([150,4000]^2 for K) regions; Table 7: 100M x at v = 0 and 1
    in the same x ranges, through the scalar-order entry points."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(20240918)

    def timed(call):
        call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            call()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    t6 = {}
    n = 10_000_000
    for kind in ("I", "K"):
        for region, lo, hi in (("small", 0.0, 150.0),
                               ("large", 150.0, 1e4 if kind == "I" else 4000.0)):
            v = torch.rand(n, generator=g, device="cuda:0", dtype=torch.float64) * (hi - lo) + lo
            x = torch.rand(n, generator=g, device="cuda:0", dtype=torch.float64) * (hi - lo) + lo
            f = lb.log_iv if kind == "I" else lb.log_kv
            ms = timed(lambda: f(v, x))
            t6[f"{kind}:{region}"] = {"ms": ms, "G_evals_s": n / ms / 1e6,
                                      "paper_ms_rtx2080ti": PAPER_TABLE6_MS[(kind, region)],
                                      "ratio_vs_paper": PAPER_TABLE6_MS[(kind, region)] / ms}
            del v, x
    t7 = {}
    n = 100_000_000
    for region, lo, hi in (("small", 0.0, 150.0), ("large", 150.0, 1e4)):
        x = torch.rand(n, generator=g, device="cuda:0", dtype=torch.float64) * (hi - lo) + lo
        for order in (0, 1):
            for kind in ("I", "K"):
                f = lb.log_iv_order if kind == "I" else lb.log_kv_order
                ms = timed(lambda: f(float(order), x))
                row = {"ms": ms, "G_evals_s": n / ms / 1e6}
                if kind == "I":
                    row["paper_ms_rtx2080ti"] = PAPER_TABLE7_MS[("I", order, region)]
                    row["ratio_vs_paper"] = row["paper_ms_rtx2080ti"] / ms
                t7[f"{kind}{order}:{region}"] = row
        del x
    return {"table6_10M": t6, "table7_100M": t7,
            "note": "paper times are the RTX 2080 Ti means of its Tables 6 and 7 (context)"}


def serving_bench(torch, count=1024, loads=(0.25, 0.5, 0.75, 0.9), resident="host"):
    """Open-loop Poisson request stream through the native server: uneven
    evaluation requests (1 .. 4M pairs, I/K, f64/f32) with their arrays in
    pinned host memory (resident="host": copied in and out by the server) or
    on the GPU (resident="device": no copies), and vMF fits (device
    features, p in {2048, 8192, 32768}, N in [1e3, 5e4]).  Saturation = all
    requests offered at once; then offered loads at the given fractions of
    the batched server's saturation rate.  Latency = completion - scheduled
    arrival."""
    from paper_2409_08729_amd import serve, workloads as wl
    reqs, gaps = wl.serving_requests(count)
    v, x = wl.serving_pool()
    dev = resident == "device"

    def place(a):
        t = torch.from_numpy(a)
        return t.to("cuda:0") if dev else t.pin_memory()
    pools = {64: (place(v), place(x)),
             32: (place(v.astype(np.float32)), place(x.astype(np.float32)))}
    feats = {p: wl.vmf_features(wl.SERVE_VMF_ROWS[1], p, seed=p, device="cuda:0")
             for p in wl.SERVE_VMF_DIMS}
    tot = {64: 0, 32: 0}
    for r in reqs:
        if r["type"] == "eval":
            tot[r["precision"]] += r["n"]
    outbuf = {64: torch.empty(tot[64], dtype=torch.float64, pin_memory=not dev,
                              device="cuda:0" if dev else "cpu"),
              32: torch.empty(tot[32], dtype=torch.float32, pin_memory=not dev,
                              device="cuda:0" if dev else "cpu")}
    results = torch.empty((count, 4), dtype=torch.float64, pin_memory=True)
    base, at = [], {64: 0, 32: 0}
    for i, r in enumerate(reqs):
        if r["type"] == "eval":
            pv, px = pools[r["precision"]]
            o, n = r["offset"], r["n"]
            a = at[r["precision"]]
            at[r["precision"]] += n
            base.append({"type": "eval_device" if dev else "eval", "kind": r["kind"],
                         "v": pv[o:o + n], "x": px[o:o + n],
                         "out": outbuf[r["precision"]][a:a + n]})
        else:
            base.append({"type": "vmf", "X": feats[r["p"]][: r["N"]], "result": results[i]})
    pairs = sum(r["n"] for r in reqs if r["type"] == "eval")
    modes = (("batched", "batched", 8), ("plain", "plain", 1), ("plain_8streams", "plain", 8))

    def run(label, times):
        _, mode, streams = [m for m in modes if m[0] == label][0]
        items = [dict(b, t=float(t)) for b, t in zip(base, times)]
        with serve.Server(mode, streams=streams, arena_bytes=4 << 30) as srv:
            infos = srv.replay(items, timeout=600)
            st = srv.stats()
        lat = np.array([i["t_done"] - i["t_arrival"] for i in infos]) * 1e3
        span = max(i["t_done"] for i in infos) - min(i["t_arrival"] for i in infos)
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                "requests_per_s": count / span, "G_evals_s": pairs / span / 1e9,
                "span_s": span, "batches": st["batches"], "kernel_launches": st["kernel_launches"],
                "max_batch_requests": st["max_batch_requests_seen"],
                "arena_peak_MiB": st["arena_peak_bytes"] / 2**20, "queue_peak": st["queue_peak"]}

    zeros = np.zeros(count)
    run("batched", zeros)                                   # warm-up (pages, code objects)
    run("plain", zeros)
    sat = {}
    for label, _, _ in modes:
        log(f"serving ({resident}): saturation, {label}")
        sat[label] = run(label, zeros)
    unit_t = np.cumsum(gaps)
    sweep = []
    for f in loads:
        qps = f * sat["batched"]["requests_per_s"]
        row = {"load": f, "offered_requests_per_s": qps}
        for label, _, _ in modes:
            log(f"serving ({resident}): load {f:.2f} ({qps:.0f} req/s), {label}")
            row[label] = run(label, unit_t / qps)
        sweep.append(row)
    n_vmf = sum(r["type"] == "vmf" for r in reqs)
    return {"requests": count, "eval_requests": count - n_vmf, "vmf_requests": n_vmf,
            "eval_pairs": pairs,
            "resident": resident,
            "mix": "eval: n log-uniform [1, 4M], kind I/K and f64/f32 equally likely, "
                   "log10 v ~ U[-3,4] (1/256 of v = 0), log10 x ~ U[-3,4], "
                   + ("in/out on the device" if dev else "host pinned in/out")
                   + "; vMF (1/8 of requests): p in {2048, 8192, 32768}, N log-uniform "
                   "[1e3, 5e4], features on the device",
            "modes": {"batched": "FIFO memory admission, continuous batching into segmented "
                                 "launches of up to 2^18 pairs, 8 batches in flight",
                      "plain": "same queue, one request at a time, one launch per request",
                      "plain_8streams": "one launch per request, 8 requests in flight"},
            "saturation": sat, "sweep": sweep}


def graph_bench(lb, torch, nseg=16, reps=400):
    """Launch cost of one small serving batch (nseg device-resident requests
    of log-uniform size in [1, 4096], log K f64, one segmented launch with
    the table in the kernel arguments): issued directly through the C-ABI,
    or captured once in a HIP graph and replayed.  Reports host time per
    submission and GPU time per batch for both (the saving a graph-replayed
    batch path could bring), and checks every replay against the eager
    result."""
    import ctypes
    from paper_2409_08729_amd import workloads as wl
    g = np.random.default_rng(41)
    v, x = wl.serving_pool(1 << 16, seed=42)
    dv = torch.from_numpy(v).to("cuda:0")
    dx = torch.from_numpy(x).to("cuda:0")
    lib = lb.lib()
    table = (lb.Segment * nseg)()
    outs, tiles, at = [], 0, 0
    for k in range(nseg):
        n = int(np.exp(g.uniform(0.0, np.log(4096.0))))
        o = torch.empty(n, dtype=torch.float64, device="cuda:0")
        table[k] = lb.Segment(dv[at:].data_ptr(), dx[at:].data_ptr(), o.data_ptr(), n, tiles)
        tiles += lib.lbessel_segment_tiles(n)
        outs.append((o, at, n))
        at += n
    addr = ctypes.addressof(table)
    stream = torch.cuda.current_stream()

    def launch():
        rc = lib.lbessel_eval_segments_inline(1, 64, addr, nseg, tiles, stream.cuda_stream)
        assert rc == 0

    launch()
    torch.cuda.synchronize()
    eager = [o.clone() for o, _, _ in outs]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        host = (time.perf_counter() - t0) / reps
        torch.cuda.synchronize()
        return host * 1e6, e0.elapsed_time(e1) * 1e3 / reps

    direct_host, direct_gpu = timed(launch)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for o, _, _ in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            rc = lib.lbessel_eval_segments_inline(1, 64, addr, nseg, tiles, side.cuda_stream)
            assert rc == 0
    torch.cuda.synchronize()
    same = True
    for _ in range(3):   # replays with eager work and synchronisation between them
        for o, _, _ in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        same = same and all(torch.equal(a.view(torch.int64), o.view(torch.int64))
                            for a, (o, _, _) in zip(eager, outs))
    graph_host, graph_gpu = timed(graph.replay)
    return {"batch": f"{nseg} log K f64 requests, {at} pairs, {tiles} tiles, one launch",
            "direct_host_us": direct_host, "direct_gpu_us_per_batch": direct_gpu,
            "graph_host_us": graph_host, "graph_gpu_us_per_batch": graph_gpu,
            "graph_replays_equal_eager": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--no-vmf", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-tables", action="store_true",
                    help="skip the order-0/1 and paper runtime-table workloads")
    ap.add_argument("--detail", default=None,
                    help="also write the detail record (indented JSON) to this file")
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
    wall, t_issue, timers = timed_steps(lb, torch, sets, outs, args.steps)
    ms_per_step = wall * 1e3 / args.steps
    evals = 2 * n_pairs
    value = evals * args.steps / wall / 1e9

    # per kernel (HIP events on the launch stream)
    per = {}
    for name, kind, e0, e1 in timers:
        per.setdefault((name, kind), []).append(e0.elapsed_time(e1))
    finite = all(torch.isfinite(o).all().item() for o in outs.values())

    mix, knodes = op_counts(lb, torch, sets)
    om = json.load(open(OPMODEL))
    kern, ops64 = launch_table(per, sets, mix, knodes, om, "f64")
    js = len(sets) - 1
    stress = sets[js][0]
    roof = roofline_block(ops64[(js, "K")], kern[f"K:{stress}"]["ms"],
                          "k_grouped<double, K, log> (lbessel_log_kv_f64)",
                          f"{stress}: {sets[js][1].numel()} pairs", sets[js][1].numel(), 24,
                          "log_kv_f64_stress")
    roof["branch_counts"] = {k: c for k, c in mix[(js, "K")].items()
                             if not (isinstance(c, list) and not any(c))}
    roof["fallback_nodes"] = knodes[js]
    all_k_ops = sum(ops64[(j, "K")] for j in range(len(sets)))
    all_k_ms = sum(kern[f"K:{nm}"]["ms"] for nm, _, _ in sets)
    roof["all_K_launches"] = {"frac": all_k_ops / (all_k_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS,
                              "ms": all_k_ms}
    i_ms = sum(kern[f"I:{nm}"]["ms"] for nm, _, _ in sets)
    k_ms = all_k_ms

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
            grp = kern[f"{kind}:{name}"]["ms"]
            ablation[f"{kind}:{name}"] = {"grouped_ms": grp, "ungrouped_ms": ung,
                                          "speedup": ung / grp}

    f32 = None
    if not args.no_f32:
        sets32 = [(nm, v.float(), x.float()) for nm, v, x in sets]
        o32 = {}
        one_step(lb, torch, sets32, o32)
        torch.cuda.synchronize()
        steps32 = max(args.steps, 3)
        wall32, issue32, timers32 = timed_steps(lb, torch, sets32, o32, steps32)
        dt = wall32 / steps32
        per32 = {}
        for name, kind, e0, e1 in timers32:
            per32.setdefault((name, kind), []).append(e0.elapsed_time(e1))
        mix32, knodes32 = op_counts(lb, torch, sets32)
        kern32, ops32 = launch_table(per32, sets32, mix32, knodes32, om, "f32")
        f32 = {"value": evals / dt / 1e9, "unit": "G evals/s", "ms_per_step": dt * 1e3,
               "host_issue_ms_per_step": issue32 * 1e3 / steps32,
               "steps": steps32, "kernels": kern32}
        if ops32 is not None:
            f32["roofline"] = roofline_block(
                ops32[(js, "K")], kern32[f"K:{stress}"]["ms"],
                "k_grouped<float, K, log> (lbessel_log_kv_f32)",
                f"{stress}: {sets[js][1].numel()} pairs", sets[js][1].numel(), 12,
                "log_kv_f32_stress")
            f32["roofline"]["branch_counts"] = mix32[(js, "K")]
            f32["roofline"]["fallback_nodes"] = knodes32[js]
        if not args.no_cpu_baseline:
            f32["errors"] = f32_errors(torch, sets32, o32)
        del sets32, o32

    ablations = None
    if not args.no_ablation:
        ablations = ablation_bench(lb, torch, sets)
    paper_k = None
    if "quad600_per_eval" in om.get("K_f64", {}):
        # the paper's own K fallback (eq. log Kv integral, 600 nodes, Debye at
        # 13 terms everywhere): lbessel_log_kv_integral_f64 on the stress grid
        c = mix[(js, "K")]
        ck = om["K_f64"]
        ops = (c["mu20"] * ck["mu20"] + (c["u13"] + c["u9"] + c["u6"] + c["u4"]) * ck["u13"]
               + c["fallback"] * ck["quad600_per_eval"])
        _, sv, sx = sets[js]
        o = lb.log_kv_integral(sv, sx)
        ts = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            lb.log_kv_integral(sv, sx)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        del o
        paper_k = roofline_block(ops, float(np.median(ts)),
                                 "k_grouped<double, K, log, u_integral> "
                                 "(lbessel_log_kv_integral_f64)",
                                 f"{stress}: {sets[js][1].numel()} pairs", sets[js][1].numel(),
                                 24, "log_kv_f64_stress_u_integral")
        paper_k["quad600_per_eval"] = ck["quad600_per_eval"]
        paper_k["speedup_of_default_path"] = paper_k["launch_ms"] / kern[f"K:{stress}"]["ms"]
    order01, paper_tables = None, None
    if not args.no_tables:
        log("orders 0/1 and the paper's runtime tables")
        order01 = order01_bench(lb, torch)
        paper_tables = paper_tables_bench(lb, torch)

    vmf_res = None
    if not args.no_vmf:
        vmf_res = vmf_bench(lb, torch)
    launch_cost = None
    if not args.no_serving:
        log("launch cost: direct vs graph replay")
        launch_cost = graph_bench(lb, torch)

    cpu, errors = None, None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        host = [(v.cpu().numpy(), x.cpu().numpy()) for _, v, x in sets]
        cpu, sample = cpu_baseline(host)
        del host
        errors = sample_errors(torch, outs, sample)

    serving = None
    if not args.no_serving:
        del outs
        torch.cuda.empty_cache()
        serving = {"host": serving_bench(torch, resident="host"),
                   "device": serving_bench(torch, resident="device")}

    workload = ("log I_v and log K_v, f64: 20M pairs per order v=2^0..2^10 with x~U[1,100) "
                "plus the 2^26-pair stress grid (log10 v~U[-3,4], log10 x~U[-4,4])")
    detail = {
        "what": "bench detail (the last line is the summary)",
        "config": {"workload": workload, "pairs_per_step": n_pairs, "evals_per_step": evals},
        "roofline": roof, "cpu_baseline": cpu, "all_finite": finite,
        "max_err_on_oracle_sample": errors, "ms_I_per_step": i_ms, "ms_K_per_step": k_ms,
        "host_issue_ms_per_step": t_issue * 1e3 / args.steps,
        "f32": f32, "paper_k": paper_k, "grouping_ablation": ablation, "ablations": ablations,
        "order01": order01, "paper_tables": paper_tables, "vmf": vmf_res, "serving": serving,
        "launch_cost": launch_cost,
        "kernels": kern,
    }
    if args.detail:
        with open(args.detail, "w") as f:
            json.dump(detail, f, indent=1)
    print(json.dumps(detail), flush=True)

    def errsum(e):
        if e is None:
            return None
        return {k: {"points": e[k]["points"], "max_cond_err": e[k]["max_cond_err"],
                    "max_rel_err": e[k]["max_rel_err"], "max_rel_floor1": e[k]["max_rel_floor1"],
                    "above_tol": e[k]["above_tol"]} for k in ("I", "K")}

    keep = ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel", "launch",
            "launch_ms", "ops_per_launch", "algorithmic_bytes_per_launch", "valu_busy",
            "active_lanes")
    line = {
        "metric": "G evals/s log I_v & log K_v (f64, f32) at max rel err; "
                  "p50/p99 latency at QPS",
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
        "config": {"workload": workload, "pairs_per_step": n_pairs, "evals_per_step": evals},
        "roofline": {k: roof[k] for k in keep if k in roof} | {
            "all_K_launches_frac": roof["all_K_launches"]["frac"]},
        "cpu_baseline": cpu,
        "all_finite": finite,
        "errors": errsum(errors),
        "ms_I_per_step": i_ms,
        "ms_K_per_step": k_ms,
        "f32": None if f32 is None else {
            "value": f32["value"], "unit": "G evals/s", "ms_per_step": f32["ms_per_step"],
            "roofline": None if "roofline" not in f32 else {
                k: f32["roofline"][k] for k in keep if k in f32["roofline"]},
            "errors": errsum(f32.get("errors"))},
        "paper_k_u_integral": None if paper_k is None else {
            k: paper_k[k] for k in ("launch_ms", "frac", "valu_busy", "active_lanes",
                                    "speedup_of_default_path")
            if k in paper_k},
        "serving": None if serving is None else {
            res: {"saturation_req_s": {k: v["requests_per_s"]
                                       for k, v in serving[res]["saturation"].items()},
                  "p50_p99_ms_at_0.9": {k: [serving[res]["sweep"][-1][k]["p50_ms"],
                                            serving[res]["sweep"][-1][k]["p99_ms"]]
                                        for k in ("batched", "plain_8streams")}}
            for res in serving},
        "launch_cost_us": None if launch_cost is None else {
            k: launch_cost[k] for k in ("direct_host_us", "direct_gpu_us_per_batch",
                                        "graph_host_us", "graph_gpu_us_per_batch",
                                        "graph_replays_equal_eager")},
    }
    print(json.dumps(line), flush=True)


def launch_table(per, sets, mix, knodes, om, prec):
    """Per-launch time, G evals/s and op-model VALU fraction, and the
    algorithmic ops of every launch ((set, kind) -> ops; None without an op
    model for this precision)."""
    ck, ci = om.get(f"K_{prec}"), om.get(f"I_{prec}")
    ops = None
    if ck is not None and ci is not None:
        ops = {}
        for j in range(len(sets)):
            c = mix[(j, "K")]
            int_ops, n_int = k_int_ops(c, ck)
            n_tm = c.get("temme", 0)
            tm_ops = 0.0
            if n_tm:
                tm_ops = (n_tm * ck["temme_setup"] + c["temme_terms"] * ck["temme_per_term"]
                          + c["temme_steps"] * ck["temme_per_step"])
            ops[(j, "K")] = (c["mu20"] * ck["mu20"]
                             + sum(c[u] * ck[u] for u in ("u13", "u9", "u6", "u4"))
                             + (c["fallback"] - n_int - n_tm) * ck["fallback_setup"]
                             + knodes[j] * ck["fallback_per_node"] + int_ops + tm_ops)
            c = mix[(j, "I")]
            ops[(j, "I")] = (c["mu20"] * ci["mu20"]
                             + sum(c[u] * ci[u] for u in ("u13", "u9", "u6", "u4"))
                             + c["fallback"] * ci["fallback"])
    kern = {}
    for (name, kind), ts in per.items():
        j = [i for i, (nm, _, _) in enumerate(sets) if nm == name][0]
        n = sets[j][1].numel()
        ms = float(np.mean(ts))
        kern[f"{kind}:{name}"] = {"ms": ms, "G_evals_s": n / ms / 1e6}
        if ops is not None:
            kern[f"{kind}:{name}"]["valu_frac"] = ops[(j, kind)] / (ms * 1e-3) / 1e12 / VALU_PEAK_TOPS
    return kern, ops


def roofline_block(ops, ms, kernel, launch, n, bytes_per_pair, counter_label):
    """Roofline record of one launch: algorithmic VALU lane-instructions (the
    op model) per launch over its measured duration, against the VALU issue
    rate; counters (traffic, VALU busy, active lanes) from the committed probe
    summary while the kernel sources match it."""
    achieved = ops / (ms * 1e-3) / 1e12
    c = counters(counter_label)
    rec = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
           "frac": achieved / VALU_PEAK_TOPS,
           "traffic": None if c is None else c["hbm_bytes"],
           "kernel": kernel, "launch": launch, "launch_ms": ms, "ops_per_launch": ops,
           "algorithmic_bytes_per_launch": bytes_per_pair * n,
           "op_model": "mu20 x n_mu + sum over Debye tiers uK x n_uK + fallback_setup x n_fb"
                       " + fallback_per_node x nodes + integer-order K elements at their"
                       " per-order cost int_le2/int_gt2 + Temme-series K elements at"
                       " temme_setup + temme_per_term x terms + temme_per_step x order steps"
                       " (paper_2409_08729_amd/opmodel.json)"}
    if c is not None:
        rec["valu_busy"] = c["valu_busy"]
        rec["active_lanes"] = c["active_lanes"]
    return rec


if __name__ == "__main__":
    main()
