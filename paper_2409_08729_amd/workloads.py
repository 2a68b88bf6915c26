"""Seeded synthetic inputs (no arithmetic of the method lives here).

Shapes follow the paper's experiments (arXiv 2409.08729):
  * per-order sets: v fixed to 2^k, k = 0..10, x uniform in [1, 100) (the
    runtime comparison of the introduction, 20M values of x per order);
  * a stress grid with v log-uniform in [1e-3, 1e4] and x log-uniform in
    [1e-4, 1e4], covering the under/overflow regions of naive evaluation;
  * the Small [0, 150]^2 and Large [150, 1e4]^2 ([150, 4000]^2 for K) test
    regions (Sec. "Test Regions"), and the v ~ 100, x ~ 0.1 corner the paper
    re-checked by hand (Sec. "Precision").
All generators use numpy's PCG64 (default_rng) with a fixed seed, so every
array is reproducible bit for bit on any host.
"""
from __future__ import annotations

import numpy as np

SEED_M1 = 20240913
SEED_M2 = 20240914
SEED_M3 = 20240915
ORDERS = tuple(float(2 ** k) for k in range(11))


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def m1(n: int = 65536, seed: int = SEED_M1):
    """v uniform on {2^0..2^10}, x uniform in [1, 100) (float64)."""
    g = rng(seed)
    v = np.ldexp(1.0, g.integers(0, 11, n)).astype(np.float64)
    x = g.uniform(1.0, 100.0, n)
    return v, x


def m2_order(k: int, n: int = 20_000_000, seed: int = SEED_M2):
    """One order of the per-order set: v = 2^k for all n, x uniform in [1, 100)."""
    g = rng(seed + 1000 * k)
    x = g.uniform(1.0, 100.0, n)
    v = np.full(n, float(2 ** k))
    return v, x


def m3(n: int = 1 << 26, seed: int = SEED_M3):
    """Stress grid: log10 v ~ U[-3, 4], log10 x ~ U[-4, 4], independent."""
    g = rng(seed)
    v = 10.0 ** g.uniform(-3.0, 4.0, n)
    x = 10.0 ** g.uniform(-4.0, 4.0, n)
    return v, x


def small_region(n: int, seed: int = 7):
    g = rng(seed)
    return g.uniform(0.0, 150.0, n), g.uniform(0.0, 150.0, n)


def large_region(n: int, kind: str = "I", seed: int = 8):
    g = rng(seed)
    hi = 1e4 if kind == "I" else 4000.0
    return g.uniform(150.0, hi, n), g.uniform(150.0, hi, n)


def corner_v100_x01(n: int, seed: int = 9):
    g = rng(seed)
    return g.uniform(90.0, 110.0, n), g.uniform(0.05, 0.2, n)


def band(n: int, vlo: float, vhi: float, xlo: float, xhi: float, seed: int = 10):
    g = rng(seed)
    return g.uniform(vlo, vhi, n), g.uniform(xlo, xhi, n)


def vmf_features(n: int, p: int, seed: int, device="cpu"):
    """Synthetic feature rows |g|, g ~ N(mu, 0.5^2 I), mu ~ N(0, I) fixed per set
    (float32, not normalised: the library normalises each row).  Generated
    with torch's seeded generator on `device` (reproducible per device type)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    mu = torch.randn(p, generator=gen, device=device, dtype=torch.float32)
    X = torch.randn(n, p, generator=gen, device=device, dtype=torch.float32)
    X.mul_(0.5).add_(mu).abs_()
    return X


# ---------------------------------------------------------------------------
# Serving request stream
# ---------------------------------------------------------------------------
SEED_SERVE = 20240916
SERVE_MAX_PAIRS = 4 << 20          # evaluation requests: 1 .. 4M pairs
SERVE_VMF_DIMS = (2048, 8192, 32768)
SERVE_VMF_ROWS = (1000, 50_000)    # N log-uniform in this range


def serving_pool(n: int = 2 * SERVE_MAX_PAIRS, seed: int = SEED_SERVE):
    """(v, x) float64 pools that evaluation requests slice: log10 v ~ U[-3, 4],
    log10 x ~ U[-3, 4], and one element in 256 with v = 0 exactly."""
    g = rng(seed)
    v = 10.0 ** g.uniform(-3.0, 4.0, n)
    x = 10.0 ** g.uniform(-3.0, 4.0, n)
    v[g.integers(0, n, n // 256)] = 0.0
    return v, x


def serving_requests(count: int, seed: int = SEED_SERVE + 1, vmf_share: float = 0.125,
                     pool: int = 2 * SERVE_MAX_PAIRS, max_pairs: int = SERVE_MAX_PAIRS,
                     vmf_rows=SERVE_VMF_ROWS):
    """A seeded request stream: a list of dicts and the unit-rate Poisson
    inter-arrival gaps (divide by the offered requests/s to get seconds).
      evaluation: {'type': 'eval', 'kind': 'I'|'K', 'precision': 64|32,
                   'n': log-uniform integer in [1, max_pairs], 'offset': start in the pool}
      vMF fit:    {'type': 'vmf', 'p': one of SERVE_VMF_DIMS,
                   'N': log-uniform integer in vmf_rows}"""
    g = rng(seed)
    reqs = []
    for _ in range(count):
        if g.random() < vmf_share:
            p = int(SERVE_VMF_DIMS[g.integers(0, len(SERVE_VMF_DIMS))])
            lo, hi = np.log(vmf_rows[0]), np.log(vmf_rows[1])
            N = int(np.clip(np.round(np.exp(g.uniform(lo, hi))), vmf_rows[0], vmf_rows[1]))
            reqs.append({"type": "vmf", "p": p, "N": N})
        else:
            n = int(np.clip(np.floor(np.exp(g.uniform(0.0, np.log(max_pairs + 1.0)))), 1, max_pairs))
            reqs.append({"type": "eval", "kind": "IK"[int(g.integers(0, 2))],
                         "precision": (64, 32)[int(g.integers(0, 2))], "n": n,
                         "offset": int(g.integers(0, pool - n + 1))})
    gaps = g.exponential(1.0, count)
    return reqs, gaps
