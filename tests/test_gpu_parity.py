"""GPU parity: the HIP path (through the C-ABI) against the binary128 oracle.

Every comparison is element by element on seeded inputs.  Floating-point
results are gated on the conditioned relative error (see parity.py) at
4e-15 (f64) / 2e-6 (f32); special values must match exactly; the grouped
and ungrouped kernels must agree bit for bit.
"""
import numpy as np
import pytest
import torch

from paper_2409_08729_amd import workloads as wl
from parity import TOL32, TOL64, cond_err, rel_err, same_specials, summary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the -m gpu tests need an MI355X")
    import paper_2409_08729_amd as m
    m.lib()
    return m


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def run(lb, kind, v, x, dtype=torch.float64):
    f = lb.log_iv if kind == "I" else lb.log_kv
    return host(f(dev(v, dtype), dev(x, dtype)))


def check64(lb, oracle, kind, v, x, what, tol=TOL64):
    y = run(lb, kind, v, x)
    hi, lo = (oracle.log_iv if kind == "I" else oracle.log_kv)(v, x)
    assert same_specials(y, hi), what
    e = cond_err(y, hi, lo, v, x)
    i = int(np.argmax(e))
    print(f"{what} {kind}: cond {summary(e)}; rel {summary(rel_err(y, hi, lo))}")
    assert e.max() <= tol, (what, kind, v[i], x[i], y[i], hi[i], e[i])
    return e


# ---------------------------------------------------------------------------
# f64 forward
# ---------------------------------------------------------------------------

def test_m1_log_iv_all_points(lb, oracle):
    v, x = wl.m1()
    check64(lb, oracle, "I", v, x, "M1 (65,536 pairs)")


def test_m1_log_kv_all_points(lb, oracle):
    v, x = wl.m1()
    check64(lb, oracle, "K", v, x, "M1 (65,536 pairs)")


@pytest.mark.parametrize("kind", ["I", "K"])
def test_stress_sample(lb, oracle, kind):
    v, x = wl.m3(n=12288, seed=31)
    check64(lb, oracle, kind, v, x, "stress log-uniform sample")


@pytest.mark.parametrize("kind", ["I", "K"])
def test_paper_regions(lb, oracle, kind):
    v1, x1 = wl.small_region(4096)
    v2, x2 = wl.large_region(2048, kind)
    v3, x3 = wl.corner_v100_x01(1024)
    v = np.concatenate([v1, v2, v3])
    x = np.concatenate([x1, x2, x3])
    check64(lb, oracle, kind, v, x, "Small/Large regions + (v~100, x~0.1)")


BOUNDARIES = {
    # (v range, x range) bands straddling each re-fitted threshold
    "I": [(0, 8.5, 21.0, 22.0), (8.3, 8.7, 21.6, 30.0), (9.0, 13.0, 23.5, 24.5),
          (0.05, 0.15, 22.5, 30.0), (14.3, 14.7, 1e-3, 23.0), (0.1, 14.5, 22.8, 23.2),
          (20.0, 200.0, 90.0, 10000.0)],
    "K": [(0, 8.5, 17.0, 18.0), (8.3, 8.7, 17.6, 30.0), (0.05, 0.15, 17.5, 30.0),
          (14.3, 14.7, 1e-3, 22.0), (8.5, 14.5, 19.8, 20.2), (10.0, 120.0, 20.0, 4000.0)],
}


@pytest.mark.parametrize("kind", ["I", "K"])
def test_regime_boundary_bands(lb, oracle, kind):
    vs, xs = [], []
    for j, (a, b, c, d) in enumerate(BOUNDARIES[kind]):
        v, x = wl.band(1536, a, b, c, d, seed=100 + j)
        vs.append(v)
        xs.append(x)
    # the curve v^2 = e^{1.4} x, +-2% in v
    g = np.random.default_rng(77)
    xc = 10 ** g.uniform(np.log10(25.0), np.log10(9000.0 if kind == "I" else 3000.0), 2048)
    vc = np.sqrt(np.exp(1.4) * xc) * g.uniform(0.98, 1.02, xc.size)
    v = np.concatenate(vs + [vc])
    x = np.concatenate(xs + [xc])
    check64(lb, oracle, kind, v, x, "regime boundary bands")


@pytest.mark.parametrize("kind", ["I", "K"])
def test_zero_crossings_and_special_orders(lb, oracle, kind):
    roots = {"I": [(1, 1.518), (2, 2.296), (4, 3.748), (8, 6.540), (16, 11.997), (32, 22.767),
                   (64, 44.150), (128, 86.746)],
             "K": [(2, 1.220), (4, 2.365), (8, 4.827), (16, 9.934), (32, 20.341), (64, 41.353),
                   (128, 83.573)]}[kind]
    g = np.random.default_rng(5)
    v = np.concatenate([np.full(256, float(a)) for a, _ in roots])
    x = np.concatenate([b + g.uniform(-1e-3, 1e-3, 256) for _, b in roots])
    # v in {0, 1} over the Small and Large argument ranges, half-integer orders
    x01 = np.concatenate([g.uniform(0, 150, 2048), g.uniform(150, 1e4, 2048)])
    v = np.concatenate([v, np.zeros(4096), np.ones(4096), 0.5 + g.integers(0, 60, 2048)])
    x = np.concatenate([x, x01, x01, 10 ** g.uniform(-3, 3, 2048)])
    check64(lb, oracle, kind, v, x, "zero crossings, v in {0,1}, half-integer v")


@pytest.mark.parametrize("kind", ["I", "K"])
def test_special_values(lb, oracle, kind):
    inf, nan = np.inf, np.nan
    big_v = 1e300 if kind == "I" else 1e12        # the K oracle stops at |v| = 1e15
    vals = [0.0, -0.0, 1e-300, 0.3, 1.0, 2.5, 30.0, 1e8, big_v, inf, -1.0, -2.5, nan]
    xs = [0.0, -0.0, 1e-300, 1e-4, 0.5, 19.9, 25.0, 1e4, 1e6, inf, -1.0, nan]
    V, X = np.meshgrid(np.array(vals), np.array(xs), indexing="ij")
    v, x = V.ravel(), X.ravel()
    y = run(lb, kind, v, x)
    hi, lo = (oracle.log_iv if kind == "I" else oracle.log_kv)(v, x)
    # -0.0 arguments: the library compares with 0, like the reference
    ok_special = ~np.isfinite(hi)
    assert np.array_equal(np.isnan(y[ok_special]), np.isnan(hi[ok_special]))
    fin = ok_special & ~np.isnan(hi)
    assert np.array_equal(y[fin], hi[fin])
    # finite references (including extreme but finite arguments)
    m = np.isfinite(hi)
    assert np.isfinite(y[m]).all(), (v[m][~np.isfinite(y[m])], x[m][~np.isfinite(y[m])])
    e = cond_err(y[m], hi[m], lo[m], v[m], x[m])
    assert e.max() <= TOL64, (v[m][np.argmax(e)], x[m][np.argmax(e)], e.max())


def test_huge_arguments_match_leading_terms(lb):
    """x up to 1e300 (beyond the oracle's range): with v^2 << x the Hankel
    correction is below rounding, so log I = x - log(2 pi x)/2 and
    log K = log(pi/(2x))/2 - x to the last bit of x; both stay finite."""
    x = np.array([1e20, 1e50, 1e100, 1e200, 1e300, 1.7e308])
    v = np.array([0.0, 0.3, 2.0, 1e3, 1e20, 1e50])
    yi = run(lb, "I", v, x)
    yk = run(lb, "K", v, x)
    assert np.isfinite(yi).all() and np.isfinite(yk).all()
    np.testing.assert_allclose(yi, x - 0.5 * (np.log(2 * np.pi) + np.log(x)), rtol=4e-16)
    np.testing.assert_allclose(yk, 0.5 * (np.log(np.pi / 2) - np.log(x)) - x, rtol=4e-16)
    # tiny x, huge v: log I -> v log(x/2) - lgamma(v+1), finite
    v = np.array([1e4, 1e8, 1e12])
    x = np.array([1e-300, 1e-100, 1e-10])
    yi = run(lb, "I", v, x)
    yk = run(lb, "K", v, x)
    assert np.isfinite(yi).all() and np.isfinite(yk).all()
    from math import lgamma
    ref = np.array([vv * np.log(xx / 2) - lgamma(vv + 1) for vv, xx in zip(v, x)])
    np.testing.assert_allclose(yi, ref, rtol=1e-13)


def test_both_sides_of_the_reciprocal_range_switch(lb, oracle):
    """The Hankel and Debye branches use reciprocals and one merged logarithm
    below 1e300 and divisions with separate logarithms from 1e300 up; both
    forms must hold on either side: log I (Debye) across v = 1e300 against
    the oracle, and both kinds (Hankel) across x = 1e300 against the leading
    terms, which are exact to rounding there."""
    v = np.repeat([9.99e299, 1e300, 1.0001e300, 1e305], 4)
    x = np.tile([1e-3, 1.0, 1e6, 1e12], 4)
    check64(lb, oracle, "I", v, x, "Debye across v = 1e300")
    x = np.array([9.9e299, 9.999e299, 1e300, 1.0001e300, 3e300])
    v = np.array([0.0, 0.5, 2.0, 30.0, 1e3])
    yi = run(lb, "I", v, x)
    yk = run(lb, "K", v, x)
    np.testing.assert_allclose(yi, x - 0.5 * (np.log(2 * np.pi) + np.log(x)), rtol=4e-16)
    np.testing.assert_allclose(yk, 0.5 * (np.log(np.pi / 2) - np.log(x)) - x, rtol=4e-16)


# ---------------------------------------------------------------------------
# branch-level pins
# ---------------------------------------------------------------------------

def test_mu20_terminates_at_half_integer_order(lb, oracle):
    """v = m + 1/2, m <= 19: the factor mu - (2j-1)^2 vanishes at j = m+1, so the
    Hankel sum is finite and equals K exactly (and I up to e^{-2x})."""
    m = np.arange(0, 20)
    v = np.repeat(m + 0.5, 8)
    x = np.tile(np.array([30.0, 45.0, 60.0, 100.0, 300.0, 1e3, 5e3, 1e4]), m.size)
    yk = host(lb.eval_branch("K", 0, dev(v), dev(x)))
    hi, lo = oracle.log_kv(v, x)
    assert cond_err(yk, hi, lo, v, x).max() <= 4 * 2.2e-16
    # for I the alternating sum cancels (amplification ~ e^{v^2/x}); check it
    # where the regime uses it, v^2 < e^{1.4} x
    m = v * v < np.exp(1.4) * x
    yi = host(lb.eval_branch("I", 0, dev(v[m]), dev(x[m])))
    hi, lo = oracle.log_iv(v[m], x[m])
    assert cond_err(yi, hi, lo, v[m], x[m]).max() <= 8 * 2.2e-16


@pytest.mark.parametrize("kind", ["K"])
def test_tiny_x_small_order(lb, oracle, kind):
    """x in [1e-300, 1e-4], v in [0, 0.5]: the integral branch and, below x = 1e-10
    for v < 0.3, the small-argument form; the oracle's trapezoid rule in t has no
    such limit."""
    g = np.random.default_rng(17)
    v = np.concatenate([g.uniform(0, 0.5, 1200), np.zeros(64), np.full(64, 0.049),
                        np.full(64, 0.051), np.full(64, 0.2999), np.full(64, 0.3)])
    x = np.concatenate([10 ** g.uniform(-300, -4, 1200)] + [10 ** g.uniform(-300, -4, 64)] * 5)
    check64(lb, oracle, kind, v, x, "tiny x, v in [0, 0.5]")


def test_k_fallback_at_half_order_matches_closed_form(lb):
    """v = 1/2: the K fallback (forced, over x from 1e-4 to 20) against
    log K_{1/2}(x) = 1/2 log(pi/(2x)) - x (DLMF 10.49.12 with n = 0) taken in
    60-digit decimal arithmetic: within a few rounding units of the result,
    four times tighter than the parity bar, so a normalisation slip of the rule
    (a wrong step weight or shift) cannot hide in the tolerance."""
    import closed_forms as cf
    x = np.concatenate([10 ** np.linspace(-4, 1.3, 64), np.linspace(0.5, 20, 40)])
    v = np.full(x.size, 0.5)
    y = host(lb.eval_branch("K", 2, dev(v), dev(x)))
    ref = np.array([cf.log_kv_half(0, xx) for xx in x])
    den = np.maximum(np.abs(ref.astype(np.float64)), 1 + np.hypot(v, x))
    err = np.array([float(abs(cf.Decimal(float(yy)) - r)) for yy, r in zip(y, ref)]) / den
    assert err.max() <= 1e-15, err.max()


@pytest.mark.parametrize("kind", ["I", "K"])
def test_each_branch_on_its_region(lb, oracle, kind):
    v, x = wl.m3(n=16384, seed=51)
    br = host(lb.classify(kind, dev(v), dev(x)))
    for b in range(3):
        sel = br == b
        if not sel.any():
            continue
        y = host(lb.eval_branch(kind, b, dev(v[sel]), dev(x[sel])))
        hi, lo = (oracle.log_iv if kind == "I" else oracle.log_kv)(v[sel], x[sel])
        e = cond_err(y, hi, lo, v[sel], x[sel])
        print(f"{kind} branch {b}: n={sel.sum()} {summary(e)}")
        assert e.max() <= TOL64


# ---------------------------------------------------------------------------
# grouping is invisible: bitwise equality with the ungrouped kernel
# ---------------------------------------------------------------------------

def _layouts():
    g = np.random.default_rng(3)
    n = 2048 * 3 + 17
    v_cheap, x_cheap = 0.7, 60.0        # mu20
    v_mid, x_mid = 40.0, 10.0           # u13
    v_fb, x_fb = 3.0, 2.0               # fallback
    tri = np.array([[v_cheap, x_cheap], [v_mid, x_mid], [v_fb, x_fb]])
    out = {}
    idx = np.arange(n) % 3
    out["alternating"] = tri[idx]
    out["all_fallback"] = np.tile(tri[2], (n, 1))
    idx = g.integers(0, 3, n)
    out["random"] = tri[idx] * g.uniform(0.9, 1.1, (n, 2))
    idx = np.zeros(n, int)
    idx[::64] = 2
    out["one_odd_lane_per_wave"] = tri[idx]
    vs, xs = wl.m3(n=n, seed=12)
    out["stress"] = np.stack([vs, xs], 1)
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["I", "K"])
def test_grouped_equals_ungrouped_bitwise(lb, kind, dtype):
    f = lb.log_iv if kind == "I" else lb.log_kv
    for name, vx in _layouts().items():
        for n in (1, 63, 64, 65, 2047, 2048, 2049, vx.shape[0]):
            v = dev(vx[:n, 0], dtype)
            x = dev(vx[:n, 1], dtype)
            a = host(f(v, x))
            b = host(lb.eval_ungrouped(kind, v, x))
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (name, n)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["I", "K"])
def test_large_launches_equal_ungrouped_bitwise(lb, kind, dtype):
    """Launches of 2^24 elements and more, including tiles with a single
    fallback element and a ragged last tile: every value equals the
    one-element-per-thread kernel's."""
    f = lb.log_iv if kind == "I" else lb.log_kv
    vs, xs = wl.m3(n=(1 << 25) + 777, seed=13)
    cases = {"stress_2^25+777": (vs, xs), "stress_2^24": (vs[:1 << 24], xs[:1 << 24])}
    n = (1 << 24) + 5
    v = np.full(n, 1.0)
    x = np.full(n, 50.0)                 # Hankel
    v[::1024], x[::1024] = 3.0, 5.0      # one fallback element per tile
    v[5::4096], x[5::4096] = 0.5, 1e-4   # a costlier bucket every 4th tile
    v[-3:], x[-3:] = 3.0, 5.0            # fallback in the ragged last tile
    cases["sparse_fallback"] = (v, x)
    for name, (v, x) in cases.items():
        dv, dx = dev(v, dtype), dev(x, dtype)
        a = host(f(dv, dx))
        b = host(lb.eval_ungrouped(kind, dv, dx))
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), name


def test_empty_input(lb):
    e = torch.empty(0, dtype=torch.float64, device="cuda:0")
    assert lb.log_iv(e, e).numel() == 0
    assert lb.log_kv(e, e).numel() == 0


# ---------------------------------------------------------------------------
# f32
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["I", "K"])
def test_f32_parity(lb, oracle, kind):
    v1, x1 = wl.m1(n=16384, seed=41)
    v2, x2 = wl.m3(n=8192, seed=42)
    v = np.concatenate([v1, v2]).astype(np.float32)
    x = np.concatenate([x1, x2]).astype(np.float32)
    y = run(lb, kind, v, x, torch.float32).astype(np.float64)
    v64, x64 = v.astype(np.float64), x.astype(np.float64)     # exact widening
    hi, lo = (oracle.log_iv if kind == "I" else oracle.log_kv)(v64, x64)
    # results of order > f32 range are not representable: compare where finite
    m = np.isfinite(hi) & (np.abs(hi) < 3e38)
    e = cond_err(y[m], hi[m], lo[m], v64[m], x64[m])
    print(f"f32 {kind}: cond {summary(e)}")
    assert e.max() <= TOL32


# ---------------------------------------------------------------------------
# derivatives and vMF
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["I", "K"])
def test_grad_x_f64(lb, oracle, kind):
    v1, x1 = wl.m1(n=8192, seed=61)
    v2, x2 = wl.m3(n=8192, seed=62)
    v = np.concatenate([v1, v2])
    x = np.concatenate([x1, x2])
    gfun = lb.log_iv_grad_x if kind == "I" else lb.log_kv_grad_x
    gout = np.random.default_rng(1).uniform(0.5, 2.0, v.size)
    d = host(gfun(dev(v), dev(x), dev(gout)))
    dh, dl = (oracle.dlog_iv if kind == "I" else oracle.dlog_kv)(v, x)
    ref = (dh + dl) * gout
    # error budget: the ratio exp(y1 - y0) inherits the absolute error of y1 - y0
    f = oracle.log_iv if kind == "I" else oracle.log_kv
    y0 = f(v, x)[0]
    y1 = f(v + 1, x)[0]
    ratio = np.exp(y1 - y0)
    s0 = np.maximum(np.abs(y0), 1 + np.hypot(v, x))
    s1 = np.maximum(np.abs(y1), 1 + np.hypot(v + 1, x))
    bound = TOL64 * (ratio * (s0 + s1) + v / x + 1.0) * np.abs(gout)
    err = np.abs(d - ref)
    i = int(np.argmax(err / bound))
    print(f"grad {kind}: max err/bound {(err / bound).max():.3f}")
    assert (err <= bound).all(), (v[i], x[i], d[i], ref[i], bound[i])


@pytest.mark.parametrize("p", [2.0, 3.0, 2048.0, 8192.0, 32768.0])
def test_vmf_log_norm(lb, oracle, p):
    g = np.random.default_rng(int(p))
    kappa = np.concatenate([10 ** g.uniform(-3, 5.5, 2048), [0.0]])
    y = host(lb.vmf_log_norm(dev(kappa), p))
    hi, lo = oracle.vmf_log_norm(kappa, p)
    v = p / 2 - 1
    scale = np.abs(v * np.log(np.where(kappa > 0, kappa, 1))) + np.abs(hi) + p * 1.0
    liv = oracle.log_iv(np.full(kappa.size, v), kappa)[0]
    scale = np.maximum(scale, np.maximum(np.abs(liv), 1 + np.hypot(v, kappa)))
    e = np.abs(y - hi - lo) / scale
    assert e.max() <= TOL64, (kappa[np.argmax(e)], e.max())


def test_autograd_matches_grad_entry_point(lb):
    v = dev(np.array([0.0, 0.5, 3.0, 40.0, 700.0]))
    x = dev(np.array([0.3, 20.0, 5.0, 80.0, 1500.0])).requires_grad_(True)
    y = lb.LogIv.apply(v, x)
    (gx,) = torch.autograd.grad(y.sum(), x)
    ref = lb.log_iv_grad_x(v, x.detach())
    assert torch.equal(gx, ref)
    y = lb.LogKv.apply(v, x)
    (gx,) = torch.autograd.grad(y.sum(), x)
    assert torch.equal(gx, lb.log_kv_grad_x(v, x.detach()))


# ---------------------------------------------------------------------------
# full-size inputs in the benchmark's launch configuration, sampled
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["m2_order0", "m2_order3", "m2_order10", "m3"])
@pytest.mark.parametrize("kind", ["I", "K"])
def test_full_size_sampled(lb, oracle, which, kind):
    if which == "m3":
        v, x = wl.m3()
    else:
        v, x = wl.m2_order(int(which.split("order")[1]))
    f = lb.log_iv if kind == "I" else lb.log_kv
    yt = f(dev(v), dev(x))
    idx = np.random.default_rng(99).choice(v.size, 3000, replace=False)
    idx = np.concatenate([idx, [0, v.size - 1]])
    y = yt[torch.as_tensor(idx, device="cuda:0")].cpu().numpy()
    assert torch.isfinite(yt).all().item()
    hi, lo = (oracle.log_iv if kind == "I" else oracle.log_kv)(v[idx], x[idx])
    e = cond_err(y, hi, lo, v[idx], x[idx])
    print(f"{which} {kind} n={v.size}: {summary(e)}")
    assert e.max() <= TOL64


def test_golden_closed_forms(lb):
    """The HIP path against the stored 40-digit half-integer closed forms."""
    from decimal import Decimal
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.tsv")
    rows = [ln.rstrip("\n").split("\t") for ln in open(path) if not ln.startswith("#")]
    for kind in ("I", "K"):
        sel = [r for r in rows if r[0] == kind]
        v = np.array([float(r[1]) for r in sel])
        x = np.array([float(r[2]) for r in sel])
        y = run(lb, kind, v, x)
        for i, r in enumerate(sel):
            ref = Decimal(r[3])
            err = abs(Decimal(float(y[i])) - ref) / max(abs(ref), Decimal(1) + Decimal(
                float(np.hypot(v[i], x[i]))))
            assert err <= Decimal(TOL64), (kind, v[i], x[i], float(err))
