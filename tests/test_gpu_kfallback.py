"""The K fallback at its own internal boundaries, against the binary128
oracle: the cosh-integral rule's switch between a window that starts at
t = 0 and an interior window (including walks that step past t = 0 and use
the mirror node of the even integrand), the binary64 Temme series at
x <= 1.25 (its bound, mu = v - rint(v) near 0 and +-1/2, every order step),
the x = 1e-10 switch to the small-argument forms, orders near zero, and the
node and term counts the op model relies on."""
import numpy as np
import pytest
import torch

from parity import TOL64, TOL32, cond_err

pytestmark = pytest.mark.gpu

# inputs whose interior window's left walk steps past t = 0 (found by a
# float64 model of the rule; about 0.1% of random small-x fallback inputs)
MIRROR = [
    (float.fromhex('0x1.193ca9819d1d3p+2'), float.fromhex('0x1.854d6cb5f349ap-14')),
    (float.fromhex('0x1.2022ac10b1ef6p+1'), float.fromhex('0x1.496fdc71f506ap-29')),
    (float.fromhex('0x1.fcbd1317db53ap+1'), float.fromhex('0x1.e1f2a0fda44b3p-16')),
    (float.fromhex('0x1.a704f2936e64cp+1'), float.fromhex('0x1.167457e0dd052p-19')),
    (float.fromhex('0x1.9140245b684f5p+2'), float.fromhex('0x1.7de2183eda95fp-9')),
    (float.fromhex('0x1.39d3174c62361p+2'), float.fromhex('0x1.3741858e2a95ep-12')),
    (float.fromhex('0x1.06b0a66743e37p+1'), float.fromhex('0x1.5f301a2281cdep-32')),
    (float.fromhex('0x1.cf53040a0419dp+1'), float.fromhex('0x1.1677cf20b654cp-17')),
    (float.fromhex('0x1.77e6c54ca33adp+2'), float.fromhex('0x1.c42e6f190492ap-10')),
    (float.fromhex('0x1.9527509075b6fp+1'), float.fromhex('0x1.322f053a0a2d8p-20')),
    (float.fromhex('0x1.4843403bcc23dp+1'), float.fromhex('0x1.26a1a6bc5f6e0p-25')),
    (float.fromhex('0x1.31a794709bc9bp+3'), float.fromhex('0x1.b591fd1cad876p-5')),
    (float.fromhex('0x1.20609de1c12b4p+3'), float.fromhex('0x1.44a87053d84b9p-5')),
    (float.fromhex('0x1.9e45e5ea4bf36p+1'), float.fromhex('0x1.d457ad9b245ccp-20')),
    (float.fromhex('0x1.5f88bf1e253d4p+1'), float.fromhex('0x1.df86b649921e8p-24')),
    (float.fromhex('0x1.a6871539a45f0p+2'), float.fromhex('0x1.3585fa51edfc5p-8')),
    (float.fromhex('0x1.3035e677acb53p+3'), float.fromhex('0x1.ae5663a101324p-5')),
    (float.fromhex('0x1.13b7c59b7cc59p+1'), float.fromhex('0x1.eb27c1251f8e4p-31')),
    (float.fromhex('0x1.0b203fc11cc2ap+1'), float.fromhex('0x1.ca02ca8d9fc2fp-32')),
    (float.fromhex('0x1.0a4abf96cb4b3p+1'), float.fromhex('0x1.d28dc80ede9bdp-32')),
    (float.fromhex('0x1.4b31b3e72a154p+3'), float.fromhex('0x1.7b5cd09aaf3e8p-4')),
    (float.fromhex('0x1.56118796abbfep+2'), float.fromhex('0x1.8ec9cf631da7dp-11')),
    (float.fromhex('0x1.8f3ca5b2c854dp+2'), float.fromhex('0x1.84473db0d1b23p-9')),
    (float.fromhex('0x1.f73591200af72p+0'), float.fromhex('0x1.ce5f265eed5bdp-34')),
]


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the -m gpu tests need an MI355X")
    import paper_2409_08729_amd as m
    m.lib()
    return m


def _check(lb, oracle, v, x, dtype=torch.float64, variant=None):
    v = np.asarray(v, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    if dtype == torch.float32:
        v = v.astype(np.float32).astype(np.float64)
        x = x.astype(np.float32).astype(np.float64)
    dv = torch.from_numpy(v).to("cuda:0", dtype)
    dx = torch.from_numpy(x).to("cuda:0", dtype)
    if variant is None:
        y = lb.log_kv(dv, dx).double().cpu().numpy()
    else:
        y = lb.eval_variant("K", variant, "grouped", dv, dx).cpu().numpy()
    hi, lo = oracle.log_kv(v, x)
    assert np.array_equal(np.isfinite(y), np.isfinite(hi))
    e = cond_err(y, hi, lo, v, x)
    return e


def test_walks_past_zero(lb, oracle):
    """The binary64 default path takes these (small-x) points through Temme's
    series; the Table 1 variant keeps the cosh rule there."""
    v, x = np.array(MIRROR).T
    for variant in ("paper_regimes", None):
        e = _check(lb, oracle, v, x, variant=variant)
        assert e.max() <= TOL64, (variant, e.max())
        # the same points perturbed: both sides of the window switch
        for s in (1 - 1e-3, 1 + 1e-3, 0.97, 1.03):
            assert _check(lb, oracle, v, x * s, variant=variant).max() <= TOL64


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_small_argument_switch(lb, oracle, dtype):
    vs = np.array([0.0, 1e-8, 0.05, 0.1, 0.29, 0.2999999, 0.3, 0.3000001, 0.31, 0.5, 1.0, 3.7,
                   9.0, 14.4])
    xs = 1e-10 * np.array([1 - 1e-6, 1 - 1e-12, 1.0, 1 + 1e-12, 1 + 1e-6, 0.5, 2.0])
    v, x = np.meshgrid(vs, xs)
    e = _check(lb, oracle, v.ravel(), x.ravel(), dtype)
    assert e.max() <= (TOL64 if dtype == torch.float64 else TOL32), e.max()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_small_argument_form_above_order_0_3(lb, oracle, dtype):
    """x < 1e-10, v >= 0.3: the two-term small-argument form, including its
    switch at v = 0.9 and orders within 1e-7 of the integers, where the
    dropped terms cancel; x down to 1e-300 (1e-38 in binary32)."""
    g = np.random.default_rng(31)
    lo_x = -300 if dtype == torch.float64 else -37
    v = np.concatenate([g.uniform(0.3, 14.4, 400), [0.3, 0.5, 0.8999, 0.9, 0.9001, 0.99999, 1.0,
                        1.00001, 1.5, 2.0 - 1e-7, 2.0, 2.0 + 1e-7, 3.0, 7.0, 14.0, 14.4]])
    x = np.concatenate([10 ** g.uniform(lo_x, -10.0001, 400), 10 ** g.uniform(lo_x, -10.0001, 16)])
    e = _check(lb, oracle, v, x, dtype)
    assert e.max() <= (TOL64 if dtype == torch.float64 else TOL32), e.max()


def test_orders_near_zero(lb, oracle):
    g = np.random.default_rng(12)
    v = np.concatenate([10 ** g.uniform(-300, -3, 800), np.zeros(100)])
    x = 10 ** g.uniform(-10, np.log10(17.0), 900)
    e = _check(lb, oracle, v, x)
    assert e.max() <= TOL64, e.max()


def test_fallback_region_grid(lb, oracle):
    """A log-spaced grid over the whole fallback region, x from just above the
    small-argument switch to the Hankel bound and v up to the Debye bound:
    peaks from t* = 0 to t* ~ 25, where the step and the peak are found in
    binary32, against the oracle."""
    vs = np.concatenate([[0.0], 10 ** np.linspace(-6, np.log10(14.4), 47)])
    xs = 10 ** np.linspace(np.log10(1.0001e-10), np.log10(17.4), 48)
    v, x = np.meshgrid(vs, xs)
    e = _check(lb, oracle, v.ravel(), x.ravel())
    assert e.max() <= TOL64, e.max()
    dv, dx = torch.from_numpy(v.ravel()).cuda(), torch.from_numpy(x.ravel()).cuda()
    n = lb.k_nodes(dv, dx).cpu().numpy()
    k = lb.k_terms(dv, dx).cpu().numpy()
    # order 0 runs its expansions; other orders Temme's series up to x = 1.25
    # and the integral above
    series = (v.ravel() != 0.0) & (x.ravel() <= 1.25)
    integral = (v.ravel() != 0.0) & (x.ravel() > 1.25)
    assert n[integral].min() > 0 and n.max() < 400 and not n[~integral].any()
    assert k[series].min() >= 1 and k.max() <= 20 and not k[~series].any()


def test_node_counts_on_the_stress_grid(lb):
    from paper_2409_08729_amd import workloads as wl
    v, x = wl.m3(1 << 20)
    dv, dx = torch.from_numpy(v).cuda(), torch.from_numpy(x).cuda()
    n = lb.k_nodes(dv, dx).cpu().numpy()
    k = lb.k_terms(dv, dx).cpu().numpy()
    fb = n > 0
    tm = k > 0
    assert not (fb & tm).any()
    # ~39% of the grid is in the fallback region, ~78% of it at x <= 1.25
    assert 0.05 < fb.mean() < 0.15 and 0.25 < tm.mean() < 0.40, (fb.mean(), tm.mean())
    assert 10 < n[fb].mean() < 40 and n.max() < 400, (n[fb].mean(), n.max())
    assert 2 < k[tm].mean() < 8 and k.max() <= 20, (k[tm].mean(), k.max())
    assert x[tm].max() <= 1.25 and x[fb].min() > 1.25


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_temme_region(lb, oracle, dtype):
    """Temme's series over its whole region: x log-spaced from the
    small-argument switch to its bound 1.25 (and one ulp either side of
    both), orders whose fractional part mu = v - rint(v) sits at 0 +- 1e-12,
    +-1e-6, +-1/4 and +-1/2 (rint rounds halves to even), for every order
    step 0..14, against the oracle."""
    xs = np.concatenate([10 ** np.linspace(-10, np.log10(1.25), 60),
                         [1e-10, np.nextafter(1e-10, 1), np.nextafter(1.25, 0), 1.25,
                          np.nextafter(1.25, 2)]])
    base = np.arange(0.0, 15.0)
    off = np.array([1e-12, -1e-12, 1e-6, -1e-6, 0.25, -0.25, 0.5, -0.4999999, 0.123])
    vs = (base[:, None] + off[None, :]).ravel()
    vs = vs[(vs > 0) & (vs <= 14.5)]
    v, x = np.meshgrid(vs, xs)
    e = _check(lb, oracle, v.ravel(), x.ravel(), dtype)
    i = int(np.argmax(e))
    tol = TOL64 if dtype == torch.float64 else TOL32
    assert e.max() <= tol, (e.max(), v.ravel()[i], x.ravel()[i])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_temme_random(lb, oracle, dtype):
    g = np.random.default_rng(41)
    v = g.uniform(0.0, 14.5, 6000)
    x = np.concatenate([10 ** g.uniform(-10, np.log10(1.25), 3000), g.uniform(0.0, 1.25, 3000)])
    x = np.maximum(x, 1e-10)
    e = _check(lb, oracle, v, x, dtype)
    assert e.max() <= (TOL64 if dtype == torch.float64 else TOL32), e.max()


def test_temme_term_counts_binary32(lb):
    """Binary32 Temme elements stop at the binary32 truncation (fewer terms
    than binary64 on the same points) and run no integral."""
    g = np.random.default_rng(42)
    v = torch.from_numpy(g.uniform(0.0, 8.9, 4000)).cuda()
    x = torch.from_numpy(10 ** g.uniform(-6, np.log10(1.25), 4000)).cuda()
    v = v[(v - v.round()).abs() > 1e-3]
    x = x[:v.numel()]
    k64 = lb.k_terms(v, x)
    k32 = lb.k_terms(v.float(), x.float())
    assert int(k64.min()) >= 1 and int(k32.min()) >= 1
    assert (k32 <= k64).all() and float(k32.double().mean()) < float(k64.double().mean())
    assert int(lb.k_nodes(v.float(), x.float()).max()) == 0
