"""Scalar-order entry points: orders 0 and 1 take the polynomial fast path
(checked against the binary128 oracle, f64 and f32, over the whole argument
range and across every internal boundary); integer orders 2..14 of I take the
integer-order path (constant-coefficient series; oracle-checked, and equal to
the general path's bits outside its series region), those of K the general
path, whose fallback runs the forward recurrence from K_0 and K_1 (oracle-
checked, the array path's bits everywhere); any other order runs the general
path with v broadcast and must give the array path's bits.  The array path of log K runs
the same integer-order code for integer orders 0..14 at x >= 1e-10, also
inside tiles that mix them with other orders."""
import numpy as np
import pytest
import torch

from parity import TOL32, TOL64, cond_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the -m gpu tests need an MI355X")
    import paper_2409_08729_amd as m
    m.lib()
    return m


def _xgrid(seed=0):
    g = np.random.default_rng(seed)
    parts = [10 ** g.uniform(-300, -10, 300), 10 ** g.uniform(-10, np.log10(2.0), 3000),
             g.uniform(2.0, 22.0, 3000), 10 ** g.uniform(np.log10(22.0), 4, 2000)]
    edges = []
    for b in (2.0, 7.5, 9.5, 17.5, 21.5):
        edges += [np.nextafter(b, 0), b, np.nextafter(b, 100), b * (1 - 1e-9), b * (1 + 1e-9)]
    # the oracle covers x <= 1e12 (I) and 1e15 (K); larger x is checked against
    # the leading Hankel term in test_order_fast_path_huge_x
    return np.concatenate(parts + [np.array(edges), np.array([5e-324, 2.2e-308, 1e11])])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("v", [0.0, 1.0])
@pytest.mark.parametrize("kind", ["I", "K"])
def test_orders_0_and_1_match_oracle(lb, oracle, kind, v, dtype):
    x = _xgrid()
    if kind == "I":
        x = x[x <= 700.0] if dtype == torch.float32 else x
    if dtype == torch.float32:
        x = x.astype(np.float32)
        x = x[(x > 0) & np.isfinite(x)]
    dx = torch.from_numpy(x).to("cuda:0")
    y = (lb.log_iv_order if kind == "I" else lb.log_kv_order)(v, dx).cpu().numpy()
    xd = x.astype(np.float64)
    hi, lo = (oracle.log_iv if kind == "I" else oracle.log_kv)(np.full(xd.size, v), xd)
    fin = np.isfinite(hi)
    assert np.array_equal(np.isfinite(y), fin)
    tol = TOL64 if dtype == torch.float64 else TOL32
    e = cond_err(y.astype(np.float64)[fin], hi[fin], lo[fin], np.full(fin.sum(), v), xd[fin])
    i = int(np.argmax(e))
    assert e.max() <= tol, (kind, v, dtype, e.max(), xd[fin][i])


@pytest.mark.parametrize("kind", ["I", "K"])
def test_order_fast_path_specials(lb, kind):
    x = torch.tensor([0.0, np.inf, np.nan, -1.0], dtype=torch.float64, device="cuda:0")
    for v in (0.0, 1.0):
        y = (lb.log_iv_order if kind == "I" else lb.log_kv_order)(v, x).cpu().numpy()
        ref = (lb.log_iv if kind == "I" else lb.log_kv)(torch.full_like(x, v), x).cpu().numpy()
        assert np.array_equal(np.isnan(y), np.isnan(ref)) and np.array_equal(
            np.nan_to_num(y), np.nan_to_num(ref)), (kind, v, y, ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["I", "K"])
def test_other_orders_equal_array_path_bitwise(lb, kind, dtype):
    x = torch.from_numpy(_xgrid(1)).to("cuda:0", dtype)
    f_ord = lb.log_iv_order if kind == "I" else lb.log_kv_order
    f_arr = lb.log_iv if kind == "I" else lb.log_kv
    it = torch.int64 if dtype == torch.float64 else torch.int32
    for v in (0.5, 2.5, 7.25, 15.0, 30.0, 1e3):
        a = f_ord(v, x)
        b = f_arr(torch.full_like(x, v), x)
        assert torch.equal(a.view(it), b.view(it)), (kind, v)


@pytest.mark.parametrize("kind", ["I", "K"])
def test_fast_path_hankel_region_equals_general_path(lb, kind):
    # above the Hankel threshold both paths run the same mu_20 code
    x = torch.linspace(22.0, 5000.0, 10007, dtype=torch.float64, device="cuda:0")
    for v in (0.0, 1.0):
        a = (lb.log_iv_order if kind == "I" else lb.log_kv_order)(v, x)
        b = (lb.log_iv if kind == "I" else lb.log_kv)(torch.full_like(x, v), x)
        assert torch.equal(a.view(torch.int64), b.view(torch.int64))


def test_k_order_is_even(lb):
    x = torch.from_numpy(_xgrid(2)).to("cuda:0")
    for v in (1.0, 3.5):
        assert torch.equal(lb.log_kv_order(-v, x).view(torch.int64),
                           lb.log_kv_order(v, x).view(torch.int64))


@pytest.mark.parametrize("kind", ["I", "K"])
def test_order_fast_path_huge_x(lb, kind):
    x = np.array([1e15, 1e100, 1e200, 1e308])
    for v in (0.0, 1.0):
        y = (lb.log_iv_order if kind == "I" else lb.log_kv_order)(
            v, torch.from_numpy(x).cuda()).cpu().numpy()
        lead = (x - 0.5 * (np.log(2 * np.pi) + np.log(x)) if kind == "I"
                else 0.5 * (np.log(np.pi / 2) - np.log(x)) - x)
        assert np.all(np.abs(y - lead) <= 4e-15 * np.abs(lead) + 1e-14), (kind, v, y, lead)


INT_ORDERS = list(range(2, 15))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["I", "K"])
def test_integer_orders_match_oracle(lb, oracle, kind, dtype):
    """Orders 2..14 on a seeded 700-point share of the argument grid each
    (tiny, series/integral region, every internal boundary, Hankel/Debye
    regions), against the binary128 oracle at the (f32-rounded) inputs."""
    xs = _xgrid(5)
    g = np.random.default_rng(6)
    f = lb.log_iv_order if kind == "I" else lb.log_kv_order
    tol = TOL64 if dtype == torch.float64 else TOL32
    for n in INT_ORDERS:
        x = np.concatenate([g.choice(xs, 700, replace=False),
                            [1e-10, np.nextafter(1e-10, 1), 2.0, 7.0, 7.5, 17.5, 20.0, 23.0]])
        if kind == "I" and dtype == torch.float32:
            x = x[x <= 700.0]
        if dtype == torch.float32:
            x = x.astype(np.float32)
            x = x[(x > 0) & np.isfinite(x)]
        y = f(float(n), torch.from_numpy(x).to("cuda:0")).cpu().numpy()
        xd = x.astype(np.float64)
        vd = np.full(xd.size, float(n))
        hi, lo = (oracle.log_iv if kind == "I" else oracle.log_kv)(vd, xd)
        fin = np.isfinite(hi)
        assert np.array_equal(np.isfinite(y), fin), (kind, n)
        e = cond_err(y.astype(np.float64)[fin], hi[fin], lo[fin], vd[fin], xd[fin])
        assert e.max() <= tol, (kind, n, dtype, e.max(), xd[fin][int(np.argmax(e))])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["I", "K"])
def test_integer_orders_outside_their_region_equal_general_path(lb, kind, dtype):
    """Where the general path runs the Hankel or Debye branch for order n,
    the integer-order path of I runs the same code: same bits; K's scalar
    integer orders run the general path itself, so every element matches;
    also the special values and negative orders for K."""
    x = torch.from_numpy(_xgrid(7)).to("cuda:0", dtype)
    f_ord = lb.log_iv_order if kind == "I" else lb.log_kv_order
    f_arr = lb.log_iv if kind == "I" else lb.log_kv
    it = torch.int64 if dtype == torch.float64 else torch.int32
    for n in INT_ORDERS:
        vv = torch.full_like(x, float(n))
        br = lb.classify(kind, vv, x)
        keep = (br != 2) if kind == "I" else torch.ones_like(br, dtype=torch.bool)
        a = f_ord(float(n), x)
        b = f_arr(vv, x)
        assert torch.equal(a[keep].view(it), b[keep].view(it)), (kind, n)
        if kind == "K":
            assert torch.equal(lb.log_kv_order(-float(n), x).view(it), a.view(it))
    sp = torch.tensor([0.0, np.inf, np.nan, -1.0], dtype=dtype, device="cuda:0")
    for n in (2, 14):
        y = f_ord(float(n), sp).cpu().numpy()
        ref = f_arr(torch.full_like(sp, float(n)), sp).cpu().numpy()
        assert np.array_equal(np.isnan(y), np.isnan(ref)) and np.array_equal(
            np.nan_to_num(y), np.nan_to_num(ref)), (kind, n, y, ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_k_array_path_integer_orders_in_mixed_tiles(lb, oracle, dtype):
    """Integer orders 0..14 interleaved with non-integer orders (and orders
    one ulp off an integer) in one array: oracle parity everywhere, and the
    integer elements at x >= 1e-10 give the bits of the scalar-order path."""
    g = np.random.default_rng(8)
    n = 12000
    x = _xgrid(9)
    x = g.choice(x[x <= 1e12], n)
    ints = g.integers(0, 15, n).astype(np.float64)
    v = np.where(g.random(n) < 0.5, ints, g.uniform(0.0, 16.0, n))
    near = g.random(n) < 0.05
    v = np.where(near, np.nextafter(ints, 20.0), v)
    np_dt = np.float64 if dtype == torch.float64 else np.float32
    v = v.astype(np_dt)
    x = x.astype(np_dt)
    keep = (x > 0) & np.isfinite(x)
    v, x = v[keep], x[keep]
    dv = torch.from_numpy(v).to("cuda:0")
    dx = torch.from_numpy(x).to("cuda:0")
    y = lb.log_kv(dv, dx).cpu().numpy()
    vd, xd = v.astype(np.float64), x.astype(np.float64)
    hi, lo = oracle.log_kv(vd, xd)
    fin = np.isfinite(hi)
    assert np.array_equal(np.isfinite(y), fin)
    tol = TOL64 if dtype == torch.float64 else TOL32
    e = cond_err(y.astype(np.float64)[fin], hi[fin], lo[fin], vd[fin], xd[fin])
    assert e.max() <= tol, (dtype, e.max(), vd[fin][int(np.argmax(e))], xd[fin][int(np.argmax(e))])
    it = torch.int64 if dtype == torch.float64 else torch.int32
    for k in range(15):
        m = (v == k) & (x >= 1e-10)
        if not m.any():
            continue
        a = lb.log_kv_order(float(k), dx[torch.from_numpy(m).to("cuda:0")])
        b = torch.from_numpy(y[m]).to("cuda:0")
        assert torch.equal(a.view(it), b.view(it)), (k, dtype)
