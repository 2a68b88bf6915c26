"""The log K fallback on the GPU against values fixed outside the oracle.

The fallback (x >= 1e-10) runs the order recurrence from K_0, K_1 at integer
orders, Temme's series at the fractional order plus the same recurrence up to
x = 1.25, and above it the trapezoid rule on K_v(x) = int_0^inf
exp(-x cosh t) cosh(v t) dt; below x = 1e-10 the small-argument form.  The
oracle integrates that same integral, so these tests pin the GPU result on
the fallback's whole region without it (half-integer orders are Temme's
series at mu = +-1/2 up to x = 1.25, integer orders the integer-order path):
  * half-integer orders n + 1/2, n = 0..14: the finite sum of DLMF 10.49.12;
  * integer orders n = 0..14: the expansion of DLMF 10.31.1;
both evaluated in decimal arithmetic (tests/closed_forms.py) on a dense
log grid of x in [1e-10, 17.5] plus tiny arguments down to 1e-300; and
  * the Wronskian I_v K_{v+1} + I_{v+1} K_v = 1/x (DLMF 10.28.2) on the GPU's
own outputs, log I from the series branch and log K from the fallback, over
the fallback region: log(I_v K_{v+1} + I_{v+1} K_v) + log x = 0.
"""
import numpy as np
import pytest
import torch

import closed_forms as cf
from parity import TOL32, TOL64, summary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the -m gpu tests need an MI355X")
    import paper_2409_08729_amd as m
    m.lib()
    return m


def _grid(dtype):
    """(v, x, closed-form log K as float64 from 60+ digits) at 2 x 15 orders."""
    xs = np.concatenate([10 ** np.linspace(-10, np.log10(17.5), 40),
                         10 ** np.linspace(-300, -10.5, 6)])
    xs = xs.astype(dtype).astype(np.float64)       # the closed forms at the exact inputs
    xs = xs[xs >= (1e-37 if dtype == np.float32 else 1e-300)]   # normal numbers only
    v, x, ref = [], [], []
    for n in range(15):
        for xx in xs:
            v.append(n + 0.5)
            x.append(xx)
            ref.append(float(cf.log_kv_half(n, xx)))
            v.append(float(n))
            x.append(xx)
            ref.append(float(cf.log_kn_int(n, xx)))
    return np.array(v), np.array(x), np.array(ref)


@pytest.fixture(scope="module")
def grid64():
    return _grid(np.float64)


@pytest.fixture(scope="module")
def grid32():
    return _grid(np.float32)


def test_log_kv_f64_closed_forms(lb, grid64):
    v, x, ref = grid64
    y = lb.log_kv(torch.from_numpy(v).to("cuda:0"), torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    e = np.abs(y - ref) / np.maximum(np.abs(ref), 1 + np.hypot(v, x))
    i = int(np.argmax(e))
    print(f"K f64 closed forms n={v.size}: {summary(e)}")
    assert v.size >= 1000
    assert e.max() <= TOL64, (v[i], x[i], y[i], ref[i], e[i])


def test_log_kv_f32_closed_forms(lb, grid32):
    v, x, ref = grid32
    y = lb.log_kv(torch.from_numpy(v.astype(np.float32)).to("cuda:0"),
                  torch.from_numpy(x.astype(np.float32)).to("cuda:0")).cpu().numpy()
    y = y.astype(np.float64)
    m = np.abs(ref) < float(np.finfo(np.float32).max)
    e = np.abs(y[m] - ref[m]) / np.maximum(np.abs(ref[m]), 1 + np.hypot(v[m], x[m]))
    i = int(np.argmax(e))
    print(f"K f32 closed forms n={m.sum()}: {summary(e)}")
    assert e.max() <= TOL32, (v[m][i], x[m][i], y[m][i], ref[m][i], e[i])


def _wronskian(lb, v, x, dtype):
    """log(I_v K_{v+1} + I_{v+1} K_v) + log x from the GPU's log-values, and
    its error bound from the parity bar of the four log-values."""
    t = lambda a: torch.from_numpy(a.astype(dtype)).to("cuda:0")
    li0 = lb.log_iv(t(v), t(x)).cpu().numpy().astype(np.float64)
    li1 = lb.log_iv(t(v + 1), t(x)).cpu().numpy().astype(np.float64)
    lk0 = lb.log_kv(t(v), t(x)).cpu().numpy().astype(np.float64)
    lk1 = lb.log_kv(t(v + 1), t(x)).cpu().numpy().astype(np.float64)
    w = np.logaddexp(li0 + lk1, li1 + lk0) + np.log(x)
    s = lambda y, vv: np.maximum(np.abs(y), 1 + np.hypot(vv, x))
    bound = np.maximum(s(li0, v) + s(lk1, v + 1), s(li1, v + 1) + s(lk0, v))
    return w, bound


def test_wronskian_on_fallback_region_f64(lb):
    g = np.random.default_rng(401)
    v = g.uniform(0.0, 13.5, 4096)
    x = 10 ** g.uniform(-10, np.log10(17.5), 4096)
    br = lb.classify("K", torch.from_numpy(v).to("cuda:0"),
                     torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    assert (br == 2).all()                       # every point on the K fallback
    w, bound = _wronskian(lb, v, x, np.float64)
    r = np.abs(w) / bound
    i = int(np.argmax(r))
    print(f"Wronskian f64 n={v.size}: |W| {summary(np.abs(w))}; |W|/bound max {r.max():.3e}")
    assert (np.abs(w) <= TOL64 * bound + 4e-16 * np.abs(np.log(x))).all(), (v[i], x[i], w[i])


def test_wronskian_on_fallback_region_f32(lb):
    g = np.random.default_rng(402)
    v = g.uniform(0.0, 8.0, 4096).astype(np.float32).astype(np.float64)
    x = (10 ** g.uniform(-10, np.log10(7.0), 4096)).astype(np.float32).astype(np.float64)
    w, bound = _wronskian(lb, v, x, np.float32)
    r = np.abs(w) / bound
    i = int(np.argmax(r))
    print(f"Wronskian f32 n={v.size}: |W|/bound max {r.max():.3e}")
    assert (np.abs(w) <= TOL32 * bound + 2e-7 * np.abs(np.log(x))).all(), (v[i], x[i], w[i])
