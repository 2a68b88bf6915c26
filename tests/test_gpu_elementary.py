"""The library's binary64 elementary functions as the kernels run them
(lbessel_elementary_f64: the hardware reciprocal and inverse square root with
two Newton steps each, the exp and log sequences of csrc/lbessel_fastmath.hpp), in units in the last
place against 60-digit references from Python's decimal module."""
import math
from decimal import Decimal, localcontext

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the -m gpu tests need an MI355X")
    import paper_2409_08729_amd as m
    m.lib()
    return m


def _ref(op, a):
    with localcontext() as ctx:
        ctx.prec = 60
        d = Decimal(a)
        if op == "rcp":
            return 1 / d
        if op == "rsqrt":
            return 1 / d.sqrt()
        if op in ("exp", "exp_bounded"):
            return d.exp()
        if op == "log":
            return d.ln()
        if d < Decimal("1e-20"):
            return d - d * d / 2 + d * d * d / 3
        return (1 + d).ln()


def _worst(lb, op, xs):
    a = np.asarray(xs, dtype=np.float64)
    y = lb.elementary(op, torch.from_numpy(a).cuda()).cpu().numpy()
    worst = 0.0
    for got, x in zip(y, a):
        ref = _ref(op, float(x))
        worst = max(worst, float(abs(Decimal(float(got)) - ref) / Decimal(math.ulp(float(ref)))))
    return worst


def test_reciprocal_within_one_ulp(lb):
    g = np.random.default_rng(11)
    k = np.arange(1.0, 41.0)
    xs = np.concatenate([10.0 ** g.uniform(-300, 300, 3000), -(10.0 ** g.uniform(-30, 30, 500)),
                         g.uniform(0.5, 2.0, 1000), (k * k)[:, None].ravel() - g.uniform(0, 0.25, 40),
                         [1.0, 2.0, 3.0, 0.1, 1e-300, 1e300]])
    assert _worst(lb, "rcp", xs) <= 1.0


def test_inverse_square_root_within_one_ulp(lb):
    """The Debye branch's 1/sqrt(v^2 + x^2): arguments from 1e-2 (v > 0.1) to
    2e300, around powers of two and exact squares."""
    g = np.random.default_rng(16)
    k = np.arange(1.0, 41.0)
    xs = np.concatenate([10.0 ** g.uniform(-2, 300, 3000), g.uniform(0.5, 4.0, 1000),
                         k * k, np.nextafter(k * k, 0), np.nextafter(k * k, 2e3),
                         [1.0, 2.0, 4.0, 0.01, 2e300]])
    assert _worst(lb, "rsqrt", xs) <= 1.0


@pytest.mark.parametrize("op", ["exp", "exp_bounded"])
def test_exp_within_one_ulp(lb, op):
    g = np.random.default_rng(12)
    xs = np.concatenate([g.uniform(-700.0, 700.0, 2000), g.uniform(-12.0, 12.0, 1500),
                         g.uniform(-1e-3, 1e-3, 500), [0.0, 1e-300, -1e-300, 709.0, -708.0]])
    assert _worst(lb, op, xs) <= 1.0


def test_log_within_one_ulp(lb):
    g = np.random.default_rng(13)
    xs = np.concatenate([10.0 ** g.uniform(-300, 300, 2500), 1.0 + g.uniform(-0.3, 0.3, 1000),
                         [5e-324, 2.2250738585072014e-308, 1.0, 2.0, 0.5,
                          math.nextafter(1.0, 2.0), math.nextafter(1.0, 0.0), 1.7e308]])
    assert _worst(lb, "log", xs) <= 1.0


def test_log1p_keeps_relative_accuracy(lb):
    g = np.random.default_rng(14)
    xs = np.concatenate([10.0 ** g.uniform(-40.0, 12.0, 3000),
                         [0.0, 5e-324, 1e-300, 2.0 ** -53, 2.0 ** -52, 1.0, 1e300]])
    assert _worst(lb, "log1p", xs) <= 1.5
