"""Pins of the binary128 oracle against facts fixed outside it.

Each test compares the oracle with mathematics it does not use itself:
closed forms (DLMF 10.49.8/10.49.12, 10.31.1), brute-force linear summation of
the defining series at exact Gamma values, the Wronskian and the three-term
recurrences (which tie the independent I and K oracles together), the
derivative identities, and the small- and large-argument limits.  The paper
(arXiv 2409.08729) prints no function values, so no stored paper value exists
to pin against.
"""
from decimal import Decimal, localcontext

import numpy as np
import pytest

import closed_forms as cf


def qd(hi, lo):
    """The oracle's (hi, lo) pair as an exact Decimal."""
    return Decimal(float(hi)) + Decimal(float(lo))


def close(ref: Decimal, got: Decimal, rel: float) -> bool:
    with localcontext() as ctx:
        ctx.prec = 60
        return abs(ref - got) <= Decimal(rel) * max(Decimal(1), abs(ref))


REL = 1e-26   # binary128 oracle vs >= 60-digit closed forms


# --------------------------------------------------------------------------
# closed forms at half-integer order
# --------------------------------------------------------------------------

KHALF = [(0, 1.0), (0, 1e-4), (0, 1e4), (1, 0.3), (3, 0.5), (7, 19.7), (10, 30.0),
         (12, 1e-3), (25, 100.0), (100, 7.0), (2000, 1e3), (5000, 0.5), (9999, 1e4)]


@pytest.mark.parametrize("n,x", KHALF)
def test_log_kv_half_integer_closed_form(oracle, n, x):
    ref = cf.log_kv_half(n, x)
    hi, lo = oracle.log_kv(n + 0.5, x)
    assert close(ref, qd(hi[0], lo[0]), REL), (n, x, float(ref), hi[0])


IHALF = [(0, 1.0), (0, 1e-3), (0, 500.0), (1, 0.7), (3, 0.5), (10, 30.0), (20, 2.0),
         (12, 19.7), (15, 0.9), (40, 80.0)]


@pytest.mark.parametrize("n,x", IHALF)
def test_log_iv_half_integer_closed_form(oracle, n, x):
    ref = cf.log_iv_half(n, x, prec=260)
    hi, lo = oracle.log_iv(n + 0.5, x)
    assert close(ref, qd(hi[0], lo[0]), REL), (n, x, float(ref), hi[0])


# --------------------------------------------------------------------------
# brute-force linear summation of the defining series (exact Gamma values)
# --------------------------------------------------------------------------

SERIES = [(0, 1.0), (0, 0.01), (2, 1.518), (2, 99.5), (1, 2.0), (5, 40.0), (4, 11.997),
          (16, 22.767), (64, 1.0), (256, 86.746), (2048, 99.0), (2048, 1.0), (41, 0.3)]


@pytest.mark.parametrize("v2,x", SERIES)
def test_log_iv_brute_force_series(oracle, v2, x):
    ref = cf.log_iv_series(v2, x)
    hi, lo = oracle.log_iv(v2 / 2, x)
    assert close(ref, qd(hi[0], lo[0]), REL), (v2, x, float(ref), hi[0])


# --------------------------------------------------------------------------
# integer order K_n from DLMF 10.31.1
# --------------------------------------------------------------------------

KINT = [(0, 1.0), (0, 1e-4), (1, 0.1), (1, 3.0), (2, 2.365), (4, 5.0), (8, 12.0),
        (16, 10.0), (32, 0.5), (3, 18.0)]


@pytest.mark.parametrize("n,x", KINT)
def test_log_kv_integer_order_series(oracle, n, x):
    ref = cf.log_kn_int(n, x, prec=110)
    hi, lo = oracle.log_kv(float(n), x)
    assert close(ref, qd(hi[0], lo[0]), REL), (n, x, float(ref), hi[0])


def test_euler_gamma_and_pi_generators():
    # Self-consistency of the two constants the closed forms use: two different
    # truncations must agree, and pi must satisfy sin(pi/6) = 1/2 via its series.
    g1 = cf.euler_gamma(60)
    assert str(g1).startswith("0.5772156649015328606065120900824024310421")
    p = cf.pi_dec(60)
    with localcontext() as ctx:
        ctx.prec = 70
        y = p / 6
        s, t, k = Decimal(0), y, 0
        while abs(t) > Decimal(10) ** -68:
            s += t
            k += 1
            t = -t * y * y / ((2 * k) * (2 * k + 1))
        assert abs(s - Decimal("0.5")) < Decimal(10) ** -55


# --------------------------------------------------------------------------
# identities that tie O-I and O-K together at general (v, x)
# --------------------------------------------------------------------------

def _exact_shift(v):
    """Round orders to multiples of 2^-30 so that v - 1 and v + 1 are exact doubles."""
    return np.round(v * 2.0 ** 30) / 2.0 ** 30


def _general_points(n=48, seed=11):
    rng = np.random.default_rng(seed)
    v = np.concatenate([10 ** rng.uniform(-3, 4, n), rng.uniform(0, 20, n)])
    x = np.concatenate([10 ** rng.uniform(-4, 4, n), rng.uniform(0.5, 60, n)])
    return _exact_shift(v), x


def test_wronskian(oracle):
    """I_v K_{v+1} + I_{v+1} K_v = 1/x (DLMF 10.28.2), both terms positive."""
    v, x = _general_points()
    li0 = oracle.log_iv(v, x)
    li1 = oracle.log_iv(v + 1, x)
    lk0 = oracle.log_kv(v, x)
    lk1 = oracle.log_kv(v + 1, x)
    with localcontext() as ctx:
        ctx.prec = 60
        for i in range(v.size):
            a = qd(li0[0][i], li0[1][i]) + qd(lk1[0][i], lk1[1][i])
            b = qd(li1[0][i], li1[1][i]) + qd(lk0[0][i], lk0[1][i])
            m = max(a, b)
            lse = m + ((a - m).exp() + (b - m).exp()).ln()
            target = -Decimal(float(x[i])).ln()
            scale = max(Decimal(1), abs(qd(li0[0][i], li0[1][i])), abs(qd(lk0[0][i], lk0[1][i])))
            assert abs(lse - target) <= Decimal(1e-27) * scale, (v[i], x[i], float(lse - target))


def test_recurrences(oracle):
    """I_{v-1} - I_{v+1} = (2v/x) I_v and K_{v+1} - K_{v-1} = (2v/x) K_v (DLMF 10.29.1)."""
    rng = np.random.default_rng(5)
    v = _exact_shift(rng.uniform(1, 60, 40))
    x = 10 ** rng.uniform(-2, 2.5, 40)
    lim = oracle.log_iv(v - 1, x)
    li = oracle.log_iv(v, x)
    lip = oracle.log_iv(v + 1, x)
    lkm = oracle.log_kv(v - 1, x)
    lk = oracle.log_kv(v, x)
    lkp = oracle.log_kv(v + 1, x)
    with localcontext() as ctx:
        ctx.prec = 60
        for i in range(v.size):
            c = Decimal(2 * float(v[i])) / Decimal(float(x[i]))
            a = (qd(lim[0][i], lim[1][i]) - qd(li[0][i], li[1][i])).exp()
            b = (qd(lip[0][i], lip[1][i]) - qd(li[0][i], li[1][i])).exp()
            assert abs((a - b) - c) <= Decimal(1e-26) * max(a, b, Decimal(1)), (v[i], x[i])
            a = (qd(lkp[0][i], lkp[1][i]) - qd(lk[0][i], lk[1][i])).exp()
            b = (qd(lkm[0][i], lkm[1][i]) - qd(lk[0][i], lk[1][i])).exp()
            assert abs((a - b) - c) <= Decimal(1e-26) * max(a, b, Decimal(1)), (v[i], x[i])


def test_k_is_even_in_order(oracle):
    v = np.array([0.3, 2.5, 17.0, 1234.5])
    x = np.array([0.2, 3.0, 40.0, 900.0])
    a = oracle.log_kv(v, x)
    b = oracle.log_kv(-v, x)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# --------------------------------------------------------------------------
# limits
# --------------------------------------------------------------------------

def test_small_x_limits(oracle):
    """log I_v ~ v log(x/2) - lnGamma(v+1); log K_v ~ lnGamma(v) - log 2 + v log(2/x);
    K_0 ~ -log(x/2) - gamma (DLMF 10.30.1-3), at x where the next term is < 1e-30."""
    x = 1e-16
    with localcontext() as ctx:
        ctx.prec = 60
        lhx = (Decimal(x) / 2).ln()
        for n in (0, 1, 3, 10):
            hi, lo = oracle.log_iv(float(n), x)
            ref = n * lhx - cf.log_factorial(n)
            assert abs(qd(hi[0], lo[0]) - ref) <= Decimal(1e-28) * max(1, abs(ref))
        for n in (3, 10):                          # K_n: next term relative x^2/(4(n-1))
            hi, lo = oracle.log_kv(float(n), x)
            ref = cf.log_factorial(n - 1) - Decimal(2).ln() - n * lhx
            assert abs(qd(hi[0], lo[0]) - ref) <= Decimal(1e-28) * abs(ref)
        hi, lo = oracle.log_kv(0.0, x)
        ref = (-lhx - cf.euler_gamma(60)).ln()
        assert abs(qd(hi[0], lo[0]) - ref) <= Decimal(1e-28)


def test_large_x_hankel_limit_k(oracle):
    """log K_v(x) = 1/2 log(pi/2x) - x + log sum_k a_k(v)/x^k (DLMF 10.40.2) at x = 1e6,
    where ten terms leave a remainder far below 1e-40."""
    x = 1e6
    with localcontext() as ctx:
        ctx.prec = 60
        xd = Decimal(x)
        for v in (0.0, 0.25, 1.0, 3.7):
            mu = 4 * Decimal(v) ** 2
            s, a = Decimal(1), Decimal(1)
            for k in range(1, 11):
                a = a * (mu - (2 * k - 1) ** 2) / (k * 8 * xd)
                s += a
            ref = (cf.pi_dec(60) / (2 * xd)).ln() / 2 - xd + s.ln()
            hi, lo = oracle.log_kv(v, x)
            assert abs(qd(hi[0], lo[0]) - ref) <= Decimal(1e-26) * abs(ref), v


# --------------------------------------------------------------------------
# derivatives
# --------------------------------------------------------------------------

def test_derivative_identities(oracle):
    """I_v' = I_{v+1} + (v/x) I_v and K_v' = -K_{v+1} + (v/x) K_v (DLMF 10.29.2):
    the oracle's derivatives come from the differentiated series / integrand,
    not from these identities."""
    v, x = _general_points(24, seed=3)
    di = oracle.dlog_iv(v, x)
    dk = oracle.dlog_kv(v, x)
    li0 = oracle.log_iv(v, x)
    li1 = oracle.log_iv(v + 1, x)
    lk0 = oracle.log_kv(v, x)
    lk1 = oracle.log_kv(v + 1, x)
    with localcontext() as ctx:
        ctx.prec = 60
        for i in range(v.size):
            vx = Decimal(float(v[i])) / Decimal(float(x[i]))
            ri = (qd(li1[0][i], li1[1][i]) - qd(li0[0][i], li0[1][i])).exp() + vx
            rk = -(qd(lk1[0][i], lk1[1][i]) - qd(lk0[0][i], lk0[1][i])).exp() + vx
            gi = qd(di[0][i], di[1][i])
            gk = qd(dk[0][i], dk[1][i])
            si = max(abs(ri), Decimal(1)) * max(Decimal(1), abs(qd(li0[0][i], li0[1][i])))
            sk = max(abs(rk), vx, Decimal(1)) * max(Decimal(1), abs(qd(lk0[0][i], lk0[1][i])))
            assert abs(gi - ri) <= Decimal(1e-25) * si, (v[i], x[i], float(gi), float(ri))
            assert abs(gk - rk) <= Decimal(1e-25) * sk, (v[i], x[i], float(gk), float(rk))


def test_derivative_finite_difference(oracle):
    """Fourth-order central differences of the log-values agree with the derivatives."""
    v = np.array([0.0, 0.5, 3.0, 12.0, 40.0, 300.0])
    x = np.array([0.7, 5.0, 20.0, 9.0, 55.0, 250.0])
    h = 1e-4 * x
    for f, df in ((oracle.log_iv, oracle.dlog_iv), (oracle.log_kv, oracle.dlog_kv)):
        vals = [qd(*map(lambda a: a[0], f(v[i:i + 1], x[i:i + 1] + s * h[i:i + 1])))
                for i in range(v.size) for s in (-2, -1, 1, 2)]
        d = df(v, x)
        for i in range(v.size):
            m2, m1, p1, p2 = vals[4 * i:4 * i + 4]
            hd = Decimal(float(x[i] + h[i])) - Decimal(float(x[i]))  # exact grid spacing
            fd = (m2 - 8 * m1 + 8 * p1 - p2) / (12 * hd)
            g = qd(d[0][i], d[1][i])
            assert abs(fd - g) <= Decimal(1e-12) * max(Decimal(1), abs(g)), (i, float(fd), float(g))


# --------------------------------------------------------------------------
# von Mises-Fisher normaliser
# --------------------------------------------------------------------------

def test_vmf_closed_forms(oracle):
    """p = 3: C_3(k) = k / (4 pi sinh k); k = 0: the uniform density 1/|S^{p-1}|,
    |S^{p-1}| = 2 pi^{p/2} / Gamma(p/2)."""
    k = np.array([1e-3, 0.5, 3.0, 40.0, 700.0])
    hi, lo = oracle.vmf_log_norm(k, 3.0)
    with localcontext() as ctx:
        ctx.prec = 60
        for i in range(k.size):
            kd = Decimal(float(k[i]))
            sinh = (kd.exp() - (-kd).exp()) / 2
            ref = kd.ln() - (4 * cf.pi_dec(60)).ln() - sinh.ln()
            assert abs(qd(hi[i], lo[i]) - ref) <= Decimal(1e-26) * max(1, abs(ref))
        for p in (2, 4, 2048, 8192):
            hi, lo = oracle.vmf_log_norm(np.array([0.0]), float(p))
            # log Gamma(p/2) - log 2 - (p/2) log pi with p even: Gamma(p/2) = (p/2-1)!
            ref = cf.log_factorial(p // 2 - 1) - Decimal(2).ln() - Decimal(p) / 2 * cf.pi_dec(60).ln()
            assert abs(qd(hi[0], lo[0]) - ref) <= Decimal(1e-26) * max(1, abs(ref)), p


# --------------------------------------------------------------------------
# special values (the convention both sides implement)
# --------------------------------------------------------------------------

def test_special_values(oracle):
    inf, nan = np.inf, np.nan
    v = np.array([0.0, 2.0, -1.0, 1.0, nan, 1.0, 3.0, inf])
    x = np.array([0.0, 0.0, 1.0, -1.0, 1.0, nan, inf, 1.0])
    hi, lo = oracle.log_iv(v, x)
    exp_i = [0.0, -inf, nan, nan, nan, nan, inf, -inf]
    np.testing.assert_array_equal(hi, np.array(exp_i))
    v = np.array([0.0, 2.0, -2.5, 1.0, nan, 1.0, 3.0, inf])
    x = np.array([0.0, 0.0, 1.0, -1.0, 1.0, nan, inf, 1.0])
    hi, lo = oracle.log_kv(v, x)
    exp_k = [inf, inf, float(hi[2]), nan, nan, nan, -inf, inf]
    np.testing.assert_array_equal(hi, np.array(exp_k))
    assert hi[2] == oracle.log_kv(np.array([2.5]), np.array([1.0]))[0][0]


# --------------------------------------------------------------------------
# supplementary: an independent arbitrary-precision library, where present
# --------------------------------------------------------------------------

def test_against_mpmath(oracle):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 45
    rng = np.random.default_rng(21)
    v = np.concatenate([rng.uniform(0, 30, 12), 10 ** rng.uniform(-3, 3, 12)])
    x = np.concatenate([rng.uniform(0.01, 50, 12), 10 ** rng.uniform(-3, 2.5, 12)])
    li = oracle.log_iv(v, x)
    lk = oracle.log_kv(v, x)
    for i in range(v.size):
        vi, xi = mp.mpf(float(v[i])), mp.mpf(float(x[i]))
        ri = mp.log(mp.besseli(vi, xi))
        rk = mp.log(mp.besselk(vi, xi))
        gi = mp.mpf(float(li[0][i])) + mp.mpf(float(li[1][i]))
        gk = mp.mpf(float(lk[0][i])) + mp.mpf(float(lk[1][i]))
        assert abs(gi - ri) <= 1e-26 * max(1, abs(ri)), (v[i], x[i])
        assert abs(gk - rk) <= 1e-26 * max(1, abs(rk)), (v[i], x[i])
