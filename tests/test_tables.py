"""Host checks of the generated constant tables (no GPU).

* Debye polynomials: the printed u_1, u_2, u_3 (DLMF 10.41.10, A&S 9.3.9) and
  u_k(1) = (-1)^k gamma_k for k <= 14, gamma_k the Stirling-series
  coefficients of Gamma*(v) = Gamma(v+1) / (sqrt(2 pi v) (v/e)^v), derived here
  independently from Bernoulli numbers (DLMF 5.11.1 / 5.11.10).
* Quadrature weights: sum to N, integrate smooth functions that vanish at 0
  to ~1e-17, and reproduce the v = 1/2 integral (exactly 1) in binary64.
"""
from fractions import Fraction
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2409_08729_amd"))
import gen_tables as gt  # noqa: E402
sys.path.pop(0)

import closed_forms as cf  # noqa: E402


def test_debye_low_orders_match_printed():
    polys = gt.debye_polys(3)
    assert polys[1] == {1: Fraction(3, 24), 3: Fraction(-5, 24)}
    assert polys[2] == {2: Fraction(81, 1152), 4: Fraction(-462, 1152), 6: Fraction(385, 1152)}
    assert polys[3] == {3: Fraction(30375, 414720), 5: Fraction(-369603, 414720),
                        7: Fraction(765765, 414720), 9: Fraction(-425425, 414720)}


def _stirling_gamma_coeffs(m):
    """gamma_1..gamma_m of Gamma*(v) ~ sum gamma_k v^-k, from
    log Gamma*(v) ~ sum_{j>=1} B_{2j} / (2j (2j-1) v^{2j-1})."""
    # log series coefficients l_k of v^-k
    lser = [Fraction(0)] * (m + 1)
    for j in range(1, m // 2 + 2):
        k = 2 * j - 1
        if k <= m:
            lser[k] = cf.bernoulli(2 * j) / (2 * j * (2 * j - 1))
    # exp of a power series with zero constant term: e' = l' e
    e = [Fraction(0)] * (m + 1)
    e[0] = Fraction(1)
    for n in range(1, m + 1):
        e[n] = sum(k * lser[k] * e[n - k] for k in range(1, n + 1)) / n
    return e


def test_debye_at_t_equal_one_is_stirling():
    m = 14
    gam = _stirling_gamma_coeffs(m)
    assert gam[1] == Fraction(1, 12) and gam[2] == Fraction(1, 288)
    polys = gt.debye_polys(m)
    for k in range(1, m + 1):
        uk1 = sum(polys[k].values())
        assert uk1 == (-1) ** k * gam[k], k


def test_debye_parity_and_degree():
    for k in range(1, 14):
        c = gt.debye_p_coeffs(k)
        assert len(c) == k + 1 and c[-1] != 0 and c[0] != 0


def test_gregory_weights():
    w = gt.trapezoid_gregory_weights()
    n = gt.QUAD_N
    assert sum(w) == n
    assert all(wj == 1 for wj in w[1:n - gt.GREGORY_ORDER])
    # functions flat at u = 0 (all derivatives < 9 vanish): integrate to ~h^10
    for d in (9, 12, 16, 25):
        approx = sum(w[j] * Fraction(j, n) ** d for j in range(n + 1)) / n
        assert abs(approx - Fraction(1, d + 1)) < Fraction(1, 10 ** 17), d
    # plain trapezoid would be off by ~d/(12 N^2)
    d = 12
    trap = (sum(Fraction(j, n) ** d for j in range(n + 1)) - Fraction(1, 2)) / n
    assert abs(trap - Fraction(1, d + 1)) > Fraction(1, 10 ** 7)


def test_half_order_integral_is_one_in_binary64():
    """v = 1/2: int_0^1 (g + h) du = (1 - 1/e) + 1/e = 1 (the Simpson constant of the
    paper printed as 1/(6N) would give 1/2 here)."""
    nodes = gt.node_constants()
    u = np.array([float(a) for a, _, _ in nodes])
    w = np.array([float(x) for x in gt.trapezoid_gregory_weights()[1:]])
    beta = 8.0
    x = 3.0
    g = beta * np.exp(-u ** beta) * (2 * x + u ** beta) ** 0.0 * u ** 7
    h = np.exp(-1 / u) * u ** -2.0 * (2 * x * u + 1) ** 0.0
    val = (w * (g + h)).sum() / gt.QUAD_N
    assert abs(val - 1.0) < 4e-16
    ws = np.array([float(x) for x in gt.simpson_weights()[1:]])
    assert abs((ws * (g + h)).sum() / gt.QUAD_N - 1.0) < 1e-9


def test_rounding_helpers():
    assert gt.to_f32_exact(Fraction(1, 3)) == float(np.float32(1 / 3))
    assert gt.to_f32_exact(Fraction(-5, 24)) == float(np.float32(-5 / 24))
    lu = gt.node_constants(600)[0][1]
    assert gt.dec_to_f64(lu) == math.log(1 / 600) or abs(gt.dec_to_f64(lu) - math.log(1 / 600)) <= 1e-15


# ----------------------------------------------------------------------------
# Orders 0 and 1 (scalar-order fast path tables)
# ----------------------------------------------------------------------------

def test_constant_literals():
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 60
        assert abs(Decimal(gt.PI_50) - cf.pi_dec(60)) < Decimal("1e-58")
        assert abs(Decimal(gt.EULER_GAMMA_50) - cf.euler_gamma(60)) < Decimal("1e-58")


def test_k01_decimal_series_matches_oracle(oracle):
    from decimal import Decimal
    xs = [1e-5, 0.3, 1.0, 2.0, 5.5, 11.0, 17.5]
    for v in (0, 1):
        hi, lo = oracle.log_kv(np.full(len(xs), float(v)), np.array(xs))
        for x, h, l in zip(xs, hi, lo):
            got = gt.k01_decimal(v, x, 80).ln()
            assert abs(got - (Decimal(h) + Decimal(l))) < Decimal("1e-28") * Decimal(max(1.0, abs(h))), (v, x)


def test_k01_chebyshev_reconstructs_g():
    # the emitted binary64 coefficients reproduce g_v(1/x) to ~1e-17 on [2, 17.5]
    from decimal import Decimal
    import math as m
    g = np.random.default_rng(4)
    sa, sb = 1 / 17.5, 0.5
    for v in (0, 1):
        c = [float(Fraction(d)) for d in gt.k01_chebyshev(v)]
        for x in g.uniform(2.0, 17.5, 12):
            u = (2 / x - (sa + sb)) / (sb - sa)
            t = [1.0, u]
            while len(t) < len(c):
                t.append(2 * u * t[-1] - t[-2])
            approx = sum(ci * ti for ci, ti in zip(c, t))
            ref = float(gt.k01_decimal(v, x, 60).ln() + Decimal(x)
                        + (2 * Decimal(x) / Decimal(gt.PI_50)).ln() / 2)
            assert abs(approx - ref) < 5e-17, (v, x, approx - ref)


def test_order01_series_tables():
    s0 = gt.i01_series(0)
    s1 = gt.i01_series(1)
    assert s0[3] == Fraction(1, 36) and s1[3] == Fraction(1, 144)
    c = gt.k0_series()
    assert c[0] == 0 and c[2] == Fraction(3, 2) / 4
    a, b = gt.k1_series()
    assert a[0] == 1 and b[1] == Fraction(1, 2) and a[1] == Fraction(1 + Fraction(3, 2), 2)
    # I_0 tail beyond the table at x = 21.5 is negligible
    q = Fraction(43, 4) ** 2
    head = sum(cc * q ** k for k, cc in enumerate(s0))
    nxt = q ** len(s0) / math.factorial(len(s0)) ** 2
    assert nxt / head < Fraction(1, 2 ** 60)


def _header_array(text: str, name: str) -> list[float]:
    import re
    m = re.search(name + r"\[64\] = \{([^}]*)\};", text)
    assert m, name
    return [float.fromhex(t.strip()) for t in m.group(1).split(",")]


def test_exp_grid_tables():
    """e^{+-n} and e^{+-f/64} for the K fallback nodes: each entry within one
    ulp of the C library's exp, e^1 the nearest double to e, and every
    product e^a e^-a within two ulps of 1."""
    text = gt.render_header()
    ei, ef = _header_array(text, "kExpInt64"), _header_array(text, "kExpFrac64")
    ni, nf = _header_array(text, "kExpNegInt64"), _header_array(text, "kExpNegFrac64")
    assert ei[0] == ef[0] == ni[0] == nf[0] == 1.0
    assert ei[1] == math.e
    for k in range(64):
        for tab, arg in ((ei, k), (ef, k / 64), (ni, -k), (nf, -k / 64)):
            ref = math.exp(arg)
            assert abs(tab[k] - ref) <= math.ulp(ref), (k, arg)
        assert abs(ei[k] * ni[k] - 1.0) <= 2 * 2 ** -52
        assert abs(ef[k] * nf[k] - 1.0) <= 2 * 2 ** -52


def test_bernoulli_numbers():
    b = gt.bernoulli_numbers(20)
    assert b[0] == 1 and b[1] == Fraction(1, 2) and b[2] == Fraction(1, 6)
    assert b[4] == Fraction(-1, 30) and b[12] == Fraction(-691, 2730)
    assert b[20] == Fraction(-174611, 330) and all(b[k] == 0 for k in range(3, 21, 2))


def test_decimal_lgamma_closed_forms():
    """log Gamma at integers (log (n-1)!) and at 1/2 (log sqrt(pi))."""
    from decimal import Decimal, getcontext
    getcontext().prec = 40
    for n in (1, 2, 3, 7, 16, 41, 60):
        ref = Decimal(math.factorial(n - 1)).ln()
        assert abs(gt.dec_lgamma(Decimal(n)) - ref) < Decimal(10) ** -35, n
    half = Decimal(gt.PI_50).sqrt().ln()
    assert abs(gt.dec_lgamma(Decimal("0.5")) - half) < Decimal(10) ** -35


def test_lgamma1p_table():
    """The binary64 polynomials of log Gamma(1 + v), evaluated by Horner as the
    kernel does, against the C library's lgamma on a grid over [0, 15], and
    zero at v = 0 and v = 1 (Gamma(1) = Gamma(2) = 1)."""
    text = gt.render_header()
    import re
    m = re.search(r"kLgamma1p64\[(\d+)\]\[(\d+)\] = \{(.*?)\n\};", text, re.S)
    nint, ncoef = int(m.group(1)), int(m.group(2))
    rows = [[float.fromhex(t.strip()) for t in row.split(",") if t.strip()]
            for row in re.findall(r"\{([^{}]*)\}", m.group(3))]
    assert len(rows) == nint == 30 and all(len(r) == ncoef for r in rows)

    def lg(v):
        j = min(int(2.0 * v), nint - 1)
        u = 4.0 * v - (2 * j + 1)
        s = rows[j][-1]
        for c in reversed(rows[j][:-1]):
            s = s * u + c
        return s

    assert abs(lg(0.0)) < 5e-17 and abs(lg(1.0)) < 1e-16
    from decimal import Decimal, getcontext
    getcontext().prec = 40
    worst, worst_libm = 0.0, 0.0
    for v in np.linspace(0.0, 15.0, 1201):
        exact = gt.dec_lgamma(1 + Decimal(float(v)))
        scale = max(1.0, abs(float(exact)))
        worst = max(worst, float(abs(Decimal(lg(v)) - exact)) / scale)
        worst_libm = max(worst_libm, abs(lg(v) - math.lgamma(1.0 + v)) / scale)
    # the decimal log Gamma is pinned above; the C library's lgamma is only
    # good to ~1e-15 near its minimum, hence the looser second bound
    assert worst < 4e-16, worst
    assert worst_libm < 2e-15, worst_libm
    # the binary32 copy, evaluated in binary32 as the binary32 path does
    f32 = np.float32
    rows32 = [[f32(c) for c in r] for r in rows]
    worst32 = 0.0
    for v in np.linspace(0.0, 15.0, 1201, dtype=np.float32):
        j = min(int(f32(2.0) * v), nint - 1)
        u = f32(f32(4.0) * v - f32(2 * j + 1))
        acc = rows32[j][-1]
        for c in reversed(rows32[j][:-1]):
            acc = f32(acc * u + c)
        ref = math.lgamma(1.0 + float(v))
        worst32 = max(worst32, abs(float(acc) - ref) / max(1.0, abs(ref)))
    assert worst32 < 1e-6, worst32


def _header_row_array(text: str, name: str) -> list[list[float]]:
    import re
    m = re.search(name + r"\[(\d+)\]\[(\d+)\] = \{(.*?)\n\};", text, re.S)
    assert m, name
    return [[float.fromhex(t.strip()) for t in row.split(",") if t.strip()]
            for row in re.findall(r"\{([^{}]*)\}", m.group(3))]


def _header_flat(text: str, name: str) -> list[float]:
    import re
    m = re.search(name + r"\[\d+\] = \{([^}]*)\};", text)
    assert m, name
    return [float.fromhex(t.strip()) if t.strip() != "0" else 0.0 for t in m.group(1).split(",")]


def _horner(c, t):
    s = c[-1]
    for a in reversed(c[:-1]):
        s = s * t + a
    return s


def test_temme_gamma_polynomials():
    """G1, G2 of Temme's series as binary64 polynomials in t = mu^2: at mu = 0
    G1 = -gamma (Euler's constant) and G2 = 1; across |mu| <= 1/2 the
    reciprocals of G2 -+ mu G1 are Gamma(1 +- mu) to the C library's
    accuracy, and G1 agrees with the difference quotient of 1/Gamma computed
    in 60-digit decimals away from mu = 0."""
    text = gt.render_header()
    g1, g2 = _header_row_array(text, "kTmG64")
    assert len(g1) == len(g2) == gt.TM_G_DEG + 1
    assert abs(g1[0] + 0.5772156649015329) <= 1.2e-16 and abs(g2[0] - 1.0) <= 2.3e-16
    worst = 0.0
    for mu in np.linspace(-0.5, 0.5, 401):
        t = mu * mu
        a, b = _horner(g1, t), _horner(g2, t)
        for sgn in (1.0, -1.0):
            ref = math.gamma(1.0 + sgn * mu)
            got = 1.0 / (b - sgn * mu * a)
            worst = max(worst, abs(got - ref) / ref)
    assert worst < 6e-16, worst
    from decimal import Decimal
    for mu in (0.013, 0.1, 0.37, 0.5):
        e1, e2 = gt.temme_g(Decimal(mu) ** 2)
        t = mu * mu
        assert abs(_horner(g1, t) - float(e1)) <= 2e-16 * abs(float(e1)), mu
        assert abs(_horner(g2, t) - float(e2)) <= 2e-16 * abs(float(e2)), mu


def test_temme_sinc_and_sinh_series():
    """sin(pi mu)/(pi mu) as a polynomial in mu^2 against the C library's sin
    on |mu| <= 1/2 (1 at 0, 2/pi at 1/2); sinh(s)/s against sinh on |s| < 1;
    the 1/k table exact."""
    text = gt.render_header()
    sc = _header_flat(text, "kTmSinc64")
    sh = _header_flat(text, "kTmSinh64")
    ik = _header_flat(text, "kTmInvK64")
    assert len(sc) == gt.TM_SINC_TERMS and len(sh) == gt.TM_SINH_TERMS
    assert sc[0] == 1.0 and abs(_horner(sc, 0.25) - 2 / math.pi) < 2.3e-16
    for mu in np.linspace(1e-3, 0.5, 300):
        ref = math.sin(math.pi * mu) / (math.pi * mu)
        assert abs(_horner(sc, mu * mu) - ref) < 3e-16, mu
    for s_ in np.linspace(1e-3, 1.0, 300):
        ref = math.sinh(s_) / s_
        assert abs(_horner(sh, s_ * s_) - ref) < 6e-16 * ref, s_   # ref: sinh and a division
    assert ik[0] == 0.0 and all(ik[k] == 1.0 / k for k in range(1, len(ik)))
    assert len(ik) == gt.TM_MAX_TERMS + 1
