"""Build-time generator of the constant tables the HIP kernels use.

Everything is derived in exact rational arithmetic and rounded once, to
nearest, into binary64 and binary32 hex literals:

* Debye polynomials u_k(t), k = 1..13, from u_0 = 1 and
  u_{k+1}(t) = 1/2 t^2 (1 - t^2) u_k'(t) + 1/8 int_0^t (1 - 5 s^2) u_k(s) ds
  (paper, Sec. "Modified Bessel function of the first kind", eqs. (u0), (uk);
  DLMF 10.41.10).  u_k(t) = t^k P_k(t^2) with P_k of degree k, so the kernels
  evaluate sum_k (t/v)^k P_k(t^2) by Horner in t^2 inside and in t/v outside.
* Node weights of the composite rule on u_j = j/N, N = 600, for the integral of
  log K_v (paper, eq. (log Kv integral) and the composite rule that follows it):
  the trapezoid rule with a Gregory end correction of order 8 at u = 1.  No
  correction is needed at u = 0, where both integrands vanish to high order
  (g ~ u^7, h ~ exp(-1/u)).  The paper's Simpson weights are emitted as well.
* Per-node constants log u_j and 1/u_j.
* Orders 0 and 1 (the scalar-order fast path):
  - the power series of I_0, I_1 (DLMF 10.25.2): 1/(k! (k+v)!), k < 48;
  - the small-argument series of K_0, K_1 (DLMF 10.31.1 with n = 0, 1,
    psi(k+1) = H_k - gamma): H_k/(k!)^2 and (H_k + H_{k+1} - 2 gamma)/(k!(k+1)!);
  - Chebyshev coefficients of g_v(s) = log K_v(1/s) + 1/s + 1/2 log(2/(pi s))
    on s = 1/x in [1/17.5, 1/2], from K_0, K_1 evaluated by the same series
    in 100-digit decimal arithmetic at the Chebyshev points (the series
    cancels there by up to ~1e15, far below that precision).

Run as a script it writes ``csrc/lbessel_tables.h``.
"""
from __future__ import annotations

import functools
import math
import os
from fractions import Fraction

U_TERMS = 13         # Debye terms on the asymptotic branch (U_13)
MU_TERMS = 20        # Hankel correction terms (mu_20)
QUAD_N = 600         # nodes of the composite rule (paper: N = 600)
GREGORY_ORDER = 8    # backward differences used by the end correction


# ----------------------------------------------------------------------------
# Debye polynomials
# ----------------------------------------------------------------------------

def debye_polys(kmax: int = U_TERMS + 1) -> list[dict[int, Fraction]]:
    """u_0..u_kmax as {power of t: coefficient}."""
    polys = [{0: Fraction(1)}]
    for _ in range(kmax):
        u = polys[-1]
        nxt: dict[int, Fraction] = {}
        # 1/2 (t^2 - t^4) u'(t)
        for p, c in u.items():
            if p == 0:
                continue
            d = c * p                                    # coefficient of t^{p-1}
            nxt[p + 1] = nxt.get(p + 1, Fraction(0)) + d / 2
            nxt[p + 3] = nxt.get(p + 3, Fraction(0)) - d / 2
        # 1/8 int_0^t (1 - 5 s^2) u(s) ds
        for p, c in u.items():
            nxt[p + 1] = nxt.get(p + 1, Fraction(0)) + c / (8 * (p + 1))
            nxt[p + 3] = nxt.get(p + 3, Fraction(0)) - 5 * c / (8 * (p + 3))
        polys.append({p: c for p, c in nxt.items() if c != 0})
    return polys


def debye_p_coeffs(k: int, polys=None) -> list[Fraction]:
    """Coefficients c_0..c_k of P_k with u_k(t) = t^k sum_j c_j t^{2j}."""
    polys = polys or debye_polys(k)
    u = polys[k]
    out = []
    for j in range(k + 1):
        out.append(u.get(k + 2 * j, Fraction(0)))
    assert set(u) <= {k + 2 * j for j in range(k + 1)}
    return out


# ----------------------------------------------------------------------------
# quadrature weights
# ----------------------------------------------------------------------------

def gregory_coefficients(m: int) -> list[Fraction]:
    """Coefficients c_0..c_m of z / log(1+z) = sum c_j z^j (c_1 = 1/2, c_2 = -1/12, ...).

    The Gregory end correction for the trapezoid rule at the right end is
    -h sum_{k>=1} |c_{k+1}| nabla^k f_N.
    """
    # log(1+z)/z = sum_j (-1)^j z^j / (j+1); invert the power series.
    a = [Fraction((-1) ** j, j + 1) for j in range(m + 1)]
    c = [Fraction(0)] * (m + 1)
    c[0] = 1 / a[0]
    for j in range(1, m + 1):
        c[j] = -sum(a[i] * c[j - i] for i in range(1, j + 1)) / a[0]
    return c


def trapezoid_gregory_weights(n: int = QUAD_N, order: int = GREGORY_ORDER) -> list[Fraction]:
    """Weights w_0..w_n (in units of h = 1/n) of the trapezoid rule on [0, 1] with
    the right-end Gregory correction using nabla^1..nabla^order at u = 1."""
    w = [Fraction(1)] * (n + 1)
    w[0] = Fraction(1, 2)
    w[n] = Fraction(1, 2)
    c = gregory_coefficients(order + 1)
    for k in range(1, order + 1):
        gk = abs(c[k + 1])
        # nabla^k f_n = sum_m (-1)^m C(k, m) f_{n-m}
        for m in range(k + 1):
            w[n - m] -= gk * (-1) ** m * math.comb(k, m)
    return w


def simpson_weights(n: int = QUAD_N) -> list[Fraction]:
    """Composite Simpson 1/3 weights in units of h = 1/n: (1, 4, 2, 4, ..., 4, 1)/3."""
    assert n % 2 == 0
    w = [Fraction(2, 3) if j % 2 == 0 else Fraction(4, 3) for j in range(n + 1)]
    w[0] = w[n] = Fraction(1, 3)
    return w


# ----------------------------------------------------------------------------
# rounding and emission
# ----------------------------------------------------------------------------

def to_f64(q: Fraction) -> float:
    return q.numerator / q.denominator          # correctly rounded in CPython


def to_f32_exact(q: Fraction) -> float:
    """Round a rational to the nearest binary32 (ties to even), returned as a float."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)                              # subnormal range
    scale = Fraction(2) ** (23 - e)
    m = a * scale                                 # in [2^23, 2^24) for normals
    mi = m.numerator // m.denominator
    rem = m - mi
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and mi % 2 == 1):
        mi += 1
    return sign * float(Fraction(mi) / scale)


def node_constants(n: int = QUAD_N):
    """(u_j, log u_j, 1/u_j) for j = 1..n as exact rationals / 50-digit decimals."""
    from decimal import Decimal, localcontext
    out = []
    with localcontext() as ctx:
        ctx.prec = 50
        for j in range(1, n + 1):
            u = Fraction(j, n)
            lu = (Decimal(j) / Decimal(n)).ln()
            out.append((u, lu, 1 / u))
    return out


def dec_to_f64(d) -> float:
    """Nearest binary64 to a Decimal (via its exact rational value)."""
    return to_f64(Fraction(d))


def dec_to_f32(d) -> float:
    return to_f32_exact(Fraction(d))


def f64_hex(x: float) -> str:
    return float(x).hex()


def f32_hex(x: float) -> str:
    return float(x).hex() + "f"


# ----------------------------------------------------------------------------
# Orders 0 and 1
# ----------------------------------------------------------------------------
I01_TERMS = 48       # I_0, I_1 series terms (x <= 21.5: tail < 2^-60)
K01_TERMS = 18       # K_0, K_1 small-argument series terms (x <= 2)
CHEB01_DEG = 20      # Chebyshev degree of g_v on x in [2, 17.5]
CHEB01_X = (Fraction(2), Fraction(35, 2))
PI_50 = "3.14159265358979323846264338327950288419716939937510582097494459"
EULER_GAMMA_50 = "0.57721566490153286060651209008240243104215933593992359880576723"


def i01_series(v: int) -> list[Fraction]:
    return [Fraction(1, math.factorial(k) * math.factorial(k + v)) for k in range(I01_TERMS)]


# Integer orders 2..14 of the scalar-order path: I_n(x) = (x/2)^n/n! (1 +
# sum_{k>=1} d_{n,k} q^k), d_{n,k} = n!/(k!(k+n)!), q = x^2/4 (DLMF 10.25.2),
# on the series region of each order (x <= 23 in binary64, x <= 7.5 in
# binary32); the term counts keep the neglected tail below 2^-60 (binary64)
# and 2^-30 (binary32) of the sum there.
INT_ORDERS = range(2, 15)
IINT_TERMS64 = 40    # k = 1..40 (37 suffice at n = 2, x = 23)
IINT_TERMS32 = 16    # (13 suffice at n = 2, x = 7.5)
IINT_XMAX64 = Fraction(23)
IINT_XMAX32 = Fraction(15, 2)


def iint_series(n: int, terms: int) -> list[Fraction]:
    f = math.factorial(n)
    return [Fraction(f, math.factorial(k) * math.factorial(k + n)) for k in range(1, terms + 1)]


def iint_tail_ok(n: int, terms: int, xmax: Fraction, bits: int) -> bool:
    """The sum beyond the last kept term, bounded by the next term over
    (1 - ratio) (terms decrease geometrically past k ~ sqrt(q)), below 2^-bits
    of the sum at x = xmax."""
    q = xmax * xmax / 4
    d = iint_series(n, terms + 1)
    nxt = d[terms] * q ** (terms + 1)
    ratio = q / ((terms + 2) * (terms + 2 + n))
    assert ratio < 1
    total = 1 + sum(c * q ** (k + 1) for k, c in enumerate(d[:terms]))
    return nxt / (1 - ratio) < total / Fraction(2) ** bits


def _harmonic(k: int) -> Fraction:
    return sum((Fraction(1, j) for j in range(1, k + 1)), Fraction(0))


def k0_series() -> list[Fraction]:
    """H_k / (k!)^2: K_0(x) = sum_k H_k q^k/(k!)^2 - (log(x/2) + gamma) I_0(x), q = x^2/4."""
    return [_harmonic(k) / math.factorial(k) ** 2 for k in range(K01_TERMS)]


def k1_series():
    """(H_k + H_{k+1})/(k!(k+1)!) and 1/(k!(k+1)!) (the -2 gamma part):
    x K_1(x) = 1 + 2 q log(x/2) S_1(q) - q sum_k (H_k + H_{k+1} - 2 gamma) q^k/(k!(k+1)!)."""
    a = [(_harmonic(k) + _harmonic(k + 1)) / (math.factorial(k) * math.factorial(k + 1))
         for k in range(K01_TERMS)]
    b = [Fraction(1, math.factorial(k) * math.factorial(k + 1)) for k in range(K01_TERMS)]
    return a, b


def _dec_cos(z, prec):
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = prec + 10
        z = Decimal(z)
        two_pi = 2 * Decimal(PI_50)
        z = z - two_pi * (z / two_pi).to_integral_value()     # |z| <= pi
        term, acc, k = Decimal(1), Decimal(1), 0
        while abs(term) > Decimal(10) ** -(prec + 5):
            k += 2
            term = -term * z * z / (k * (k - 1))
            acc += term
        return +acc


def k01_decimal(v: int, x, prec: int = 100):
    """K_v(x), v in {0, 1}, by the DLMF 10.31.1 series in `prec`-digit decimals."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = prec
        x = Decimal(x)
        g = Decimal(EULER_GAMMA_50)
        q = x * x / 4
        l2 = (x / 2).ln()
        s_i = s_k = Decimal(0)
        term = Decimal(1) if v == 0 else Decimal(1)
        h, h1 = Decimal(0), Decimal(1)          # H_k, H_{k+1}
        k = 0
        while True:
            s_i += term
            s_k += (h if v == 0 else h + h1 - 2 * g) * term
            if k > 8 and term < Decimal(10) ** -(prec - 5) * s_i:
                break
            k += 1
            h += Decimal(1) / k
            h1 += Decimal(1) / (k + 1)
            term = term * q / (k * (k + v))
        if v == 0:
            return s_k - (l2 + g) * s_i
        return 1 / x + l2 * (x / 2) * s_i - x / 4 * s_k


def k01_chebyshev(v: int, deg: int = CHEB01_DEG, prec: int = 100):
    """Chebyshev coefficients c_0..c_deg of g_v(s) = log K_v(x) + x + 1/2 log(2x/pi),
    s = 1/x on [1/17.5, 1/2], mapped to u in [-1, 1] (u = -1 at x = 17.5)."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = prec
        pi = Decimal(PI_50)
        sa = Decimal(1) / Decimal(float(CHEB01_X[1]))
        sb = Decimal(1) / Decimal(float(CHEB01_X[0]))
        n = deg + 1
        th = [pi * (Decimal(k) + Decimal("0.5")) / n for k in range(n)]
        us = [_dec_cos(t, prec) for t in th]
        gs = []
        for u in us:
            s_ = (sa + sb) / 2 + (sb - sa) / 2 * u
            x = 1 / s_
            gs.append(k01_decimal(v, x, prec).ln() + x + (2 * x / pi).ln() / 2)
        cs = []
        for j in range(n):
            c = sum(gs[k] * _dec_cos(j * th[k], prec) for k in range(n)) * 2 / n
            cs.append(c / 2 if j == 0 else c)
        return cs


# ----------------------------------------------------------------------------
# log Gamma(1 + v) on 0 <= v <= 15 (prefactor of the I series, binary64)
# ----------------------------------------------------------------------------
LG_INTERVALS = 30    # half-unit intervals [j/2, (j+1)/2] of v
LG_DEG = 15          # polynomial degree on each interval
LG_NODES = 32        # Chebyshev points of the interpolant that is truncated


@functools.lru_cache(maxsize=None)
def bernoulli_numbers(n: int) -> tuple[Fraction, ...]:
    """B_0 .. B_n (B_1 = +1/2) by the Akiyama-Tanigawa recurrence."""
    a = [Fraction(0)] * (n + 1)
    out = []
    for m in range(n + 1):
        a[m] = Fraction(1, m + 1)
        for j in range(m, 0, -1):
            a[j - 1] = j * (a[j - 1] - a[j])
        out.append(a[0])
    return tuple(out)


def dec_lgamma(z, prec: int = 40):
    """log Gamma(z) for z > 0 in `prec`-digit decimals: shift to w = z + m >= 40
    by Gamma(z) = Gamma(w) / (z (z+1) ... (w-1)), then Stirling's series with
    20 terms (DLMF 5.11.1; remainder below the first omitted term, ~1e-51)."""
    from decimal import Decimal, localcontext
    bern = bernoulli_numbers(40)
    with localcontext() as ctx:
        ctx.prec = prec + 15
        z = Decimal(z)
        prod = Decimal(1)
        w = z
        while w < 40:
            prod *= w
            w += 1
        half_log_2pi = (2 * Decimal(PI_50)).ln() / 2
        acc = (w - Decimal("0.5")) * w.ln() - w + half_log_2pi
        wp = w
        for k in range(1, 21):
            b = bern[2 * k]
            acc += Decimal(b.numerator) / Decimal(b.denominator) / (2 * k * (2 * k - 1) * wp)
            wp *= w * w
        res = acc - prod.ln()
    with localcontext() as ctx:
        ctx.prec = prec
        return +res


def lgamma1p_poly(j: int, deg: int = LG_DEG, nodes: int = LG_NODES, prec: int = 32):
    """Monomial coefficients a_0..a_deg in u of the degree-`deg` truncation of the
    Chebyshev interpolant (at `nodes` points) of log Gamma(1 + v) on the
    interval v = (2j + 1 + u)/4, u in [-1, 1]."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = prec + 10
        pi = Decimal(PI_50)
        us = [_dec_cos(pi * (Decimal(k) + Decimal("0.5")) / nodes, prec + 10)
              for k in range(nodes)]
        gs = [dec_lgamma(1 + (2 * j + 1 + u) / 4, prec + 10) for u in us]
        # T_m(u_k) by the three-term recurrence
        tk = [[Decimal(1)] * nodes, list(us)]
        for m in range(2, deg + 1):
            tk.append([2 * us[k] * tk[m - 1][k] - tk[m - 2][k] for k in range(nodes)])
        cs = []
        for m in range(deg + 1):
            c = sum(gs[k] * tk[m][k] for k in range(nodes)) * 2 / nodes
            cs.append(c / 2 if m == 0 else c)
        # monomial form: T_0 = 1, T_1 = u, T_{m+1} = 2 u T_m - T_{m-1}
        tpoly = [[Decimal(1)], [Decimal(0), Decimal(1)]]
        for m in range(2, deg + 1):
            nxt = [Decimal(0)] * (m + 1)
            for i, c in enumerate(tpoly[m - 1]):
                nxt[i + 1] += 2 * c
            for i, c in enumerate(tpoly[m - 2]):
                nxt[i] -= c
            tpoly.append(nxt)
        a = [Decimal(0)] * (deg + 1)
        for m in range(deg + 1):
            for i, c in enumerate(tpoly[m]):
                a[i] += cs[m] * c
        return a


# ----------------------------------------------------------------------------
# Temme's series for K_mu(x), K_{mu+1}(x), |mu| <= 1/2 (the small-argument K
# fallback, x <= 1.25): the even functions of mu it needs, as polynomials in
# t = mu^2 on [0, 1/4]
#   G1(mu) = (1/Gamma(1-mu) - 1/Gamma(1+mu)) / (2 mu),  G1(0) = -gamma,
#   G2(mu) = (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2,       G2(0) = 1,
# (1/Gamma(1 + mu) = G2 - mu G1, 1/Gamma(1 - mu) = G2 + mu G1), and
#   sin(pi mu) / (pi mu) = sum_k (-1)^k pi^{2k} t^k / (2k+1)!  (Taylor, exact
# up to the rounding of pi^2), whose reciprocal is the factor mu pi / sin(mu pi).
# ----------------------------------------------------------------------------
TM_X = Fraction(5, 4)   # x bound of the Temme branch
TM_G_DEG = 8            # degree of G1, G2 in t
TM_SINC_TERMS = 12      # sinc terms (t^0 .. t^11; next term < 1e-18 at t = 1/4)
TM_SINH_TERMS = 10      # sinh(s)/s = sum s^{2k}/(2k+1)!, |s| < 1 (next term < 2e-20)
TM_MAX_TERMS = 40       # cap of the series loop (x <= 1.25 stops by ~13 terms)


def _dec_sin(z, prec):
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = prec + 10
        z = Decimal(z)
        term, acc, k = z, z, 1
        while abs(term) > Decimal(10) ** -(prec + 5):
            k += 2
            term = -term * z * z / (k * (k - 1))
            acc += term
        return +acc


def temme_g(t, prec: int = 60):
    """(G1, G2) at mu = sqrt(t) > 0 in `prec`-digit decimals (log Gamma by
    dec_lgamma; the difference of G1 loses ~log10(1/mu) of the extra digits)."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = prec + 20
        mu = Decimal(t).sqrt()
        rp = (-dec_lgamma(1 + mu, prec + 20)).exp()
        rm = (-dec_lgamma(1 - mu, prec + 20)).exp()
        g1 = (rm - rp) / (2 * mu)
        g2 = (rm + rp) / 2
    with localcontext() as ctx:
        ctx.prec = prec
        return +g1, +g2


@functools.lru_cache(maxsize=None)
def temme_g_poly(which: int, deg: int = TM_G_DEG, prec: int = 60):
    """Monomial coefficients b_0..b_deg in t of the Chebyshev interpolant (at
    deg + 8 points of [0, 1/4]) of G1 (which = 0) or G2 (which = 1)."""
    from decimal import Decimal, localcontext
    nodes = deg + 8
    tmax = Decimal(1) / 4
    with localcontext() as ctx:
        ctx.prec = prec + 20
        pi = Decimal(PI_50)
        us = [_dec_cos(pi * (Decimal(k) + Decimal("0.5")) / nodes, prec + 20)
              for k in range(nodes)]
        fs = [temme_g(tmax / 2 * (1 + u), prec)[which] for u in us]
        tk = [[Decimal(1)] * nodes, list(us)]
        for m in range(2, deg + 1):
            tk.append([2 * us[k] * tk[m - 1][k] - tk[m - 2][k] for k in range(nodes)])
        cs = []
        for m in range(deg + 1):
            c = sum(fs[k] * tk[m][k] for k in range(nodes)) * 2 / nodes
            cs.append(c / 2 if m == 0 else c)
        tpoly = [[Decimal(1)], [Decimal(0), Decimal(1)]]
        for m in range(2, deg + 1):
            nxt = [Decimal(0)] * (m + 1)
            for i, c in enumerate(tpoly[m - 1]):
                nxt[i + 1] += 2 * c
            for i, c in enumerate(tpoly[m - 2]):
                nxt[i] -= c
            tpoly.append(nxt)
        a = [Decimal(0)] * (deg + 1)
        for m in range(deg + 1):
            for i, c in enumerate(tpoly[m]):
                a[i] += cs[m] * c
        # u = 8 t - 1
        b = [Decimal(0)] * (deg + 1)
        for i, ai in enumerate(a):
            for j in range(i + 1):
                b[j] += ai * math.comb(i, j) * Decimal(8) ** j * (-1) ** (i - j)
    return tuple(b)


def temme_sinc_series(terms: int = TM_SINC_TERMS, prec: int = 60):
    """(-1)^k pi^{2k} / (2k+1)!, k = 0..terms-1 (decimals)."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = prec
        pi2 = Decimal(PI_50) ** 2
        return [(-1) ** k * pi2 ** k / math.factorial(2 * k + 1) for k in range(terms)]


def _debye_arrays():
    polys = debye_polys(U_TERMS)
    rows = [debye_p_coeffs(k, polys) for k in range(1, U_TERMS + 1)]
    return rows


def render_header() -> str:
    rows = _debye_arrays()
    lines = [
        "// Generated by paper_2409_08729_amd/gen_tables.py: do not edit.",
        "// Exact rationals rounded once to nearest.",
        "#pragma once",
        "",
        "namespace lbessel {",
        "namespace tables {",
        "",
        f"constexpr int kUTerms = {U_TERMS};",
        f"constexpr int kMuTerms = {MU_TERMS};",
        f"constexpr int kQuadN = {QUAD_N};",
        f"constexpr int kGregoryOrder = {GREGORY_ORDER};",
        "",
        "// P_k(p), u_k(t) = t^k P_k(t^2); row k-1 holds c_0..c_k (unused tail = 0).",
    ]
    for name, conv, fmt, ty in (("kDebyeP64", to_f64, f64_hex, "double"),
                                ("kDebyeP32", to_f32_exact, f32_hex, "float")):
        lines.append(f"__constant__ const {ty} {name}[{U_TERMS}][{U_TERMS + 1}] = {{")
        for k, row in enumerate(rows, start=1):
            vals = [fmt(conv(c)) for c in row] + ["0"] * (U_TERMS - k)
            lines.append("    {" + ", ".join(vals) + "},")
        lines.append("};")
    # Hankel expansion: c_k = c_{k-1} (mu - (2k-1)^2) / k * s/(8x), k = 1..20:
    # rows {1/k, (2k-1)^2}.
    lines.append("")
    lines.append("// Hankel recurrence constants, row k-1 = {1/k, (2k-1)^2}, k = 1..20.")
    for name, conv, fmt, ty in (("kHankel64", to_f64, f64_hex, "double"),
                                ("kHankel32", to_f32_exact, f32_hex, "float")):
        lines.append(f"__constant__ const {ty} {name}[{MU_TERMS}][2] = {{")
        for k in range(1, MU_TERMS + 1):
            lines.append("    {" + fmt(conv(Fraction(1, k))) + ", "
                         + fmt(conv(Fraction((2 * k - 1) ** 2))) + "},")
        lines.append("};")
    # quadrature: right-end weights that differ from 1 (trapezoid + Gregory)
    w = trapezoid_gregory_weights()
    tail = [w[j] for j in range(QUAD_N - GREGORY_ORDER, QUAD_N + 1)]
    lines.append("")
    lines.append("// Weights of nodes N-order..N (h = 1/N units); all interior weights are 1.")
    for name, conv, fmt, ty in (("kGregoryTail64", to_f64, f64_hex, "double"),
                                ("kGregoryTail32", to_f32_exact, f32_hex, "float")):
        lines.append(f"__constant__ const {ty} {name}[{GREGORY_ORDER + 1}] = {{"
                     + ", ".join(fmt(conv(t)) for t in tail) + "};")
    # per-node constants, j = 1..N (index j-1)
    nodes = node_constants()
    lines.append("")
    lines.append("// Node constants for u_j = j/N, j = 1..N (row j-1): {u_j, log u_j, 1/u_j}.")
    for name, conv_q, conv_d, fmt, ty in (
            ("kQuadNode64", to_f64, dec_to_f64, f64_hex, "double"),
            ("kQuadNode32", to_f32_exact, dec_to_f32, f32_hex, "float")):
        lines.append(f"__constant__ const {ty} {name}[{QUAD_N}][3] = {{")
        for u, lu, iu in nodes:
            lines.append("    {" + ", ".join((fmt(conv_q(u)), fmt(conv_d(lu)), fmt(conv_q(iu))))
                         + "},")
        lines.append("};")
    # orders 0 and 1
    lines.append("")
    lines.append(f"constexpr int kI01Terms = {I01_TERMS};")
    lines.append(f"constexpr int kK01Terms = {K01_TERMS};")
    lines.append(f"constexpr int kCheb01Deg = {CHEB01_DEG};")
    lines.append("// I_v series coefficients 1/(k!(k+v)!), v = 0, 1.")
    for name, conv, fmt, ty in (("kI01Ser64", to_f64, f64_hex, "double"),
                                ("kI01Ser32", to_f32_exact, f32_hex, "float")):
        lines.append(f"__constant__ const {ty} {name}[2][{I01_TERMS}] = {{")
        for v in (0, 1):
            lines.append("    {" + ", ".join(fmt(conv(c)) for c in i01_series(v)) + "},")
        lines.append("};")
    k1a, k1b = k1_series()
    lines.append("// K_0: H_k/(k!)^2; K_1: (H_k + H_{k+1})/(k!(k+1)!).")
    for name, conv, fmt, ty in (("kK0Ser64", to_f64, f64_hex, "double"),
                                ("kK0Ser32", to_f32_exact, f32_hex, "float")):
        lines.append(f"__constant__ const {ty} {name}[{K01_TERMS}] = {{"
                     + ", ".join(fmt(conv(c)) for c in k0_series()) + "};")
    for name, conv, fmt, ty in (("kK1Ser64", to_f64, f64_hex, "double"),
                                ("kK1Ser32", to_f32_exact, f32_hex, "float")):
        lines.append(f"__constant__ const {ty} {name}[{K01_TERMS}] = {{"
                     + ", ".join(fmt(conv(c)) for c in k1a) + "};")
    # integer orders 2..14: I_n series coefficients and log n!
    for n in INT_ORDERS:
        assert iint_tail_ok(n, IINT_TERMS64, IINT_XMAX64, 60), n
        assert iint_tail_ok(n, IINT_TERMS32, IINT_XMAX32, 30), n
    lines.append(f"constexpr int kIntOrderMin = {INT_ORDERS[0]};")
    lines.append(f"constexpr int kIntOrderMax = {INT_ORDERS[-1]};")
    lines.append(f"constexpr int kIIntTerms64 = {IINT_TERMS64};")
    lines.append(f"constexpr int kIIntTerms32 = {IINT_TERMS32};")
    lines.append("// I_n(x) = (x/2)^n / n! (1 + sum_k d[n-2][k-1] q^k), d = n!/(k!(k+n)!), k >= 1.")
    for name, conv, fmt, ty, terms in (("kIIntSer64", to_f64, f64_hex, "double", IINT_TERMS64),
                                       ("kIIntSer32", to_f32_exact, f32_hex, "float",
                                        IINT_TERMS32)):
        lines.append(f"__constant__ const {ty} {name}[{len(INT_ORDERS)}][{terms}] = {{")
        for n in INT_ORDERS:
            lines.append("    {" + ", ".join(fmt(conv(c)) for c in iint_series(n, terms)) + "},")
        lines.append("};")
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 50
        logfact = [Decimal(math.factorial(n)).ln() for n in range(INT_ORDERS[-1] + 1)]
    lines.append("// log n!, n = 0..14.")
    lines.append(f"__constant__ const double kLogFact64[{len(logfact)}] = {{"
                 + ", ".join(f64_hex(dec_to_f64(d)) for d in logfact) + "};")
    lines.append(f"__constant__ const float kLogFact32[{len(logfact)}] = {{"
                 + ", ".join(f32_hex(dec_to_f32(d)) for d in logfact) + "};")
    lines.append("// Chebyshev coefficients of log K_v(x) + x + 1/2 log(2x/pi) in s = 1/x,")
    lines.append("// s in [1/17.5, 1/2] mapped to u in [-1, 1]; rows v = 0, 1.")
    cheb = [k01_chebyshev(0), k01_chebyshev(1)]
    for name, conv, fmt, ty in (("kK01Cheb64", dec_to_f64, f64_hex, "double"),
                                ("kK01Cheb32", dec_to_f32, f32_hex, "float")):
        lines.append(f"__constant__ const {ty} {name}[2][{CHEB01_DEG + 1}] = {{")
        for row in cheb:
            lines.append("    {" + ", ".join(fmt(conv(c)) for c in row) + "},")
        lines.append("};")
    from decimal import Decimal, localcontext
    # e^{+-n} and e^{+-f/64}: e^{t} and e^{-t} for t a multiple of 1/64 in
    # [0, 64) as one product each
    with localcontext() as ctx:
        ctx.prec = 50
        eint = [Decimal(n).exp() for n in range(64)]
        efrac = [(Decimal(f) / 64).exp() for f in range(64)]
        enint = [(-Decimal(n)).exp() for n in range(64)]
        enfrac = [(-Decimal(f) / 64).exp() for f in range(64)]
    lines.append("// e^n, n = 0..63, and e^{f/64}, f = 0..63 (K fallback grid nodes),")
    lines.append("// and their reciprocals e^-n, e^{-f/64}.")
    for name, vals in (("kExpInt64", eint), ("kExpFrac64", efrac),
                       ("kExpNegInt64", enint), ("kExpNegFrac64", enfrac)):
        lines.append(f"__constant__ const double {name}[64] = {{"
                     + ", ".join(f64_hex(dec_to_f64(d)) for d in vals) + "};")
    lines.append(f"// log Gamma(1 + v), 0 <= v <= {LG_INTERVALS // 2}: on v in [j/2, (j+1)/2] the "
                 f"polynomial sum_i a[j][i] u^i,")
    lines.append("// u = 4 v - 2 j - 1 in [-1, 1] (truncated Chebyshev interpolant, monomial form).")
    lines.append(f"constexpr int kLgIntervals = {LG_INTERVALS};")
    lines.append(f"constexpr int kLgCoefs = {LG_DEG + 1};")
    lines.append(f"__constant__ const double kLgamma1p64[{LG_INTERVALS}][{LG_DEG + 1}] = {{")
    for j in range(LG_INTERVALS):
        lines.append("    {" + ", ".join(f64_hex(dec_to_f64(c)) for c in lgamma1p_poly(j)) + "},")
    lines.append("};")
    lines.append("// Temme's series (K fallback, x <= kTemmeX): G1, G2 as polynomials in t = mu^2")
    lines.append("// (index = power), sin(pi mu)/(pi mu) in t, sinh(s)/s in s^2, 1/k; binary64")
    lines.append("// and binary32 copies.")
    lines.append(f"constexpr double kTemmeX = {f64_hex(to_f64(TM_X))};")
    lines.append(f"constexpr int kTmGCoefs = {TM_G_DEG + 1};")
    lines.append(f"constexpr int kTmSincTerms = {TM_SINC_TERMS};")
    lines.append(f"constexpr int kTmSinhTerms = {TM_SINH_TERMS};")
    lines.append(f"constexpr int kTmMaxTerms = {TM_MAX_TERMS};")
    lines.append(f"__constant__ const double kTmG64[2][{TM_G_DEG + 1}] = {{")
    for which in (0, 1):
        lines.append("    {" + ", ".join(f64_hex(dec_to_f64(c)) for c in temme_g_poly(which))
                     + "},")
    lines.append("};")
    lines.append(f"__constant__ const double kTmSinc64[{TM_SINC_TERMS}] = {{"
                 + ", ".join(f64_hex(dec_to_f64(c)) for c in temme_sinc_series()) + "};")
    lines.append(f"__constant__ const double kTmInvK64[{TM_MAX_TERMS + 1}] = {{0, "
                 + ", ".join(f64_hex(to_f64(Fraction(1, k))) for k in range(1, TM_MAX_TERMS + 1))
                 + "};")
    lines.append(f"__constant__ const double kTmSinh64[{TM_SINH_TERMS}] = {{"
                 + ", ".join(f64_hex(to_f64(Fraction(1, math.factorial(2 * k + 1))))
                             for k in range(TM_SINH_TERMS)) + "};")
    lines.append(f"__constant__ const float kTmG32[2][{TM_G_DEG + 1}] = {{")
    for which in (0, 1):
        lines.append("    {" + ", ".join(f32_hex(dec_to_f32(c)) for c in temme_g_poly(which))
                     + "},")
    lines.append("};")
    lines.append(f"__constant__ const float kTmSinc32[{TM_SINC_TERMS}] = {{"
                 + ", ".join(f32_hex(dec_to_f32(c)) for c in temme_sinc_series()) + "};")
    lines.append(f"__constant__ const float kTmInvK32[{TM_MAX_TERMS + 1}] = {{0, "
                 + ", ".join(f32_hex(to_f32_exact(Fraction(1, k)))
                             for k in range(1, TM_MAX_TERMS + 1)) + "};")
    lines.append(f"__constant__ const float kTmSinh32[{TM_SINH_TERMS}] = {{"
                 + ", ".join(f32_hex(to_f32_exact(Fraction(1, math.factorial(2 * k + 1))))
                             for k in range(TM_SINH_TERMS)) + "};")
    lines.append(f"constexpr double kEulerGamma64 = {f64_hex(dec_to_f64(Decimal(EULER_GAMMA_50)))};")
    lines.append(f"constexpr float kEulerGamma32 = {f32_hex(dec_to_f32(Decimal(EULER_GAMMA_50)))};")
    lines.append("")
    lines.append("}  // namespace tables")
    lines.append("}  // namespace lbessel")
    lines.append("")
    return "\n".join(lines)


def write_header(path: str | None = None) -> str:
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc",
                                "lbessel_tables.h")
    text = render_header()
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as f:
            f.write(text)
    return path


if __name__ == "__main__":
    print(write_header())
