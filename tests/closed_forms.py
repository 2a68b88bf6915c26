"""Independent high-precision values of I_v and K_v from closed forms.

Pure ``decimal``/``fractions`` arithmetic: no mpmath, no scipy, no oracle.
These are the pins that fix the binary128 oracle from outside:

* ``log_kv_half``   K_{n+1/2}(x) = sqrt(pi/2x) e^{-x} sum_{k<=n} (n+k)!/(k!(n-k)!(2x)^k)
                    (DLMF 10.49.12 with 10.47.9: a finite, positive, exact sum).
* ``log_iv_half``   I_{n+1/2}(x) from the finite form of the modified spherical
                    Bessel function i_n^(1) (DLMF 10.49.8 with 10.47.7).
* ``log_iv_series`` the defining series I_v = sum (x/2)^{2k+v}/(k! Gamma(k+v+1))
                    summed directly in linear space for integer and half-integer v,
                    where Gamma is exact (brute force, no logarithms, no peak).
* ``log_kn_int``    integer-order K_n from its small-x expansion with harmonic
                    numbers and Euler's constant (DLMF 10.31.1).
* ``euler_gamma``   Euler's constant from the Euler-Maclaurin expansion of H_N
                    with Bernoulli numbers (exact rationals).
"""
from __future__ import annotations

from decimal import Decimal, localcontext
from fractions import Fraction
from functools import lru_cache
from math import comb, factorial


def _to_dec(q) -> Decimal:
    if isinstance(q, Fraction):
        return Decimal(q.numerator) / Decimal(q.denominator)
    return Decimal(q)


@lru_cache(maxsize=None)
def pi_dec(prec: int) -> Decimal:
    """pi by Machin's formula pi = 16 atan(1/5) - 4 atan(1/239)."""
    with localcontext() as ctx:
        ctx.prec = prec + 10

        def atan_inv(n: int) -> Decimal:
            x = Decimal(1) / n
            x2 = x * x
            term, s, k = x, Decimal(0), 0
            eps = Decimal(10) ** (-(prec + 8))
            while abs(term) > eps:
                s += term / (2 * k + 1) if k % 2 == 0 else -term / (2 * k + 1)
                term *= x2
                k += 1
            return s

        r = 16 * atan_inv(5) - 4 * atan_inv(239)
    with localcontext() as ctx:
        ctx.prec = prec
        return +r


@lru_cache(maxsize=None)
def bernoulli(m: int) -> Fraction:
    """B_m (B_1 = -1/2) from sum_{j=0}^{m} C(m+1, j) B_j = 0."""
    b = [Fraction(1)]
    for n in range(1, m + 1):
        b.append(-sum(comb(n + 1, j) * b[j] for j in range(n)) / (n + 1))
    return b[m]


@lru_cache(maxsize=None)
def euler_gamma(prec: int) -> Decimal:
    """gamma = H_N - ln N - 1/(2N) + sum_{k=1}^{m} B_{2k} / (2k N^{2k})."""
    N, m = 200, 40
    with localcontext() as ctx:
        ctx.prec = prec + 10
        h = _to_dec(sum(Fraction(1, j) for j in range(1, N + 1)))
        g = h - Decimal(N).ln() - Decimal(1) / (2 * N)
        for k in range(1, m + 1):
            g += _to_dec(bernoulli(2 * k) / (2 * k * Fraction(N) ** (2 * k)))
    with localcontext() as ctx:
        ctx.prec = prec
        return +g


def _dec(x) -> Decimal:
    """Exact decimal value of a binary float (or pass through)."""
    return x if isinstance(x, Decimal) else Decimal(float(x))


def log_kv_half(n: int, x, prec: int = 60) -> Decimal:
    """log K_{n+1/2}(x), x > 0 (DLMF 10.49.12)."""
    with localcontext() as ctx:
        ctx.prec = prec + 20
        xd = _dec(x)
        s = Decimal(0)
        t = Decimal(1)           # (n+k)! / (k! (n-k)! (2x)^k), exact ratio update
        for k in range(n + 1):
            s += t
            t = t * (n + k + 1) * (n - k) / ((k + 1) * 2 * xd)
        r = (pi_dec(prec + 20) / (2 * xd)).ln() / 2 - xd + s.ln()
    with localcontext() as ctx:
        ctx.prec = prec
        return +r


def log_iv_half(n: int, x, prec: int = 200) -> Decimal:
    """log I_{n+1/2}(x), x > 0, from the finite form of i_n^(1) (DLMF 10.49.8).

    i_n^(1)(z) = 1/2 e^z sum (-1)^k a_k / z^{k+1} + (-1)^{n+1} 1/2 e^{-z} sum a_k / z^{k+1},
    a_k = (n+k)! / (2^k k! (n-k)!), and I_{n+1/2}(z) = sqrt(2z/pi) i_n^(1)(z).
    The two sums cancel for small z; ``prec`` must cover the digits lost.
    """
    with localcontext() as ctx:
        ctx.prec = prec + 20
        z = _dec(x)
        s_plus = Decimal(0)
        s_minus = Decimal(0)
        for k in range(n + 1):
            a = Decimal(factorial(n + k)) / (2 ** k * factorial(k) * factorial(n - k))
            t = a / z ** (k + 1)
            s_plus += t if k % 2 == 0 else -t
            s_minus += t
        sign = -1 if n % 2 == 0 else 1          # (-1)^{n+1}
        i1 = (z.exp() * s_plus + sign * (-z).exp() * s_minus) / 2
        r = (2 * z / pi_dec(prec + 20)).ln() / 2 + i1.ln()
    with localcontext() as ctx:
        ctx.prec = prec
        return +r


def _gamma_int_or_half(a2: int, prec: int) -> Decimal:
    """Gamma(a2/2) for a positive integer a2 (integer or half-integer argument)."""
    if a2 % 2 == 0:
        return Decimal(factorial(a2 // 2 - 1))
    m = (a2 - 1) // 2                            # Gamma(m + 1/2) = (2m)! sqrt(pi) / (4^m m!)
    return (Decimal(factorial(2 * m)) / (Decimal(4) ** m * factorial(m))) * pi_dec(prec).sqrt()


def log_iv_series(v2: int, x, prec: int = 60) -> Decimal:
    """log I_{v2/2}(x) by direct linear summation of the defining series.

    ``v2`` is twice the order (so integer and half-integer orders are exact).
    All terms are positive; the sum stops once the terms fall below 10^-(prec+5)
    of the partial sum after the peak.
    """
    with localcontext() as ctx:
        ctx.prec = prec + 20
        z = _dec(x)
        hz = z / 2
        q = hz * hz
        v = Decimal(v2) / 2
        # Gamma(k + v + 1) for k = 0
        g = _gamma_int_or_half(v2 + 2, prec + 20)
        term = hz ** v / g if v2 % 2 == 0 else (hz.ln() * v).exp() / g
        s = Decimal(0)
        k = 0
        eps = Decimal(10) ** (-(prec + 5))
        while True:
            s += term
            k += 1
            term = term * q / (k * (k + v))
            if k > float(z) / 2 + 2 and term < eps * s:
                break
        r = s.ln()
    with localcontext() as ctx:
        ctx.prec = prec
        return +r


def log_kn_int(n: int, x, prec: int = 90) -> Decimal:
    """log K_n(x) for integer n >= 0 from DLMF 10.31.1 (cancels like e^{2x})."""
    with localcontext() as ctx:
        ctx.prec = prec + 20
        z = _dec(x)
        hz = z / 2
        q = hz * hz
        gam = euler_gamma(prec + 20)
        eps = Decimal(10) ** (-(prec + 15))
        # first finite sum
        s1 = Decimal(0)
        for k in range(n):
            s1 += Decimal(factorial(n - k - 1)) / factorial(k) * (-q) ** k
        part1 = s1 / (2 * hz ** n) if n > 0 else Decimal(0)
        # I_n(z) by its series
        i_n = Decimal(0)
        t = hz ** n / factorial(n)
        k = 0
        while True:
            i_n += t
            k += 1
            t = t * q / (k * (k + n))
            if k > float(z) + 5 and t < eps * i_n:
                break
        # psi(m+1) = -gamma + H_m
        s3 = Decimal(0)
        h_k = Decimal(0)                       # H_k
        h_nk = sum((Decimal(1) / j for j in range(1, n + 1)), Decimal(0))  # H_{n+k}
        t = Decimal(1) / factorial(n)          # q^k / (k! (n+k)!)
        k = 0
        while True:
            s3 += (2 * (-gam) + h_k + h_nk) * t
            k += 1
            h_k += Decimal(1) / k
            h_nk += Decimal(1) / (n + k)
            t = t * q / (k * (n + k))
            if k > float(z) + 5 and abs(t) * (h_k + h_nk + 2) < eps * abs(s3):
                break
        sign_ln = -1 if n % 2 == 0 else 1      # (-1)^{n+1}
        sign_3 = 1 if n % 2 == 0 else -1       # (-1)^n
        kn = part1 + sign_ln * hz.ln() * i_n + sign_3 * hz ** n * s3 / 2
        r = kn.ln()
    with localcontext() as ctx:
        ctx.prec = prec
        return +r


def log_factorial(m: int, prec: int = 60) -> Decimal:
    with localcontext() as ctx:
        ctx.prec = prec
        return Decimal(factorial(m)).ln()
