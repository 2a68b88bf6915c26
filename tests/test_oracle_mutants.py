"""Strength of the oracle pins: plausible mistakes planted in copies of the
oracle (on the CPU) must each be caught.

Every mutant is the oracle source with one textual change (a dropped term, an
off-by-one index, a flipped sign, a loosened truncation, a wrong weight),
compiled into a temporary library.  `pins_pass` runs a compact version of
the pins of test_oracle_pins.py (closed forms at half-integer order, brute
force at exact Gamma values, integer-order K_n, the Wronskian, a derivative
identity, the vMF closed form) and must accept the real oracle and reject
every mutant.
"""
import os
from decimal import Decimal, localcontext

import numpy as np
import pytest

import closed_forms as cf
from oracle import oracle as oracle_mod

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbessel_oracle.c")

MUTANTS = {
    "series ratio index": ("t *= r2 / ((k + 1) * (k + 1 + v));", "t *= r2 / ((k + 1) * (k + v));"),
    "downward ratio index": ("t *= (k * (k + v)) / r2;", "t *= ((k + 1) * (k + v)) / r2;"),
    "dropped lgamma(i0+1)": ("- lgammaq(i0 + 1) - lgammaq(i0 + v + 1);",
                             "- lgammaq(i0 + v + 1);"),
    "peak term exponent": ("const qf log_ai = 2 * i0 * lhx", "const qf log_ai = i0 * lhx"),
    "loose series tail": ("SERIES_TAIL = 3.00926553810505e-36Q", "SERIES_TAIL = 1e-12Q"),
    "derivative weight sign": ("s1 += (2 * (k + 1) + v) * t;", "s1 += (2 * (k + 1) - v) * t;"),
    "log cosh constant": ("return a + log1pq(expq(-2 * a)) - M_LN2q;",
                          "return a + log1pq(expq(-2 * a));"),
    "trapezoid end weight": ("wt[n] = (j == 0) ? 0.5Q : 1;\n        ++n;\n        if (f > fmax)\n            fmax = f;\n        if (f < fmax - TRAP_DROP && f < prev)\n            break;\n        prev = f;\n    }\n    /* left",
                             "wt[n] = 1;\n        ++n;\n        if (f > fmax)\n            fmax = f;\n        if (f < fmax - TRAP_DROP && f < prev)\n            break;\n        prev = f;\n    }\n    /* left"),
    "short integrand tail": ("TRAP_DROP = 110.0Q", "TRAP_DROP = 8.0Q"),
    "K derivative sign": ("return -expq(klog_integral(&p1) - klog_integral(&p0));",
                          "return expq(klog_integral(&p1) - klog_integral(&p0));"),
    "vMF power of 2pi": ("return v * logq(kappa) - (p / 2) * log2pi - log_iv_q(v, kappa);",
                         "return v * logq(kappa) - v * log2pi - log_iv_q(v, kappa);"),
    "K order sign": ("qf r = -p->x * coshq(t) + log_cosh(p->v * t);",
                     "qf r = -p->x * coshq(t) + log_cosh(p->v * t + t);"),
}


class _NotFinite(Exception):
    pass


def qd(hi, lo):
    if not (np.isfinite(hi) and np.isfinite(lo)):
        raise _NotFinite()
    return Decimal(float(hi)) + Decimal(float(lo))


def pins_pass(o) -> bool:
    """Compact pin set; False at the first violated fact (or non-finite value)."""
    try:
        return _pins(o)
    except _NotFinite:
        return False


def _pins(o) -> bool:
    tol = Decimal("1e-24")
    with localcontext() as ctx:
        ctx.prec = 60
        for n, x in ((0, 0.5), (3, 2.0), (12, 19.7), (40, 300.0)):
            ref = cf.log_kv_half(n, x)
            h, l = o.log_kv(np.array([n + 0.5]), np.array([x]))
            if abs(qd(h[0], l[0]) - ref) > tol * max(1, abs(ref)):
                return False
        for n, x in ((0, 1.0), (3, 5.0), (10, 30.0)):
            ref = cf.log_iv_half(n, x, prec=200)
            h, l = o.log_iv(np.array([n + 0.5]), np.array([x]))
            if abs(qd(h[0], l[0]) - ref) > tol * max(1, abs(ref)):
                return False
        for v2, x in ((2, 1.5), (16, 22.0), (4, 0.3)):
            ref = cf.log_iv_series(v2, x)
            h, l = o.log_iv(np.array([v2 / 2]), np.array([x]))
            if abs(qd(h[0], l[0]) - ref) > tol * max(1, abs(ref)):
                return False
        for n, x in ((0, 1.0), (2, 3.0)):
            ref = cf.log_kn_int(n, x, prec=100)
            h, l = o.log_kv(np.array([float(n)]), np.array([x]))
            if abs(qd(h[0], l[0]) - ref) > tol * max(1, abs(ref)):
                return False
        # Wronskian at a non-special order
        v = np.array([0.375, 7.25, 40.125])        # v + 1 exact
        x = np.array([0.7, 12.0, 90.0])
        li0, li1, lk0, lk1 = o.log_iv(v, x), o.log_iv(v + 1, x), o.log_kv(v, x), o.log_kv(v + 1, x)
        for i in range(v.size):
            a = qd(li0[0][i], li0[1][i]) + qd(lk1[0][i], lk1[1][i])
            b = qd(li1[0][i], li1[1][i]) + qd(lk0[0][i], lk0[1][i])
            m = max(a, b)
            lse = m + ((a - m).exp() + (b - m).exp()).ln()
            if abs(lse + Decimal(float(x[i])).ln()) > Decimal("1e-25") * 100:
                return False
        # derivative identities
        di, dk = o.dlog_iv(v, x), o.dlog_kv(v, x)
        for i in range(v.size):
            vx = Decimal(float(v[i])) / Decimal(float(x[i]))
            ri = (qd(li1[0][i], li1[1][i]) - qd(li0[0][i], li0[1][i])).exp() + vx
            rk = vx - (qd(lk1[0][i], lk1[1][i]) - qd(lk0[0][i], lk0[1][i])).exp()
            if abs(qd(di[0][i], di[1][i]) - ri) > Decimal("1e-22") * max(1, abs(ri)):
                return False
            if abs(qd(dk[0][i], dk[1][i]) - rk) > Decimal("1e-22") * max(1, abs(rk)):
                return False
        # vMF at p = 3
        k = 3.0
        h, l = o.vmf_log_norm(np.array([k]), 3.0)
        kd = Decimal(k)
        ref = kd.ln() - (4 * cf.pi_dec(60)).ln() - ((kd.exp() - (-kd).exp()) / 2).ln()
        if abs(qd(h[0], l[0]) - ref) > tol * max(1, abs(ref)):
            return False
    return True


def test_real_oracle_passes_compact_pins(oracle):
    assert pins_pass(oracle)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique: {name}"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = oracle_mod.compile_oracle(str(src), str(tmp_path / "mutant.so"))
    mutant = oracle_mod.Oracle(lib)
    assert not pins_pass(mutant), f"mutant not caught: {name}"
