"""Coefficients of the binary64 exp/log kernels in csrc/lbessel_fastmath.hpp.

Both are Chebyshev interpolants (near-minimax) computed in 60-digit
arithmetic with mpmath and rounded once to binary64:

  exp: e^r on |r| <= ln(2)/2, degree 11 (max relative error 4.5e-18);
       exp(y) = 2^k e^r with k = rint(y / ln 2), r = y - k ln 2.
  log: P(z) = (2 atanh(sqrt z)/sqrt z - 2)/z on 0 <= z <= ((sqrt2-1)/(sqrt2+1))^2,
       degree 6 (max absolute error 3.1e-16, i.e. 4.6e-18 relative in log);
       log(m) = 2s + s z P(z), s = (m-1)/(m+1), z = s^2, m in [sqrt(1/2), sqrt 2).
Also the split of ln 2 into a 32-bit head (exact products with |k| < 2^21)
and a binary64 tail.

    python paper_2409_08729_amd/fit_elementary.py   # prints the C++ constants
"""
import mpmath as mp


def fit():
    mp.mp.dps = 60
    a = mp.log(2) / 2
    pe, ee = mp.chebyfit(mp.exp, [-a, a], 12, error=True)
    smax = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
    g = lambda z: (2 * mp.atanh(mp.sqrt(z)) / mp.sqrt(z) - 2) / z if z != 0 else mp.mpf(2) / 3
    pl, el = mp.chebyfit(g, [0, smax ** 2], 7, error=True)
    ln2 = mp.log(2)
    head = mp.ldexp(mp.nint(mp.ldexp(ln2, 31)), -31)     # 32 significant bits
    tail = ln2 - head
    return pe, ee, pl, el, head, tail


def hexd(x) -> str:
    return float(x).hex()


if __name__ == "__main__":
    pe, ee, pl, el, head, tail = fit()
    print("// exp: e^r, |r| <= ln2/2, highest degree first; max rel err", mp.nstr(ee, 3))
    print("kExpC[] = {" + ", ".join(hexd(c) for c in pe) + "};")
    print("// log: P(z), highest degree first; max abs err", mp.nstr(el, 3))
    print("kLogP[] = {" + ", ".join(hexd(c) for c in pl) + "};")
    print("ln2 head", hexd(head), "tail", hexd(tail))
    print("log2(e)", hexd(1 / mp.log(2)))
