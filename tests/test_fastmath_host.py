"""Host build of the binary64 elementary functions of the device code
(csrc/lbessel_fastmath.hpp: exp64, log64, log1p64), compiled with g++ and
checked in units in the last place against 60-digit references from Python's
decimal module (an independent arbitrary-precision ln / exp)."""
import math
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_08729_amd", "csrc")

DRIVER = r"""
#define __host__
#define __device__
#define __forceinline__ inline
#include "lbessel_fastmath.hpp"
#include <stdio.h>
int main() {
    char op[8];
    double a;
    while (scanf("%7s %la", op, &a) == 2) {
        double r = 0.0;
        if (op[0] == 'e') r = lbessel::fm::exp64(a);
        else if (op[0] == 'l') r = lbessel::fm::log64(a);
        else r = lbessel::fm::log1p64(a);
        printf("%a\n", r);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def fm(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("fm")
    src = d / "fm.cpp"
    src.write_text(DRIVER)
    exe = d / "fm"
    subprocess.run([cxx, "-O2", "-ffp-contract=off", "-std=c++17", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)

    def run(op, xs):
        inp = "".join(f"{op} {float(x).hex()}\n" for x in xs)
        out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
        return [float.fromhex(t) for t in out.stdout.split()]
    return run


def _ulps(got, ref: Decimal):
    r = float(ref)
    return abs(Decimal(got) - ref) / Decimal(math.ulp(r))


def _ref(op, a):
    getcontext().prec = 60
    d = Decimal(a)
    if op == "e":
        return d.exp()
    if op == "l":
        return d.ln()
    if d < Decimal("1e-20"):      # 1 + d would round in 60 digits: series
        return d - d * d / 2 + d * d * d / 3
    return (1 + d).ln()


def _worst(fm, op, xs):
    got = fm(op, xs)
    return max(_ulps(g, _ref(op, a)) for g, a in zip(got, xs))


def test_exp64_within_one_ulp(fm):
    g = np.random.default_rng(1)
    xs = list(g.uniform(-700.0, 700.0, 3000)) + list(g.uniform(-1.0, 1.0, 1000)) \
        + [0.0, 1e-300, -1e-300, 0.5 * math.log(2), -0.5 * math.log(2), 709.0, -708.0]
    assert _worst(fm, "e", xs) <= 1.0


def test_log64_within_one_ulp(fm):
    g = np.random.default_rng(2)
    xs = list(10.0 ** g.uniform(-300.0, 300.0, 3000)) \
        + list(1.0 + g.uniform(-0.3, 0.3, 1000)) \
        + [5e-324, 1e-310, 2.2250738585072014e-308, 1.0, 2.0, 0.5, math.sqrt(0.5),
           math.nextafter(1.0, 2.0), math.nextafter(1.0, 0.0), 1.7e308]
    assert _worst(fm, "l", xs) <= 1.0


def test_log1p64_keeps_relative_accuracy_near_zero(fm):
    """log1p64(t) is ~1 ulp relative for every t >= 0, where log64(1 + t)
    loses all relative accuracy as t -> 0 (the case the I series needs:
    log I_v(x) ~ small corrections of size x^2/4)."""
    g = np.random.default_rng(3)
    xs = list(10.0 ** g.uniform(-40.0, 12.0, 4000)) \
        + [0.0, 5e-324, 1e-300, 2.0 ** -53, 2.0 ** -52, 3 * 2.0 ** -54, 1.0, 1e300]
    assert _worst(fm, "p", xs) <= 1.5
    # and log64 of the rounded sum really is the worse choice there
    t = 2.5e-9
    plain = fm("l", [1.0 + t])[0]
    assert _ulps(plain, _ref("p", t)) > 1e6
