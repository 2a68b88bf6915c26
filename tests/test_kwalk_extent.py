"""Extent of the K fallback's integration walks (host model, no GPU).

The node tables of the cosh-integral rule hold e^{+-n} for integer parts
n < 32 only, so every walk must end before t = 32.  This model follows the
rule's placement of the grid (peak t* from the same start estimates and
Newton iteration, step h = min(cv / (1 + v/20), cs / sqrt(x cosh t*)) rounded
down to a multiple of 1/64, the window cut kDrop below the log-integrand at
the grid point nearest t*) in binary64 instead of the kernel's binary32, and
checks the largest node it visits over the fallback region of both
precisions' rules (and beyond it, v up to 16 and x up to 60)."""
import math

import numpy as np

GRID = 1.0 / 64.0
T_TABLE = 32.0   # integer parts held by the node tables


def _peak_step(v, x, cv, cs):
    t = 0.0
    if v * v > x:
        q = v / x
        r = v * q
        tu = math.asinh(q)
        ts = math.asinh(r)
        ts = math.asinh(r * ts)
        ts = math.asinh(r * ts)
        t = min(tu, ts)
        for _ in range(16):
            e = math.exp(t)
            z = math.exp(-2.0 * v * t)
            iz = 1.0 / (1.0 + z)
            psi = 0.5 * x * (e - 1.0 / e) - v * (1.0 - z) * iz
            dpsi = 0.5 * x * (e + 1.0 / e) - 4.0 * v * v * z * iz * iz
            if not dpsi > 0.0:
                t = tu
                continue
            dt = psi / dpsi
            t = max(t - dt, 0.0)
            if abs(dt) < 4e-3:
                break
    ch = math.cosh(t)
    hq = max(int(math.floor(min(cv / (1.0 + 0.05 * v), cs / math.sqrt(x * ch)) * 64.0)), 1)
    return int(round(t * 64.0)), hq


def _largest_node(v, x, kdrop, cv, cs):
    t0q, hq = _peak_step(v, x, cv, cs)
    t0 = t0q * GRID
    m = -x * math.cosh(t0) + v * t0 + math.log1p(math.exp(-2.0 * v * t0)) - math.log(2.0)

    def walk(i0, di, past_t0):
        far = 0
        for j in range(1024):
            iq = i0 + j * di
            far = max(far, abs(iq))
            ap = -x * math.cosh(iq * GRID) - m + v * iq * GRID
            if ap < -kdrop and (not past_t0 or iq > t0q):
                break
        return far

    if -x - m >= -kdrop:
        return walk(0, hq, True) * GRID
    return max(walk(t0q, hq, False), walk(t0q, -hq, False)) * GRID


def test_walks_end_inside_the_node_tables():
    worst = 0.0
    for x in np.geomspace(1e-10, 60.0, 40):
        for v in np.concatenate([[0.0], np.geomspace(1e-4, 16.0, 30)]):
            for kdrop, cv, cs in ((40.0, 0.25, 0.5), (18.0, 0.44, 1.0)):   # binary64, binary32 rules
                worst = max(worst, _largest_node(float(v), float(x), kdrop, cv, cs))
    assert worst < T_TABLE - 2.0, worst
