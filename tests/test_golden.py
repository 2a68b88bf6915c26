"""The oracle against the stored closed-form fixture (tests/golden)."""
import os
from decimal import Decimal

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load():
    rows = []
    for line in open(os.path.join(HERE, "golden", "closed_forms.tsv")):
        if line.startswith("#"):
            continue
        k, v, x, y = line.rstrip("\n").split("\t")
        rows.append((k, float(v), float(x), Decimal(y)))
    return rows


def test_oracle_matches_golden(oracle):
    for kind, v, x, ref in load():
        f = oracle.log_iv if kind == "I" else oracle.log_kv
        hi, lo = f(np.array([v]), np.array([x]))
        got = Decimal(float(hi[0])) + Decimal(float(lo[0]))
        assert abs(got - ref) <= Decimal("1e-26") * max(Decimal(1), abs(ref)), (kind, v, x)
