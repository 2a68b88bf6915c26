"""Write closed_forms.tsv: 40-digit log K_{n+1/2}(x) and log I_{n+1/2}(x).

Values come only from tests/closed_forms.py (finite sums of DLMF 10.49.12
and 10.49.8 in decimal arithmetic); neither the oracle nor the GPU library is
involved.  Run from the repository root:

    python tests/golden/make_closed_forms.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import closed_forms as cf  # noqa: E402

POINTS_K = [(0, 1e-4), (0, 1.0), (0, 50.0), (1, 0.25), (2, 3.0), (5, 10.0), (7, 19.75),
            (12, 0.125), (14, 18.5), (20, 35.0), (60, 5.0), (200, 180.0), (1000, 2500.0)]
POINTS_I = [(0, 1e-3), (0, 1.0), (0, 120.0), (1, 0.75), (2, 2.5), (5, 10.0), (7, 19.75),
            (12, 0.5), (14, 22.5), (20, 35.0), (30, 90.0)]


def main():
    out = os.path.join(HERE, "closed_forms.tsv")
    with open(out, "w") as f:
        f.write("# kind\tv\tx\tlog_value (40 digits)\t"
                "source: DLMF 10.49.12 (K), DLMF 10.49.8 (I), half-integer orders\n")
        for n, x in POINTS_K:
            f.write(f"K\t{n + 0.5!r}\t{x!r}\t{cf.log_kv_half(n, x, prec=45):.40e}\n")
        for n, x in POINTS_I:
            f.write(f"I\t{n + 0.5!r}\t{x!r}\t{cf.log_iv_half(n, x, prec=260):.40e}\n")
    print(out)


if __name__ == "__main__":
    main()
