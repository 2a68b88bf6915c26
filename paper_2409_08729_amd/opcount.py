"""Branch probe for instruction counters.

Runs every branch of log I and log K (f64) on 2^18 identical elements, one
dispatch per branch, so that a counter run such as

    rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES -- python -m paper_2409_08729_amd.opcount

reports the VALU instructions one evaluation of that branch issues without
divergence (per element = SQ_INSTS_VALU / SQ_WAVES).  Dispatch order:
I mu20, I u13, I series, K mu20, K u13, K integral.
"""
import torch

import paper_2409_08729_amd as lb

POINTS = {  # (v, x) well inside each branch's region
    ("I", 0): (3.0, 40.0), ("I", 1): (40.0, 10.0), ("I", 2): (3.0, 5.0),
    ("K", 0): (3.0, 40.0), ("K", 1): (40.0, 10.0), ("K", 2): (3.0, 5.0),
}


def main(n: int = 1 << 18) -> None:
    for (kind, b), (v0, x0) in POINTS.items():
        v = torch.full((n,), v0, dtype=torch.float64, device="cuda:0")
        x = torch.full((n,), x0, dtype=torch.float64, device="cuda:0")
        lb.eval_branch(kind, b, v, x)
        torch.cuda.synchronize()
        print(f"{kind} branch {b} at v={v0} x={x0}: {n} elements", flush=True)


if __name__ == "__main__":
    main()
