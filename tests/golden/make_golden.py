"""Write the stored expected values of the tiny workload.

Calls only the CPU oracle and the seeded input generator; never the GPU
library.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import rfgen  # noqa: E402


def main():
    p = rfgen.tiny()
    vis = p.make_vis()
    du, dv = p.cell()
    plan = oracle.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv,
                       kdm=p.kdm, threshold=p.threshold, nint=p.nint)
    stats, cands, _ = oracle.search(vis, plan)
    out = {
        "_what": "oracle results for the tiny workload (27-antenna Y array, 32 x 5 ms, 64 channels 1-2 GHz, "
                 "DM {0,50,100,150}, width 1, 256^2, seed 0, one DM=100 S/N 20 pulse at pixel (138, 121))",
        "_made_by": "tests/golden/make_golden.py (oracle only)",
        "W": plan.W,
        "du": du,
        "delays": plan.delays.tolist(),
        "candidates": [list(c) for c in cands],
        "stats": {f"{i},{j},{k}": list(v) for (i, j, k), v in sorted(stats.items())},
    }
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(len(cands), "candidates:", cands)


if __name__ == "__main__":
    main()
