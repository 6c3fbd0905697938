"""Write tests/golden/plane_wall_k10.json from the FP64 oracle only.

The paper prints no worked example for the nearest-points search or the
covariance (Sec. III-C.1), so this fixture is not a paper value: it freezes
the oracle's output on the seeded 2,048-point plane + wall cloud (self-query,
k = 10, no radius cap) for 32 rows, so that any later change of the oracle's
arithmetic shows up as a failing test that must name its justification.
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_2308_07173_amd import workloads  # noqa: E402

ROWS = list(range(0, 2048, 64))


def main():
    p = workloads.plane_wall(2048, seed=0)
    idx, d2, cnt = oracle.knn(p, p, 10)
    cov = oracle.covariances(p, idx, cnt)
    out = {
        "source": "oracle/lkc_oracle.c on workloads.plane_wall(2048, seed=0); self-query, "
                  "k=10, radius=inf, eps=1e-3 (paper Sec. III-C.1 prints no values)",
        "rows": ROWS,
        "idx": idx[ROWS].tolist(),
        "d2": [[float(v) for v in r] for r in d2[ROWS]],
        "count": cnt[ROWS].tolist(),
        "mean": cov["mean"][ROWS].tolist(),
        "cov": cov["cov"][ROWS].reshape(len(ROWS), 9).tolist(),
        "reg": cov["reg"][ROWS].reshape(len(ROWS), 9).tolist(),
        "valid": cov["valid"][ROWS].tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plane_wall_k10.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
