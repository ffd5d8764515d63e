#!/usr/bin/env python3
"""Write sampled rows of the FP64 oracle's result for the full-size 3-D
nonnormal Laplacian (128^3, +100 on the superdiagonal, p = 2, r = 2,
t = (0.5, 1) * 1e-3, v_j ~ U(-1, 1)) at tol 1e-6 and 1e-12.

The oracle needs minutes at this size, too long for every test run; the
parity tests pin the solve to the stored (shift, s) and compare the stored
rows.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_lap3d_nonnormal.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

NROWS = 1024


def sample_rows(n: int) -> np.ndarray:
    rng = np.random.default_rng(20250926)
    rows = np.concatenate([np.arange(4), n - 1 - np.arange(4),
                           rng.choice(n, NROWS - 8, replace=False)])
    return np.unique(rows)


def main() -> None:
    for tol in (1e-6, 1e-12):
        pr = wl.config3(nonnormal=True, tol=tol)
        prm = oracle.params(pr.op, pr.tol, pr.v)
        W, st = oracle.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol,
                             prm["shift"], prm["s"])
        rows = sample_rows(pr.n)
        out = {
            "problem": pr.name, "n": pr.n, "tol": tol,
            "params": {k: (float(v) if isinstance(v, float) else int(v))
                       for k, v in prm.items() if np.ndim(v) == 0},
            "stats": {k: int(v) for k, v in st.items()},
            "col_norm2": [float(x) for x in np.linalg.norm(W, axis=0)],
            "rows": [int(i) for i in rows],
            "W": [[float(x) for x in W[i]] for i in rows],
        }
        path = os.path.join(HERE, f"lap3d_128_nonnormal_tol{tol:.0e}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(path, st, flush=True)


if __name__ == "__main__":
    main()
