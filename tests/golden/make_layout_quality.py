"""Writes layout_quality_sbm_1k.json: final-layout quality of the FP64 oracle
on the 1,000-node SBM (10 blocks of 100, p_in 0.08, p_out 0.002), 300
iterations, N_int = 64, for 20 seeded uniform starts in [-1, 1]^2.

Per seed: normalised stress error SE and neighbourhood preservation NP1,
NP2 (Sec. 4, Metrics) of the final layout, for the exact repulsion
(k_mode 0) and for the interpolated repulsion with the k schedule
(k_mode -1). Calls only the oracle and the input generators.

Run from the repository root: python tests/golden/make_layout_quality.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synthgraphs as sg  # noqa: E402
from oracle import metrics as om  # noqa: E402
from oracle import tfdp as ot  # noqa: E402

SEEDS = list(range(20))
SEED_BASE = 9000


def main():
    w = sg.sbm_1k()
    g = w.graph
    out = {"graph": "sbm_1k", "n": g.n, "nnz": g.nnz, "n_int": 64, "total_iters": 300,
           "position_seeds": [SEED_BASE + s for s in SEEDS], "modes": {}}
    for k_mode in (-1, 0):
        rows = []
        t0 = time.time()
        for s in SEEDS:
            pos = sg.uniform_positions(g.n, SEED_BASE + s)
            p = ot.Params(n_int=64, k_mode=k_mode, total_iters=300)
            x = ot.layout(pos, g.row_ptr, g.col_idx, p)
            rows.append({
                "seed": SEED_BASE + s,
                "se": om.stress_error(x, g.row_ptr, g.col_idx),
                "np1": om.neighborhood_preservation(x, g.row_ptr, g.col_idx, 1),
                "np2": om.neighborhood_preservation(x, g.row_ptr, g.col_idx, 2),
            })
            print(k_mode, rows[-1], f"{time.time() - t0:.0f}s", flush=True)
        out["modes"][str(k_mode)] = rows
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "layout_quality_sbm_1k.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
