"""Writes tile512_entries.json: estimator values of the 512 x 512 x 48
workload (192 subdomains, 2 hops of overlap) at sampled nodes, for the
samples x = normals((8, n), 91), computed by the oracle on windows of the
grid (tests/window.py: the oracle's model and overlap growth, Q_AA^-1 e_i by a
sparse LU), with the per-entry rounding bounds of
window.estimator_entries_bounded.  Calls only the oracle (and SciPy's sparse
LU as a library step); takes several minutes per subdomain.

  python tests/golden/make_tile512_entries.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2309_05435_amd.inputs import WORKLOADS, normals  # noqa: E402
from window import estimator_entries_bounded  # noqa: E402

WL = WORKLOADS["tile512"]
SEED, NK = 91, 8
# (t, y, x) picks: corner core at the domain corner, an edge core, two
# interior cores (core corner, edge and centre nodes), the last slab
PICKS = [(0, 0, 0), (2, 63, 5), (20, 100, 130), (17, 64, 64), (24, 300, 250), (30, 255, 256),
         (47, 511, 511), (40, 500, 260)]


def main():
    mask = WL.mask()
    x = normals((NK, WL.n), SEED)
    lab = O.grid_cores(WL.m, WL.m, WL.T, WL.n_tslabs, WL.n_tiles, WL.n_tiles)
    ns = WL.m * WL.m
    by_core = {}
    for t, y, xg in PICKS:
        i = t * ns + y * WL.m + xg
        by_core.setdefault(int(lab[i]), []).append(i)
    out = {"workload": WL.name, "x_seed": SEED, "n_k": NK,
           "note": "windowed oracle (sparse LU of Q_AA); bound = per-entry rounding bound",
           "entries": []}
    for p, nodes in sorted(by_core.items()):
        t0 = time.time()
        vals = estimator_entries_bounded(WL, mask, p, nodes, x)
        for i, (det, full, bdet, bfull) in zip(nodes, vals):
            out["entries"].append({"core": p, "node": i, "det": det, "full": full,
                                   "bound_det": bdet, "bound_full": bfull})
        print(f"core {p}: {len(nodes)} nodes, {time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "tile512_entries.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
