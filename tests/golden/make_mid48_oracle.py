"""Writes mid48_oracle.npz: the whole oracle estimator (every diagonal entry,
its deterministic part, and the four traces with their deterministic parts)
on a 48 x 48 x 16 grid split into 8 time slabs with 2 hops of overlap (8
subdomains with spatial blocks of 3096 nodes), for the samples
x = normals((16, n), 61).  Calls only the oracle; takes some minutes.

  python tests/golden/make_mid48_oracle.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2309_05435_amd.inputs import WORKLOADS, normals  # noqa: E402

WL = WORKLOADS["mid48"]
X_SEED = 61


def main():
    M = O.OracleModel.from_workload(WL)
    lab = O.grid_cores(WL.m, WL.m, WL.T, WL.n_tslabs, 1, 1)
    x = normals((WL.n_k, M.n), X_SEED)
    t = time.time()
    ref = M.rbmc(lab, WL.n_tslabs, WL.n_l, x, 0b1111)
    print(f"oracle estimator: {time.time() - t:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "mid48_oracle.npz"), diag=ref["diag"],
                        diag_det=ref["diag_det"], trace=ref["trace"],
                        trace_det=ref["trace_det"])


if __name__ == "__main__":
    main()
