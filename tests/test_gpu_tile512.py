"""Parity on the 512 x 512 x 48 workload (n = 12,582,912; 3 time slabs x 8 x 8
spatial tiles = 192 subdomains with 2 hops of overlap, regions of 4614-5144
nodes, chains of 18-20 steps), on the Kronecker-Woodbury method the
benchmark times.  The whole oracle does not run at this size: sampled
entries (the domain corner, an edge tile, interior tiles at a tile corner,
edge and centre, the last slab) are checked against the oracle on windows of
the grid (tests/golden/tile512_entries.json, written by
tests/golden/make_tile512_entries.py); the bar is 8 u max_p cond(Q_AA),
1.3e-7 (tests/cond_bars.py).  The log tau / log sigma trace identities are
checked at full size on the deterministic part and on an estimate from
samples of the model (spectral-preconditioned sampler, device normals: the
timed path).  With the fixture's white-noise x the Monte Carlo part of the
log tau identity is a zero formed from terms of size ||Q|| |mu| (||Q|| ~
1.6e9 here), so it is not checked on that run."""
import json
import os

import numpy as np
import pytest

from cond_bars import parity_bar
from paper_2309_05435_amd.inputs import WORKLOADS, normals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402

WL = WORKLOADS["tile512"]
with open(os.path.join(os.path.dirname(__file__), "golden", "tile512_entries.json")) as f:
    REF = json.load(f)


def test_sampled_entries_and_identities_tile512():
    bar = parity_bar(WL)
    print("tile512: building the model", flush=True)
    gm = B.Model(WL)
    try:
        x = torch.from_numpy(normals((REF["n_k"], gm.n), REF["x_seed"])).cuda()
        out = {}
        for xs, key in ((x, "full"), (None, "det")):
            print(f"tile512: estimate_from_samples ({key})", flush=True)
            diag, tr, st, rep = gm.estimate_from_samples(xs, grad_mask=0b1111,
                                                         method=B.RBMC_SEL_KRON)
            assert st == B.RBMC_OK
            out[key] = (diag.cpu().numpy(), np.asarray(tr))
        for e in REF["entries"]:
            i = e["node"]
            for key in ("det", "full"):
                g = out[key][0][i]
                print(f"tile512: core {e['core']} node {i} {key} gpu={g:.15e} "
                      f"oracle={e[key]:.15e} rel={abs(g - e[key]) / e[key]:.2e}", flush=True)
                assert abs(g - e[key]) <= bar * e[key]
        del x
        torch.cuda.empty_cache()
        print("tile512: estimate with 8 model samples", flush=True)
        diag, tr, st, rep = gm.estimate(None, grad_mask=0b1111, precond=B.RBMC_PC_SPECTRAL,
                                        method=B.RBMC_SEL_KRON, n_samples=8, seed=5,
                                        rtol=WL.rtol)
        assert st == B.RBMC_OK
        out["sampled"] = (diag.cpu().numpy(), np.asarray(tr))
        D = WL.mask() / WL.sigma ** 2
        for key in ("det", "sampled"):
            d, tr = out[key]
            s2 = float(np.sum(D * d))
            print(f"tile512: identities ({key}): {tr[1] + s2 - gm.n:.3e}, "
                  f"{(tr[3] + 2.0 * s2) / s2:.3e}", flush=True)
            assert abs(tr[1] + s2 - gm.n) < 1e-9 * gm.n
            assert abs(tr[3] + 2.0 * s2) < 1e-10 * s2
    finally:
        gm.close()
