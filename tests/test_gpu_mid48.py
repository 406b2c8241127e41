"""Whole-oracle parity on the 48 x 48 x 16 workload: 8 time slabs of 2 steps
grown by 2 hops, i.e. chains of 4-6 dense blocks of 2304 nodes, the shape that
takes the batched multi-block update sweeps of the block-tridiagonal method.
Both subdomain methods (block-tridiagonal factor and selected inverse;
Kronecker-Woodbury) against tests/golden/mid48_oracle.npz, written by
tests/golden/make_mid48_oracle.py from the oracle alone: every diagonal
entry and the four traces, with the samples x and without (the deterministic
part).  cond(Q_AA) <= 1.55e6 here, so two backward-stable FP64 evaluations
agree to a few u cond ~ 1.7e-10 relative; the bar is 8 u max cond(Q_AA) =
1.4e-9 (tests/cond_bars.py), for the diagonal and for the traces, whose
sums cancel little on this workload."""
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

WL = WORKLOADS["mid48"]
X_SEED = 61  # the samples of the fixture
TOL = parity_bar(WL)
REF = np.load(os.path.join(os.path.dirname(__file__), "golden", "mid48_oracle.npz"))


@pytest.fixture(scope="module")
def model():
    print("mid48: building the model", flush=True)
    gm = B.Model(WL)
    yield gm
    gm.close()


@pytest.mark.parametrize("method", [B.RBMC_SEL_BLOCKTRI, B.RBMC_SEL_KRON])
def test_every_entry_and_trace_mid48(model, method):
    gm = model
    x = torch.from_numpy(normals((WL.n_k, gm.n), X_SEED)).cuda()
    for xs, dkey, tkey in ((x, "diag", "trace"), (None, "diag_det", "trace_det")):
        print(f"mid48: method {method} samples {0 if xs is None else WL.n_k}", flush=True)
        diag, tr, st, rep = gm.estimate_from_samples(xs, grad_mask=0b1111, method=method)
        assert st == B.RBMC_OK
        d = diag.cpu().numpy()
        t = np.asarray(tr)
        ed = np.max(np.abs(d - REF[dkey]) / np.abs(REF[dkey]))
        et = np.abs(t - REF[tkey]) / np.abs(REF[tkey])
        print(f"mid48: {dkey} max rel {ed:.3e}; {tkey} rel {et}", flush=True)
        assert ed <= TOL
        assert np.all(et <= TOL)
