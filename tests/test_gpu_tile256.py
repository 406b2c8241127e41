"""Parity at the 256 x 256 x 64 workload (n = 4,194,304; 8 time slabs x 8 x 8
spatial tiles = 512 subdomains with one hop of overlap; dense blocks of
1153-1284 nodes; block-Jacobi blocks = whole 64-step chains of 16 x 16
spatial tiles, the workload's shape).  The whole oracle model is too large to
build at this size, so sampled outputs are checked against the oracle on
windows of the grid that contain each subdomain (exact, see tests/window.py),
and the trace identities are checked at full size."""
import numpy as np
import pytest

import oracle as O
from paper_2309_05435_amd.inputs import WORKLOADS, normals
from cond_bars import parity_bar
from window import estimator_entries, q_row

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402

WL = WORKLOADS["tile256"]
# 8 u max_p cond(Q_AA), cond bounded through the Kronecker factors of each
# Q_AA: 1.37e7 at the corner tiles of the first and last slabs, bar 1.2e-8
TOL = parity_bar(WL)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def model():
    say("tile256: building the model")
    gm = B.Model(WL)  # the workload's block-Jacobi shape (whole time chains of 16 x 16 tiles)
    yield gm, WL.mask()
    gm.close()


def test_estimator_sampled_entries_tile256(model):
    gm, mask = model
    x = normals((WL.n_k, gm.n), 91)
    say("tile256: estimate_from_samples")
    diag, tr, st, rep = gm.estimate_from_samples(torch.from_numpy(x).cuda(), grad_mask=0b1111)
    assert st == B.RBMC_OK
    d = diag.cpu().numpy()
    ns = WL.m * WL.m
    # cores: corner (slab 0, tile 0), interior, last slab at the far corner;
    # nodes at a core corner, edge, centre, and next to the domain boundary
    lab = O.grid_cores(WL.m, WL.m, WL.T, WL.n_tslabs, WL.n_tiles, WL.n_tiles)
    picks = {}
    for t, y, xg in [(0, 0, 0), (3, 5, 17), (7, 31, 31), (27, 100, 131), (28, 96, 96),
                     (63, 255, 255), (60, 250, 224)]:
        i = t * ns + y * WL.m + xg
        picks.setdefault(int(lab[i]), []).append(i)
    for p, nodes in picks.items():
        ref = estimator_entries(WL, mask, p, nodes, x)
        for i, (det, full) in zip(nodes, ref):
            say(f"tile256: core {p} node {i}: gpu {d[i]:.15e} oracle {full:.15e}")
            assert abs(d[i] - full) <= TOL * full
    D = mask / WL.sigma ** 2
    s2 = float(np.sum(D * d))
    assert abs(tr[1] + s2 - gm.n) < 1e-9 * gm.n
    assert abs(tr[3] + 2.0 * s2) < 1e-10 * s2


def test_operator_rows_tile256(model):
    gm, mask = model
    x = normals((2, gm.n), 92)
    xd = torch.from_numpy(x).cuda()
    rng = np.random.default_rng(5)
    nodes = [0, gm.n - 1] + list(rng.integers(0, gm.n, 6))
    for op, sel in [(B.RBMC_OP_Q, O.Q), (B.RBMC_OP_DQ_LOGKAPPA, O.DQ_LOGKAPPA),
                    (B.RBMC_OP_DQ_RHO, O.DQ_RHO)]:
        y = gm.apply(op, xd).cpu().numpy()
        for i in nodes:
            ref = q_row(WL, mask, sel, int(i), x)
            np.testing.assert_allclose(y[:, i], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_sampler_tile256(model):
    gm, mask = model
    z = torch.from_numpy(normals((8, gm.n + gm.n_obs), 93)).cuda()
    say("tile256: sample")
    x, st, rep = gm.sample(z, rtol=WL.rtol, maxit=5000)
    say(f"tile256: pcg iters max {rep.pcg_it_max} mean {rep.pcg_it_mean:.1f}")
    assert st == B.RBMC_OK
    b = gm.apply(B.RBMC_OP_F, z)
    r = b - gm.apply(B.RBMC_OP_Q, x)
    rel = (torch.linalg.norm(r, dim=1) / torch.linalg.norm(b, dim=1)).max().item()
    say(f"tile256: true relative residual {rel:.3e}")
    assert rel <= 1.05 * WL.rtol
