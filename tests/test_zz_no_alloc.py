"""rbmc_apply_op_noalloc (operators without device allocation) against
rbmc_apply_op on the same inputs: two calls in a row per operator, the second
with fewer columns; the results must be identical (same kernels), and the
calls must leave the device's free memory unchanged."""
import numpy as np
import pytest

from paper_2309_05435_amd.inputs import Workload, normals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402

OPS = [B.RBMC_OP_Q, B.RBMC_OP_DQ_LOGKAPPA, B.RBMC_OP_DQ_LOGTAU, B.RBMC_OP_DQ_RHO,
       B.RBMC_OP_DQ_LOGSIGMA, B.RBMC_OP_F]


def test_noalloc_operators_match_allocating_calls():
    # 37 x 37 spans 2 x 3 stencil tiles with ragged edges
    wl = Workload(name="na", m=37, T=5, range_=0.3, rho=0.9, tau=1.0, sigma=0.5, obs_frac=0.3,
                  n_tslabs=2, n_tiles=1, n_l=1, n_k=0, rtol=1e-12, mask_seed=71, z_seed=72)
    gm = B.Model(wl)
    ins, outs = {}, {}
    for op in OPS:
        ncol = gm.n + gm.n_obs if op == B.RBMC_OP_F else gm.n
        for n_rhs, seed in ((5, 11), (2, 12)):
            ins[op, n_rhs] = torch.from_numpy(normals((n_rhs, ncol), seed + op)).cuda()
            outs[op, n_rhs] = torch.full((n_rhs, gm.n), float("nan"), dtype=torch.float64,
                                         device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for op in OPS:
        for n_rhs in (5, 2):  # two calls in a row, the second smaller
            B.rbmc_apply_op_noalloc(gm.m, op, ins[op, n_rhs], outs[op, n_rhs], n_rhs)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, f"device free memory changed by {free0 - free1} bytes"
    for op in OPS:
        for n_rhs in (5, 2):
            ref = gm.apply(op, ins[op, n_rhs])
            np.testing.assert_array_equal(outs[op, n_rhs].cpu().numpy(), ref.cpu().numpy())
    with pytest.raises(B.RbmcError) as e:
        B.rbmc_apply_op_noalloc(gm.m, B.RBMC_OP_Q, ins[B.RBMC_OP_Q, 5], outs[B.RBMC_OP_Q, 5],
                                70000)
    assert e.value.status == B.RBMC_E_ARG
    gm.close()
