"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  FP64 throughout; the bar is 1e-10 relative for the
estimator from given samples and a
residual-derived bound for quantities that pass through PCG."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2309_05435_amd.inputs import Workload, normals, obs_mask

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402

RTOL = 1e-10


def wl_of(m, T, P, tiles, n_l, frac=0.3, range_=0.3, rho=0.9, sigma=0.5, seed=11, mx=None):
    return Workload(name="t", m=m, T=T, range_=range_, rho=rho, tau=1.0, sigma=sigma,
                    obs_frac=frac, n_tslabs=P, n_tiles=tiles, n_l=n_l, n_k=0, rtol=1e-12,
                    mask_seed=seed, z_seed=seed + 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def oracle_model(wl):
    return O.OracleModel.from_workload(wl)


CASES = [
    # m, T, P, tiles, n_l  -- slabs, tiles, wider overlap, no overlap, single core
    (12, 8, 3, 1, 1),
    (14, 9, 3, 2, 1),
    (11, 7, 2, 2, 2),
    (10, 8, 4, 1, 0),
    (9, 6, 1, 1, 1),
    (13, 1, 1, 2, 1),
    # spatial blocks above 256 nodes take the two-level (rank-256) inversion
    (20, 6, 2, 1, 1),
    (24, 5, 2, 1, 1),
    (34, 4, 1, 2, 1),
]


@pytest.mark.parametrize("op", [B.RBMC_OP_Q, B.RBMC_OP_DQ_LOGKAPPA, B.RBMC_OP_DQ_LOGTAU,
                                B.RBMC_OP_DQ_RHO, B.RBMC_OP_DQ_LOGSIGMA, B.RBMC_OP_F])
def test_apply_op_matches_oracle(op):
    wl = wl_of(37, 5, 2, 1, 1)  # 37 x 37 spans 2 x 3 stencil tiles with ragged edges
    say("apply_op", op, wl.m, wl.T)
    M = oracle_model(wl)
    gm = B.Model(wl)
    ncol = M.n + M.n_obs if op == B.RBMC_OP_F else M.n
    x = normals((3, ncol), 5)
    which = {B.RBMC_OP_Q: O.Q, B.RBMC_OP_DQ_LOGKAPPA: O.DQ_LOGKAPPA, B.RBMC_OP_DQ_LOGTAU: O.DQ_LOGTAU,
             B.RBMC_OP_DQ_RHO: O.DQ_RHO, B.RBMC_OP_DQ_LOGSIGMA: O.DQ_LOGSIGMA, B.RBMC_OP_F: O.F}[op]
    ref = M.apply(which, x)
    got = gm.apply(op, dev(x)).cpu().numpy()
    scale = np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * scale)
    gm.close()


@pytest.mark.parametrize("case", CASES)
def test_deterministic_part_matches_oracle(case):
    m, T, P, tiles, n_l = case
    wl = wl_of(m, T, P, tiles, n_l)
    say("det", case)
    M = oracle_model(wl)
    lab = O.grid_cores(m, m, T, P, tiles, tiles)
    ref = M.rbmc(lab, P * tiles * tiles, n_l, None, 0b1111)
    gm = B.Model(wl)
    diag, tr, st, rep = gm.estimate_from_samples(None, grad_mask=0b1111)
    d = diag.cpu().numpy()
    np.testing.assert_allclose(d, ref["diag_det"], rtol=RTOL)
    np.testing.assert_allclose(tr, ref["trace_det"], rtol=RTOL)
    gm.close()


@pytest.mark.parametrize("case", CASES)
def test_estimator_from_samples_matches_oracle(case):
    m, T, P, tiles, n_l = case
    wl = wl_of(m, T, P, tiles, n_l)
    say("from_samples", case)
    M = oracle_model(wl)
    lab = O.grid_cores(m, m, T, P, tiles, tiles)
    x = normals((67, M.n), 21)   # 67 samples: one full 64-sample tile and a ragged tail
    ref = M.rbmc(lab, P * tiles * tiles, n_l, x, 0b1111)
    gm = B.Model(wl)
    diag, tr, st, rep = gm.estimate_from_samples(dev(x), grad_mask=0b1111)
    np.testing.assert_allclose(diag.cpu().numpy(), ref["diag"], rtol=RTOL)
    np.testing.assert_allclose(tr, ref["trace"], rtol=RTOL)
    gm.close()


def test_more_samples_than_block_order():
    """n_k > n_p: the two directions of the correction solves take turns with
    one work panel instead of sharing launches (the block order is 64 here)."""
    wl = wl_of(8, 6, 2, 1, 1)
    say("samples > block order")
    M = oracle_model(wl)
    lab = O.grid_cores(8, 8, 6, 2, 1, 1)
    x = normals((150, M.n), 23)
    ref = M.rbmc(lab, 2, 1, x, 0b1111)
    gm = B.Model(wl)
    diag, tr, st, rep = gm.estimate_from_samples(dev(x), grad_mask=0b1111)
    np.testing.assert_allclose(diag.cpu().numpy(), ref["diag"], rtol=RTOL)
    np.testing.assert_allclose(tr, ref["trace"], rtol=RTOL)
    gm.close()


@pytest.mark.parametrize("case", [(12, 8, 3, 1, 1), (14, 9, 3, 2, 1), (11, 7, 2, 2, 2)])
def test_sampler_matches_exact_solve(case):
    """PCG x = Q^-1 F z against the oracle's banded-Cholesky solve; the error bound
    follows from the stopping rule: ||x - x*|| <= kappa(Q) * rtol * ||x*||."""
    m, T, P, tiles, n_l = case
    wl = wl_of(m, T, P, tiles, n_l)
    say("sampler", case)
    M = oracle_model(wl)
    z = normals((70, M.n + M.n_obs), 31)
    x_ref = M.sample(z)
    gm = B.Model(wl)
    x, st, rep = gm.sample(dev(z), rtol=1e-13, maxit=5000)
    assert st == B.RBMC_OK
    x = x.cpu().numpy()
    # residual computed by the oracle
    b = M.rhs(z)
    res = np.linalg.norm(M.apply(O.Q, x) - b, axis=1) / np.linalg.norm(b, axis=1)
    assert res.max() < 1e-12
    err = np.linalg.norm(x - x_ref, axis=1) / np.linalg.norm(x_ref, axis=1)
    assert err.max() < 1e-9
    assert rep.pcg_it_max >= 1 and rep.max_rel_residual <= 1e-13
    gm.close()


@pytest.mark.parametrize("precond", [B.RBMC_PC_BJ, B.RBMC_PC_SPECTRAL])
def test_solve_unit_vectors_gives_inverse_diagonal(precond):
    """rbmc_solve with b = e_i: x_i = (Q^-1)_ii, against a dense inverse of the
    oracle's Q (3 x 3 tiles of a 17 x 17 grid, ragged; both preconditioners)."""
    wl = wl_of(17, 6, 2, 3, 1)
    say("solve", precond)
    M = oracle_model(wl)
    Sigma = np.linalg.inv(M.csr(O.Q).dense())
    nodes = np.random.default_rng(41).choice(M.n, size=24, replace=False)
    E = np.zeros((len(nodes), M.n))
    E[np.arange(len(nodes)), nodes] = 1.0
    gm = B.Model(wl)
    bd = dev(E)
    x, st, rep = gm.solve(bd, rtol=1e-13, maxit=5000, precond=precond)
    assert st == B.RBMC_OK
    assert np.array_equal(bd.cpu().numpy(), E)  # b untouched
    x = x.cpu().numpy()
    np.testing.assert_allclose(x, Sigma[nodes], rtol=0, atol=1e-10 * np.abs(Sigma).max())
    np.testing.assert_allclose(x[np.arange(len(nodes)), nodes], np.diag(Sigma)[nodes],
                               rtol=1e-9)
    gm.close()


@pytest.mark.parametrize("pc", [(1, 2, 2), (2, 3, 1), (8, 1, 1)])
def test_sampler_with_other_block_jacobi_blocks(pc):
    """Preconditioner blocks other than the cores change the iteration count,
    not the solution the sampler converges to."""
    wl = wl_of(14, 8, 2, 1, 1)
    say("sampler pc", pc)
    M = oracle_model(wl)
    z = normals((9, M.n + M.n_obs), 32)
    x_ref = M.sample(z)
    gm = B.Model(wl, pc=pc)
    x, st, rep = gm.sample(dev(z), rtol=1e-13, maxit=5000)
    assert st == B.RBMC_OK
    err = np.linalg.norm(x.cpu().numpy() - x_ref, axis=1) / np.linalg.norm(x_ref, axis=1)
    assert err.max() < 1e-9
    gm.close()


@pytest.mark.parametrize("m,T", [(16, 6), (21, 5), (32, 3)])
def test_single_chain_sampler(m, T):
    """One block-Jacobi chain over the whole domain (the exact preconditioner):
    its inversions of order 256, 448 (a half-width last sweep step) and 1024
    (eight steps) run the two-block twisted factorization with rank-128
    sweeps.  The samples match the oracle's exact solve and PCG converges at
    once."""
    wl = wl_of(m, T, 2, 1, 1)
    say("single-chain sampler", m, T)
    M = oracle_model(wl)
    z = normals((40, M.n + M.n_obs), 33)
    x_ref = M.sample(z)
    gm = B.Model(wl, pc=(1, 1, 1))
    x, st, rep = gm.sample(dev(z), rtol=1e-12, maxit=50)
    assert st == B.RBMC_OK and rep.pcg_it_max <= 2
    err = np.linalg.norm(x.cpu().numpy() - x_ref, axis=1) / np.linalg.norm(x_ref, axis=1)
    assert err.max() < 1e-9
    gm.close()


def test_full_estimate_matches_oracle_pipeline():
    wl = wl_of(12, 8, 3, 1, 1)
    say("estimate")
    M = oracle_model(wl)
    lab = O.grid_cores(12, 12, 8, 3, 1, 1)
    z = normals((80, M.n + M.n_obs), 41)
    ref = M.rbmc(lab, 3, 1, M.sample(z), 0b1111)
    gm = B.Model(wl)
    diag, tr, st, rep = gm.estimate(dev(z), grad_mask=0b1111, rtol=1e-13)
    assert st == B.RBMC_OK
    np.testing.assert_allclose(diag.cpu().numpy(), ref["diag"], rtol=1e-8)
    np.testing.assert_allclose(tr, ref["trace"], rtol=1e-8)
    gm.close()


def test_single_core_is_exact_inverse():
    wl = wl_of(10, 6, 1, 1, 1)
    say("single core")
    M = oracle_model(wl)
    S = np.linalg.inv(M.csr(O.Q).dense())
    gm = B.Model(wl)
    x = normals((5, M.n), 2)
    diag, tr, st, rep = gm.estimate_from_samples(dev(x), grad_mask=0b1111)
    np.testing.assert_allclose(diag.cpu().numpy(), np.diag(S), rtol=1e-10)
    for j, s in enumerate((O.DQ_LOGKAPPA, O.DQ_LOGTAU, O.DQ_RHO, O.DQ_LOGSIGMA)):
        assert abs(tr[j] - np.sum(S * M.csr(s).dense())) < 1e-10 * abs(tr[j])
    gm.close()


def test_logtau_identity_on_gpu():
    wl = wl_of(16, 10, 4, 2, 1)
    say("identity")
    gm = B.Model(wl)
    x = normals((33, gm.n), 8)
    diag, tr, st, rep = gm.estimate_from_samples(dev(x), grad_mask=0b1010)
    D = wl.mask() / wl.sigma ** 2
    s = np.sum(D * diag.cpu().numpy())
    assert abs(tr[0] + s - gm.n) < 1e-9 * gm.n
    assert abs(tr[1] + 2 * s) < 1e-10 * s
    gm.close()


def test_error_codes():
    wl = wl_of(8, 4, 2, 1, 1)
    say("errors")
    mask = wl.mask()
    ctx = B.rbmc_ctx_create(0, None)
    for theta in [(1.0, 0.0, 1.0, 0.0), (float("nan"), 0.0, 0.5, 0.0)]:
        desc, _m = B.make_desc(8, 8, 4, 1 / 7, theta, mask)
        with pytest.raises(B.RbmcError) as e:
            B.rbmc_model_create(ctx, desc, B.rbmc_decomp_desc(2, 1, 1, 1))
        assert e.value.status == B.RBMC_E_ARG
    desc, _m = B.make_desc(8, 8, 4, 1 / 7, wl.theta, mask)
    with pytest.raises(B.RbmcError) as e:
        B.rbmc_model_create(ctx, desc, B.rbmc_decomp_desc(2, 1, 1, -1))
    assert e.value.status == B.RBMC_E_ARG
    m = B.rbmc_model_create(ctx, desc, B.rbmc_decomp_desc(2, 1, 1, 1))
    z = torch.zeros((4, 8 * 8 * 4 + int(mask.sum())), dtype=torch.float64, device="cuda")
    z[:, :10] = 1.0
    x = torch.empty((4, 8 * 8 * 4), dtype=torch.float64, device="cuda")
    st, rep = B.rbmc_sample(m, B.make_opts(4, pcg_maxit=1, pcg_rtol=1e-14), z, x)
    assert st == B.RBMC_W_NOT_CONVERGED
    with pytest.raises(B.RbmcError) as e:
        B.rbmc_sample(m, B.make_opts(4, pcg_maxit=0), z, x)
    assert e.value.status == B.RBMC_E_ARG
    with pytest.raises(B.RbmcError) as e:
        B.rbmc_sample(m, B.make_opts(4, precision=7), z, x)
    assert e.value.status == B.RBMC_E_ARG
    with pytest.raises(B.RbmcError) as e:
        B.rbmc_sample(m, B.make_opts(4, precond=B.RBMC_PC_SPECTRAL + 1), z, x)
    assert e.value.status == B.RBMC_E_ARG
    B.rbmc_model_destroy(m)
    B.rbmc_ctx_destroy(ctx)


def test_empty_inputs_and_column_limit():
    """Zero columns: the call succeeds and leaves its outputs untouched.  More
    than 65535 columns: rejected before any work (the buffers passed are far
    smaller and are never read).  An estimate with no samples is the
    deterministic part: bit-identical to the estimator run on no samples, and
    equal to the oracle's."""
    wl = wl_of(10, 4, 2, 1, 1)
    say("empty inputs and column limit")
    gm = B.Model(wl)
    n, n_obs = gm.n, gm.n_obs
    x = torch.full((1, n), 7.0, dtype=torch.float64, device="cuda")
    y = torch.full((1, n), 3.0, dtype=torch.float64, device="cuda")
    assert B.rbmc_apply_op(gm.m, B.RBMC_OP_Q, x, y, 0) == B.RBMC_OK
    for bad in (-1, 65536):
        with pytest.raises(B.RbmcError) as e:
            B.rbmc_apply_op(gm.m, B.RBMC_OP_Q, x, y, bad)
        assert e.value.status == B.RBMC_E_ARG
    z = torch.ones((1, n + n_obs), dtype=torch.float64, device="cuda")
    xs = torch.full((1, n), 5.0, dtype=torch.float64, device="cuda")
    st, _rep = B.rbmc_sample(gm.m, B.make_opts(0), z, xs)
    assert st == B.RBMC_OK
    with pytest.raises(B.RbmcError) as e:
        B.rbmc_sample(gm.m, B.make_opts(65536), z, xs)
    assert e.value.status == B.RBMC_E_ARG
    torch.cuda.synchronize()
    assert torch.all(y == 3.0) and torch.all(xs == 5.0)
    d_est = torch.empty(n, dtype=torch.float64, device="cuda")
    st, tr_est, _rep = B.rbmc_estimate(gm.m, B.make_opts(0, grad_mask=0b1111), None, 0, d_est, 4)
    assert st == B.RBMC_OK
    d_det, tr_det, st, _rep = gm.estimate_from_samples(None, grad_mask=0b1111)
    assert torch.equal(d_est, d_det) and tr_est == tr_det
    M = oracle_model(wl)
    ref = M.rbmc(O.grid_cores(10, 10, 4, 2, 1, 1), 2, 1, None, 0b1111)
    np.testing.assert_allclose(d_est.cpu().numpy(), ref["diag_det"], rtol=RTOL)
    np.testing.assert_allclose(tr_est, ref["trace_det"], rtol=RTOL)
    gm.close()


# Mixed precision: FP32 matrix-core products in the correction solves, FP64
# factorizations.  Every entry of Q_AA^-1 and of the corrections
# then carries a relative error of about 1e-6 (operand rounding to FP32), so
# the bar is 1e-5 relative per diagonal entry and, for a trace
# sum_ik S_ik (dQ_j)_ik, 1e-5 times its condition number
# c_j = sum_ik |S_ik (dQ_j)_ik| / |sum_ik S_ik (dQ_j)_ik| (the traces of
# dQ/dlog kappa and dQ/drho cancel strongly).  The measured errors are printed.
MIXED_TOL = 1e-5
GRADS = (O.DQ_LOGKAPPA, O.DQ_LOGTAU, O.DQ_RHO, O.DQ_LOGSIGMA)


def trace_condition(M):
    S = np.linalg.inv(M.csr(O.Q).dense())
    out = []
    for sel in GRADS:
        P = S * M.csr(sel).dense()
        out.append(np.abs(P).sum() / abs(P.sum()))
    return np.array(out)


def check_mixed(tag, d, tr, ref, cond):
    e_d = np.max(np.abs(d - ref["diag"]) / ref["diag"])
    e_t = np.abs(np.array(tr) - ref["trace"]) / np.abs(ref["trace"])
    say(f"{tag}: max rel err diag {e_d:.2e}; traces {np.array2string(e_t, precision=2)}"
        f" (condition {np.array2string(cond, precision=1)})")
    assert e_d < MIXED_TOL
    assert np.all(e_t < MIXED_TOL * cond)


@pytest.mark.parametrize("case", [(12, 8, 3, 1, 1), (20, 6, 2, 1, 1), (34, 4, 1, 2, 1)])
def test_mixed_precision_from_samples_error(case):
    m, T, P, tiles, n_l = case
    wl = wl_of(m, T, P, tiles, n_l)
    say("mixed from_samples", case)
    M = oracle_model(wl)
    lab = O.grid_cores(m, m, T, P, tiles, tiles)
    x = normals((67, M.n), 21)
    ref = M.rbmc(lab, P * tiles * tiles, n_l, x, 0b1111)
    gm = B.Model(wl)
    diag = torch.empty(gm.n, dtype=torch.float64, device="cuda")
    st, tr, rep = B.rbmc_estimate_from_samples(
        gm.m, B.make_opts(67, grad_mask=0b1111, precision=B.RBMC_MIXED), dev(x), diag, 4)
    check_mixed(f"mixed {case}", diag.cpu().numpy(), tr, ref, trace_condition(M))
    gm.close()


def test_mixed_precision_full_estimate():
    wl = wl_of(16, 8, 2, 1, 1)
    say("mixed estimate")
    M = oracle_model(wl)
    lab = O.grid_cores(16, 16, 8, 2, 1, 1)
    z = normals((70, M.n + M.n_obs), 43)
    ref = M.rbmc(lab, 2, 1, M.sample(z), 0b1111)
    cond = trace_condition(M)
    for pc in [None, (1, 1, 1)]:
        gm = B.Model(wl, pc=pc)
        diag = torch.empty(gm.n, dtype=torch.float64, device="cuda")
        st, tr, rep = B.rbmc_estimate(
            gm.m, B.make_opts(70, 5000, 1e-12, 0b1111, precision=B.RBMC_MIXED), dev(z), 0,
            diag, 4)
        assert st == B.RBMC_OK
        check_mixed(f"mixed estimate pc={pc} iters {rep.pcg_it_max}", diag.cpu().numpy(), tr,
                    ref, cond)
        gm.close()


def test_mixed_gemm_ragged_shapes():
    """The mixed product path on a ragged sample count (n_k = 37, not a
    multiple of the tile), through the correction solves: the estimate agrees
    with the FP64 one to the mixed-precision bar.  The sampler stays FP64 under
    RBMC_MIXED: its samples equal the FP64 ones bit for bit."""
    wl = wl_of(14, 9, 3, 2, 1)
    say("mixed ragged")
    M = oracle_model(wl)
    z = normals((37, M.n + M.n_obs), 31)
    gm = B.Model(wl, pc=(1, 1, 1))
    xs = []
    for prec in (B.RBMC_FP64, B.RBMC_MIXED):
        x = torch.empty((37, gm.n), dtype=torch.float64, device="cuda")
        st, rep = B.rbmc_sample(gm.m, B.make_opts(37, 5000, 1e-13, precision=prec), dev(z), x)
        assert st == B.RBMC_OK
        xs.append(x)
    assert torch.equal(xs[0], xs[1])
    x_ref = M.sample(z)
    err = np.linalg.norm(xs[0].cpu().numpy() - x_ref, axis=1) / np.linalg.norm(x_ref, axis=1)
    assert err.max() < 1e-9
    d64, tr64, st, _ = gm.estimate_from_samples(xs[0], grad_mask=0b1111)
    assert st == B.RBMC_OK
    ref = {"diag": d64.cpu().numpy(), "trace": np.array(tr64)}
    o = B.make_opts(37, grad_mask=0b1111, precision=B.RBMC_MIXED)
    dm = torch.empty_like(d64)
    st, trm, rep = B.rbmc_estimate_from_samples(gm.m, o, xs[0], dm, 4)
    assert st == B.RBMC_OK
    check_mixed("mixed ragged", dm.cpu().numpy(), trm, ref, trace_condition(M))
    gm.close()
