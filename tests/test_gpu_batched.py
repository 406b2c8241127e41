"""Batched estimation of many uneven models in one call (rbmc_estimate_batched)
against separate rbmc_estimate calls on the same inputs, and against the
oracle's full pipeline for a few small models."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2309_05435_amd.inputs import Workload, batched_models, normals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small(m, T, P, tiles, n_l, seed, pc=None, rho=0.9, range_=0.3):
    return Workload(name=f"b{seed}", m=m, T=T, range_=range_, rho=rho, tau=1.0, sigma=0.5,
                    obs_frac=0.3, n_tslabs=P, n_tiles=tiles, n_l=n_l, n_k=0, rtol=1e-13,
                    mask_seed=seed, z_seed=seed + 1, pc=pc)


# uneven grids, time lengths, decompositions, overlaps and preconditioner blocks
SMALL = [small(12, 8, 3, 1, 1, 501), small(9, 5, 2, 2, 0, 502, pc=(1, 1, 1)),
         small(14, 6, 2, 2, 2, 503, rho=0.5, range_=0.2), small(20, 4, 1, 1, 1, 504),
         small(11, 1, 1, 2, 1, 505)]


def zs_for(ms, n_k, seed):
    return [torch.from_numpy(normals((n_k, n + no), seed + j)).cuda()
            for j, (n, no) in enumerate(zip(ms.n, ms.n_obs))]


def test_batched_matches_oracle_and_separate_calls():
    say("batched: small uneven models")
    ms = B.ModelSet(SMALL)
    zs = zs_for(ms, 40, 900)
    d_b, t_b, st, rep = ms.estimate(zs, grad_mask=0b1111, rtol=1e-13)
    assert st == B.RBMC_OK
    d_s, t_s, sts, _ = ms.estimate_each(zs, grad_mask=0b1111, rtol=1e-13)
    assert all(s == B.RBMC_OK for s in sts)
    for j, wl in enumerate(SMALL):
        say(f"batched: model {j} m={wl.m} T={wl.T}")
        np.testing.assert_allclose(d_b[j].cpu().numpy(), d_s[j].cpu().numpy(), rtol=1e-10)
        np.testing.assert_allclose(t_b[j], t_s[j], rtol=1e-10)
        M = O.OracleModel.from_workload(wl)
        lab = O.grid_cores(wl.m, wl.m, wl.T, wl.n_tslabs, wl.n_tiles, wl.n_tiles)
        ref = M.rbmc(lab, wl.n_tslabs * wl.n_tiles ** 2, wl.n_l, M.sample(zs[j].cpu().numpy()),
                     0b1111)
        np.testing.assert_allclose(d_b[j].cpu().numpy(), ref["diag"], rtol=1e-8)
        np.testing.assert_allclose(t_b[j], ref["trace"], rtol=1e-8)
    ms.close()


def test_batched_generated_models_match_separate_calls():
    """A slice of the generated uneven workload (grids 16-48, T 8-24, 2-8
    slabs) at its own tolerance, twice in a row (factors are reused)."""
    wls = batched_models()[:12]
    say("batched: generated models")
    ms = B.ModelSet(wls)
    zs = zs_for(ms, 24, 1200)
    for rep_i in range(2):
        d_b, t_b, st, rep = ms.estimate(zs, rtol=1e-10)
        assert st == B.RBMC_OK
        d_s, t_s, sts, _ = ms.estimate_each(zs, rtol=1e-10)
        for j in range(len(wls)):
            db, ds = d_b[j].cpu().numpy(), d_s[j].cpu().numpy()
            # the samples agree to the PCG tolerance; the estimator is linear
            # in the second moments of the samples
            assert np.max(np.abs(db - ds) / ds) < 1e-7, (rep_i, j)
            np.testing.assert_allclose(t_b[j], t_s[j], rtol=1e-7)
    ms.close()


def test_batched_without_gradients_and_samples():
    say("batched: no gradients, no samples")
    ms = B.ModelSet(SMALL[:3])
    zs = zs_for(ms, 8, 77)
    d_b, t_b, st, rep = ms.estimate(zs, grad_mask=0)
    assert st == B.RBMC_OK and all(t == [] for t in t_b)
    d_s, _, _, _ = ms.estimate_each(zs, grad_mask=0)
    for a, b in zip(d_b, d_s):
        np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-10)
    # n_k = 0: the deterministic part (diag of the subdomain inverses) only
    z0 = [z[:0] for z in zs]
    d0, _, st, _ = ms.estimate(z0, grad_mask=0)
    assert st == B.RBMC_OK
    for j, wl in enumerate(SMALL[:3]):
        M = O.OracleModel.from_workload(wl)
        lab = O.grid_cores(wl.m, wl.m, wl.T, wl.n_tslabs, wl.n_tiles, wl.n_tiles)
        ref = M.rbmc(lab, wl.n_tslabs * wl.n_tiles ** 2, wl.n_l, np.zeros((0, M.n)), 0)
        np.testing.assert_allclose(d0[j].cpu().numpy(), ref["diag_det"], rtol=1e-10)
    ms.close()


def test_batched_argument_errors():
    say("batched: errors")
    ms = B.ModelSet(SMALL[:2])
    other = B.ModelSet(SMALL[2:3])
    zs = zs_for(ms, 4, 5)
    diags = ms._diags()
    opts = B.make_opts(4)
    with pytest.raises(B.RbmcError) as e:  # a model listed twice
        B.rbmc_estimate_batched(ms.ctx, [ms.models[0], ms.models[0]], opts, [zs[0], zs[0]],
                                [diags[0], diags[0]], 3)
    assert e.value.status == B.RBMC_E_ARG
    with pytest.raises(B.RbmcError) as e:  # a model of another context
        B.rbmc_estimate_batched(ms.ctx, [ms.models[0], other.models[0]], opts, zs, diags, 3)
    assert e.value.status == B.RBMC_E_ARG
    st, trs, rep = B.rbmc_estimate_batched(ms.ctx, [], opts, [], [], 3)
    assert st == B.RBMC_OK
    other.close()
    ms.close()
