"""The autotuner (rbmc_autotune): it times the candidate launch shapes end to
end, keeps the fastest on the context and caches it by workload signature;
estimates under any tuning agree with the default ones up to rounding."""
import numpy as np
import pytest

from paper_2309_05435_amd.inputs import Workload, normals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402


def say(*a):
    print(*a, flush=True)


WL = Workload(name="t", m=24, T=12, range_=0.3, rho=0.9, tau=1.0, sigma=0.5, obs_frac=0.3,
              n_tslabs=4, n_tiles=1, n_l=1, n_k=0, rtol=1e-10, mask_seed=21, z_seed=22)


def estimate(gm, z, grad=0b111):
    o = B.make_opts(z.shape[0], 5000, 1e-10, grad_mask=grad)
    d = torch.empty(gm.n, dtype=torch.float64, device="cuda")
    B.rbmc_model_set_theta(gm.m, *WL.theta)
    st, tr, rep = B.rbmc_estimate(gm.m, o, z, 0, d, B.popcount(grad))
    assert st == B.RBMC_OK
    return d.cpu().numpy(), np.array(tr)


def test_autotune_cache_and_agreement(tmp_path):
    cache = str(tmp_path / "tune.txt")
    gm = B.Model(WL, pc=(1, 1, 1))
    z = torch.from_numpy(normals((16, gm.n + gm.n_obs), 23)).cuda()
    d0, t0 = estimate(gm, z)                      # defaults
    default = B.rbmc_ctx_get_tune(gm.ctx)
    assert (default.small_k, default.small_tiles, default.wide_from) == (256, 768, 2048)
    rep = B.rbmc_autotune(gm.ctx, [gm.m], B.make_opts(16, 5000, 1e-10), [z], cache)
    say(f"autotune: best ({rep.best.small_k}, {rep.best.small_tiles}, {rep.best.wide_from}) "
        f"{rep.best_ms:.2f} ms, defaults {rep.default_ms:.2f} ms")
    assert rep.n_candidates == 8 and rep.cache_written == 1 and rep.from_cache == 0
    assert 0 < rep.best_ms <= rep.default_ms
    now = B.rbmc_ctx_get_tune(gm.ctx)
    assert (now.small_k, now.small_tiles, now.wide_from) == \
        (rep.best.small_k, rep.best.small_tiles, rep.best.wide_from)
    with open(cache) as f:
        lines = f.read().splitlines()
    assert len(lines) == 1 and len(lines[0].split()[0]) == 16
    # every candidate gives the same estimate up to rounding
    for sk, stl in ((512, 1536), (256, 0)):
        B.rbmc_ctx_set_tune(gm.ctx, sk, stl, 2048)
        d1, t1 = estimate(gm, z)
        assert np.max(np.abs(d1 / d0 - 1)) < 1e-10
        assert np.all(np.abs(t1 - t0) <= 1e-9 * np.abs(t0))
    # a fresh context reads the same choice from the cache, without runs
    gm2 = B.Model(WL, pc=(1, 1, 1))
    rep2 = B.rbmc_autotune(gm2.ctx, [gm2.m], B.make_opts(16, 5000, 1e-10), [z], cache)
    assert rep2.from_cache == 1 and rep2.default_ms == -1.0
    assert (rep2.best.small_k, rep2.best.small_tiles, rep2.best.wide_from) == \
        (rep.best.small_k, rep.best.small_tiles, rep.best.wide_from)
    # another workload (other sample count) is a different cache key
    rep3 = B.rbmc_autotune(gm2.ctx, [gm2.m], B.make_opts(0, 5000, 1e-10), [None], cache)
    assert rep3.from_cache == 0
    with open(cache) as f:
        assert len(f.read().splitlines()) == 2
    gm2.close()
    gm.close()


def test_set_tune_rejects_bad_values():
    gm = B.Model(WL, pc=(1, 1, 1))
    with pytest.raises(B.RbmcError):
        B.rbmc_ctx_set_tune(gm.ctx, 256, 768, 1024)   # below the workspace bound
    with pytest.raises(B.RbmcError):
        B.rbmc_ctx_set_tune(gm.ctx, -1, 768, 2048)
    gm.close()
