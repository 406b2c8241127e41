"""GPU parity of the Kronecker method for the subdomains and of the spectral
preconditioner, through the C ABI, against the CPU oracle on the same seeded
inputs.

The Kronecker method computes the same entries of Q_AA^-1 as the oracle's
direct solves (the Woodbury identity is exact), so the estimator from given
samples must agree to 1e-10 relative, as the block-tridiagonal method does.
The spectral preconditioner changes only the path of PCG to the same
solution: samples are compared with the oracle's exact solve at a bound that
follows from the stopping rule."""
import numpy as np
import pytest

import oracle as O
from paper_2309_05435_amd.inputs import Workload, normals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402

RTOL = 1e-10


def wl_of(m, T, P, tiles, n_l, frac=0.3, range_=0.3, rho=0.9, sigma=0.5, seed=11):
    return Workload(name="k", m=m, T=T, range_=range_, rho=rho, tau=1.0, sigma=sigma,
                    obs_frac=frac, n_tslabs=P, n_tiles=tiles, n_l=n_l, n_k=0, rtol=1e-12,
                    mask_seed=seed, z_seed=seed + 1)


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [
    # m, T, P, tiles, n_l
    (12, 8, 3, 1, 1),
    (14, 9, 3, 2, 1),
    (11, 7, 2, 2, 2),
    (10, 8, 4, 1, 0),
    (9, 6, 1, 1, 1),
    (13, 1, 1, 2, 1),
    (20, 6, 2, 1, 1),
    (34, 4, 1, 2, 1),
    # 3 x 3 tiles, 3 slabs: rim products (r on the rim of R only) in the
    # first, middle and last slabs
    (30, 7, 3, 3, 1),
]


@pytest.mark.parametrize("case", CASES)
def test_kron_from_samples_matches_oracle(case):
    m, T, P, tiles, n_l = case
    wl = wl_of(m, T, P, tiles, n_l)
    say("kron from_samples", case)
    M = O.OracleModel.from_workload(wl)
    lab = O.grid_cores(m, m, T, P, tiles, tiles)
    x = normals((67, M.n), 21)
    ref = M.rbmc(lab, P * tiles * tiles, n_l, x, 0b1111)
    gm = B.Model(wl)
    d0, t0, st, _ = gm.estimate_from_samples(None, grad_mask=0b1111, method=B.RBMC_SEL_KRON)
    assert st == B.RBMC_OK
    np.testing.assert_allclose(d0.cpu().numpy(), ref["diag_det"], rtol=RTOL)
    np.testing.assert_allclose(t0, ref["trace_det"], rtol=RTOL)
    diag, tr, st, _ = gm.estimate_from_samples(dev(x), grad_mask=0b1111, method=B.RBMC_SEL_KRON)
    assert st == B.RBMC_OK
    np.testing.assert_allclose(diag.cpu().numpy(), ref["diag"], rtol=RTOL)
    np.testing.assert_allclose(tr, ref["trace"], rtol=RTOL)
    gm.close()


def test_kron_sparse_observations():
    """1% observed: some time steps have no observations at all (their
    Woodbury groups are empty and their correction panels must be zero)."""
    wl = wl_of(14, 9, 3, 2, 1, frac=0.01, seed=29)
    say("kron sparse observations")
    M = O.OracleModel.from_workload(wl)
    mask = wl.mask().reshape(wl.T, -1)
    assert (mask.sum(axis=1) == 0).any()  # steps without observations
    lab = O.grid_cores(14, 14, 9, 3, 2, 2)
    x = normals((67, M.n), 22)
    ref = M.rbmc(lab, 12, 1, x, 0b1111)
    gm = B.Model(wl)
    diag, tr, st, _ = gm.estimate_from_samples(dev(x), grad_mask=0b1111, method=B.RBMC_SEL_KRON)
    assert st == B.RBMC_OK
    np.testing.assert_allclose(diag.cpu().numpy(), ref["diag"], rtol=RTOL)
    np.testing.assert_allclose(tr, ref["trace"], rtol=RTOL)
    gm.close()


def test_kron_strong_observations():
    """sigma = 0.05: the observations carry most of the posterior precision,
    the Woodbury correction cancels most of the prior variance."""
    wl = wl_of(12, 8, 2, 1, 1, frac=0.5, sigma=0.05)
    say("kron strong observations")
    M = O.OracleModel.from_workload(wl)
    lab = O.grid_cores(12, 12, 8, 2, 1, 1)
    x = normals((40, M.n), 22)
    ref = M.rbmc(lab, 2, 1, x, 0b1111)
    gm = B.Model(wl)
    diag, tr, st, _ = gm.estimate_from_samples(dev(x), grad_mask=0b1111, method=B.RBMC_SEL_KRON)
    np.testing.assert_allclose(diag.cpu().numpy(), ref["diag"], rtol=RTOL)
    np.testing.assert_allclose(tr, ref["trace"], rtol=RTOL)
    gm.close()


def test_kron_batches(monkeypatch):
    """A workspace cap of one byte makes every subdomain a batch of its own;
    the result must not depend on the batching."""
    wl = wl_of(14, 9, 3, 2, 1)
    M = O.OracleModel.from_workload(wl)
    lab = O.grid_cores(14, 14, 9, 3, 2, 2)
    x = normals((30, M.n), 24)
    ref = M.rbmc(lab, 12, 1, x, 0b1111)
    monkeypatch.setenv("RBMC_KRON_BATCH_BYTES", "1")
    gm = B.Model(wl)
    diag, tr, st, _ = gm.estimate_from_samples(dev(x), grad_mask=0b1111, method=B.RBMC_SEL_KRON)
    np.testing.assert_allclose(diag.cpu().numpy(), ref["diag"], rtol=RTOL)
    np.testing.assert_allclose(tr, ref["trace"], rtol=RTOL)
    gm.close()


def test_kron_and_blocktri_agree_mid_size():
    """A mid-size model on both methods (blocks of order 1600, 6 subdomains)."""
    wl = wl_of(36, 12, 3, 2, 2, range_=0.25, rho=0.95, frac=0.15)
    say("kron vs blocktri 36x36x12")
    gm = B.Model(wl)
    x = dev(normals((48, gm.n), 25))
    a, ta, _, _ = gm.estimate_from_samples(x, grad_mask=0b1111, method=B.RBMC_SEL_KRON)
    b, tb, _, _ = gm.estimate_from_samples(x, grad_mask=0b1111, method=B.RBMC_SEL_BLOCKTRI)
    rel = ((a - b).abs() / b.abs()).max().item()
    say(f"max rel diff diag {rel:.3e}")
    assert rel < 1e-10
    np.testing.assert_allclose(ta, tb, rtol=1e-10)
    gm.close()


@pytest.mark.parametrize("case", [(12, 8, 3, 1, 1), (14, 9, 3, 2, 1), (37, 5, 2, 1, 1),
                                  (16, 20, 2, 1, 1), (16, 40, 2, 1, 1), (16, 60, 2, 1, 1),
                                  (16, 70, 2, 1, 1)])
def test_spectral_sampler_matches_exact_solve(case):
    """Spectral-preconditioned PCG against the oracle's banded-Cholesky solve:
    ||x - x*|| <= cond(Q) rtol ||x*||; the residual is checked directly.  The
    time lengths cover each register size of the tridiagonal solve (T <= 16,
    32, 48, 64) and the chunked walk beyond 64."""
    m, T, P, tiles, n_l = case
    wl = wl_of(m, T, P, tiles, n_l)
    say("spectral sampler", case)
    M = O.OracleModel.from_workload(wl)
    z = normals((33, M.n + M.n_obs), 31)
    x_ref = M.sample(z)
    gm = B.Model(wl)
    x, st, rep = gm.sample(dev(z), rtol=1e-13, maxit=200, precond=B.RBMC_PC_SPECTRAL)
    bad = (~torch.isfinite(x)).any(dim=1).nonzero().flatten().tolist()
    say(f"status {st} pcg iterations max {rep.pcg_it_max} mean {rep.pcg_it_mean:.2f} "
        f"residual {rep.max_rel_residual:.3e} non-finite columns {bad}")
    assert st == B.RBMC_OK
    assert not bad
    assert rep.pcg_it_max <= 12
    x = x.cpu().numpy()
    b = M.rhs(z)
    res = np.linalg.norm(M.apply(O.Q, x) - b, axis=1) / np.linalg.norm(b, axis=1)
    assert res.max() <= 1.05e-13
    err = np.abs(x - x_ref).max() / np.abs(x_ref).max()
    assert err < 1e-8
    gm.close()


@pytest.mark.parametrize("mx,my,routes", [(64, 64, ("fft", "gemm", "direct")),
                                           (128, 32, ("fft", "direct")),
                                           (32, 32, ("fft", "direct"))])
def test_spectral_transform_routes_agree(monkeypatch, mx, my, routes):
    """The three DCT routes of the spectral preconditioner (FFT, matrix-core
    GEMM, direct kernel) give the same M^-1 b: after one PCG iteration the
    sampler returns x_1 = alpha M^-1 b, compared across routes."""
    wl = Workload(name="r", m=mx, T=5, range_=0.2, rho=0.9, tau=1.0, sigma=0.5, obs_frac=0.2,
                  n_tslabs=1, n_tiles=1, n_l=0, n_k=0, rtol=1e-12, mask_seed=51, z_seed=52)
    xs = {}
    for r in routes:
        monkeypatch.setenv("RBMC_SPEC_ROUTE", r)
        gm = B.Model(wl, shape=(mx, my))
        z = normals((9, gm.n + gm.n_obs), 53)
        x, st, rep = gm.sample(dev(z), rtol=1e-14, maxit=1, precond=B.RBMC_PC_SPECTRAL)
        assert st in (B.RBMC_OK, B.RBMC_W_NOT_CONVERGED)
        xs[r] = x.cpu().numpy()
        gm.close()
    ref = xs[routes[-1]]
    for r in routes[:-1]:
        err = np.abs(xs[r] - ref).max() / np.abs(ref).max()
        say(f"route {r} vs {routes[-1]} at {mx}x{my}: {err:.3e}")
        assert err < 1e-12


@pytest.mark.parametrize("route", ["fft", "gemm"])
def test_spectral_sampler_routes_converge(monkeypatch, route):
    """On a 64 x 64 grid both the FFT and the matrix-core DCT routes are
    available; the sampler must reach the tolerance with a true residual
    below it on either."""
    monkeypatch.setenv("RBMC_SPEC_ROUTE", route)
    wl = wl_of(64, 6, 2, 1, 1, range_=0.2, rho=0.95, frac=0.2)
    say(f"spectral {route} route 64x64x6")
    M = O.OracleModel.from_workload(wl)
    z = normals((20, M.n + M.n_obs), 32)
    gm = B.Model(wl)
    x, st, rep = gm.sample(dev(z), rtol=1e-12, maxit=200, precond=B.RBMC_PC_SPECTRAL)
    assert st == B.RBMC_OK
    say(f"pcg iterations {rep.pcg_it_max}")
    assert rep.pcg_it_max <= 8
    x = x.cpu().numpy()
    b = M.rhs(z)
    res = np.linalg.norm(M.apply(O.Q, x) - b, axis=1) / np.linalg.norm(b, axis=1)
    say(f"true residual {res.max():.3e}")
    assert res.max() <= 1.05e-12
    gm.close()


def test_estimate_spectral_kron_end_to_end():
    """rbmc_estimate with the spectral sampler and the Kronecker method against
    the oracle's estimator on its exact samples of the same z."""
    wl = wl_of(16, 10, 4, 1, 1, frac=0.5)
    M = O.OracleModel.from_workload(wl)
    lab = O.grid_cores(16, 16, 10, 4, 1, 1)
    z = normals((50, M.n + M.n_obs), 41)
    ref = M.rbmc(lab, 4, 1, M.sample(z), 0b1111)
    gm = B.Model(wl)
    diag, tr, st, rep = gm.estimate(dev(z), grad_mask=0b1111, rtol=1e-13, maxit=200,
                                    precond=B.RBMC_PC_SPECTRAL, method=B.RBMC_SEL_KRON)
    assert st == B.RBMC_OK
    np.testing.assert_allclose(diag.cpu().numpy(), ref["diag"], rtol=1e-8)
    np.testing.assert_allclose(tr, ref["trace"], rtol=1e-8)
    gm.close()


def test_device_normals_match_host_reference():
    import philox_ref
    gm = B.Model(wl_of(8, 4, 2, 1, 1))
    out = torch.empty(600, dtype=torch.float64, device="cuda")
    B.rbmc_normals(gm.ctx, 987654321012345, 1001, 600, out)
    ref = philox_ref.normals(987654321012345, 1001, 600)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-13, atol=1e-13)
    gm.close()


def test_device_z_and_sample_passes():
    """z = NULL draws the seed's stream; passes of 7 samples (a ragged last
    pass) equal one pass of 30 up to summation order."""
    wl = wl_of(14, 9, 3, 2, 1)
    gm = B.Model(wl)
    nz = gm.n + gm.n_obs
    zs = torch.empty(30 * nz, dtype=torch.float64, device="cuda")
    B.rbmc_normals(gm.ctx, 77, 0, 30 * nz, zs)
    kw = dict(grad_mask=0b1111, rtol=1e-12, maxit=200, precond=B.RBMC_PC_SPECTRAL,
              method=B.RBMC_SEL_KRON)
    d1, t1, st1, r1 = gm.estimate(zs.view(30, nz), **kw)
    d2, t2, st2, r2 = gm.estimate(None, n_samples=30, seed=77, **kw)
    d3, t3, st3, r3 = gm.estimate(None, n_samples=30, seed=77, sample_chunk=7, **kw)
    assert st1 == st2 == st3 == B.RBMC_OK
    np.testing.assert_allclose(d2.cpu().numpy(), d1.cpu().numpy(), rtol=1e-12)
    np.testing.assert_allclose(t2, t1, rtol=1e-12)
    np.testing.assert_allclose(d3.cpu().numpy(), d1.cpu().numpy(), rtol=1e-10)
    np.testing.assert_allclose(t3, t1, rtol=1e-10)
    say(f"plug-in error one pass {r1.err_estimate:.4e}, passes {r3.err_estimate:.4e}")
    assert abs(r3.err_estimate - r1.err_estimate) <= 1e-8 * r1.err_estimate
    gm.close()


@pytest.mark.parametrize("method,precond", [(B.RBMC_SEL_KRON, B.RBMC_PC_SPECTRAL),
                                            (B.RBMC_SEL_BLOCKTRI, B.RBMC_PC_BJ)])
def test_estimate_is_deterministic(method, precond):
    """The same call twice gives bitwise the same diagonal, traces and report:
    every reduction has a fixed order (no atomics on the outputs)."""
    wl = wl_of(20, 8, 2, 2, 1)
    gm = B.Model(wl)
    kw = dict(grad_mask=0b1111, rtol=1e-10, maxit=500, precond=precond, method=method)
    if method == B.RBMC_SEL_KRON:  # device normals, passes of 10
        kw.update(n_samples=24, seed=5, sample_chunk=10)
        z = None
    else:
        z = dev(normals((24, gm.n + gm.n_obs), 5))
    runs = [gm.estimate(z, **kw) for _ in range(2)]
    (d1, t1, s1, r1), (d2, t2, s2, r2) = runs
    assert s1 == s2 == B.RBMC_OK
    assert torch.equal(d1, d2)
    assert np.array_equal(np.asarray(t1), np.asarray(t2))
    assert r1.err_estimate == r2.err_estimate and r1.pcg_it_max == r2.pcg_it_max
    gm.close()
