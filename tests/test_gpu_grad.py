"""GPU parity of rbmc_grad_log_posterior (the gradient of log pi(theta | y),
Sec. 3.4, eq:hyperpar:1-4; no fixed effects, flat prior on theta) against
the oracle, through the C ABI, term by term.

Both sides take tr(Q^-1 d_j Q) from the RBMC estimator on the same samples
and decomposition; the library's closed-form prior terms meet the oracle's
dense traces of Q_u^-1 d_j Q_u.  Bars per component j: the estimator's trace
parity (1e-10 relative) on 1/2 tr_j, plus what the solve's tolerance allows
in the mu terms: with ||mu - mu*|| <= d ||mu||, d = rtol cond(Q) (cond(Q)
bounded through the Kronecker factors), 1/2 mu^T A mu moves by at most
d ||A|| ||mu||^2 and tau_y ||r||^2 by 2 tau_y ||r|| d ||mu||; four times
these for rounding."""
import numpy as np
import pytest

import oracle as O
from cond_bars import cond_bound
from oracle.gradient import gradient
from paper_2309_05435_amd.inputs import WORKLOADS, Workload, normals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402

RTOL = 1e-13


def say(*a):
    print(*a, flush=True)


def wl_of(m, T, P, tiles, n_l, frac, seed):
    return Workload(name="grad", m=m, T=T, range_=0.3, rho=0.85, tau=1.0, sigma=0.5,
                    obs_frac=frac, n_tslabs=P, n_tiles=tiles, n_l=n_l, n_k=0, rtol=RTOL,
                    mask_seed=seed, z_seed=seed + 1)


CASES = [
    # m, T, slabs, tiles, n_l, obs fraction, samples, preconditioner
    (12, 8, 3, 1, 1, 0.3, 16, B.RBMC_PC_BJ),
    (14, 9, 3, 2, 1, 0.2, 8, B.RBMC_PC_SPECTRAL),
    (11, 7, 2, 2, 2, 0.4, 0, B.RBMC_PC_SPECTRAL),   # the estimator's deterministic part only
    (10, 6, 2, 1, 1, 0.0, 5, B.RBMC_PC_BJ),         # no observations
]


@pytest.mark.parametrize("m,T,P,tiles,n_l,frac,nk,precond", CASES)
def test_gradient_matches_oracle(m, T, P, tiles, n_l, frac, nk, precond):
    seed = 700 + m + T + nk
    wl = wl_of(m, T, P, tiles, n_l, frac, seed)
    say(f"grad {m}x{m}x{T} cores {P}x{tiles}x{tiles} n_l {n_l} obs {frac} samples {nk}")
    M = O.OracleModel.from_workload(wl)
    y = normals(M.n_obs, seed)
    x = normals((nk, M.n), seed + 5) if nk else None
    lab = O.grid_cores(m, m, T, P, tiles, tiles)
    tr = M.rbmc(lab, P * tiles * tiles, n_l, x, 0b1111)["trace"]
    ref = gradient(M, y, tr)
    gm = B.Model(wl)
    g, terms, mu, st, rep = gm.grad_log_posterior(
        torch.from_numpy(y).cuda(), None if x is None else torch.from_numpy(x).cuda(),
        rtol=RTOL, precond=precond)
    gm.close()
    assert st == B.RBMC_OK
    mu_o = ref["mu"]
    d = RTOL * cond_bound(wl.replace(n_tslabs=1, n_tiles=1))["K"]
    tau_y = 1.0 / wl.sigma ** 2
    r = y - mu_o[np.flatnonzero(M.mask)]
    nmu = np.linalg.norm(mu_o)
    for j in range(4):
        A = M.csr((O.DQ_LOGKAPPA, O.DQ_LOGTAU, O.DQ_RHO)[j]).dense() if j < 3 else None
        bar = 0.5e-10 * abs(ref["terms"][j, 2])
        if j < 3:
            bar += d * np.linalg.norm(A, 2) * nmu ** 2
        else:
            bar += 2 * tau_y * np.linalg.norm(r) * d * nmu
        bar = 4 * bar + 1e-13 * np.abs(ref["terms"][j]).sum()
        err = np.abs(terms[j] - ref["terms"][j])
        say(f"  component {j}: grad {g[j]:.6e} oracle {ref['grad'][j]:.6e}, term errors "
            f"{np.array2string(err, precision=2)}, bar {bar:.2e}")
        assert err.max() <= bar
        assert abs(g[j] - ref["grad"][j]) <= 5 * bar
    np.testing.assert_allclose(mu.cpu().numpy(), mu_o, rtol=0, atol=10 * d * nmu)


def test_gradient_full_size_device_samples():
    """512 x 512 x 48, the configuration's 200 samples drawn on the device:
    the closed-form terms, and the traces equal to those of a separate
    rbmc_estimate call with the same seed and options (the same samples; the
    subdomain batches follow the free memory, so the sums may be grouped
    differently: equal to rounding)."""
    wl = WORKLOADS["tile512"]
    say("grad tile512: building the model")
    gm = B.Model(wl)
    y = torch.from_numpy(normals(gm.n_obs, 512)).cuda()
    kw = dict(n_samples=wl.n_k, seed=77, rtol=wl.rtol, maxit=500, precond=B.RBMC_PC_SPECTRAL,
              method=B.RBMC_SEL_KRON)
    g, terms, mu, st, rep = gm.grad_log_posterior(y, **kw)
    say(f"grad tile512: {rep.t_total:.2f} s, grad {g}, pcg iters {rep.pcg_it_max}")
    assert st == B.RBMC_OK and np.all(np.isfinite(terms))
    assert terms[1, 1] == 0.5 * gm.n and terms[3, 0] == -gm.n_obs
    assert terms[3, 1] == 0.0 and terms[3, 4] == 0.0 and terms[3, 3] > 0
    diag = torch.empty(gm.n, dtype=torch.float64, device="cuda")
    _, tr, _ = B.rbmc_estimate(gm.m, B.make_opts(wl.n_k, 500, wl.rtol, grad_mask=0b1111,
                                                 precond=B.RBMC_PC_SPECTRAL,
                                                 method=B.RBMC_SEL_KRON), None, 77, diag, 4)
    np.testing.assert_allclose(terms[:, 2], -0.5 * np.asarray(tr), rtol=1e-12)
    gm.close()
