"""Pins of the oracle's gradient of log pi(theta | y) (Sec. 3.4,
eq:hyperpar:1-4; no fixed effects, flat prior on theta), on the CPU.

The oracle assembles the gradient term by term from its definitions; the pin
is the central finite difference of the log posterior itself, evaluated
from exact log-determinants (sparse LU) and the exact posterior mean, with
the exact traces tr(Q^-1 d_j Q) plugged into the gradient.  A dropped term,
a wrong sign or factor, or a prior derivative taken from the wrong operator
fails it.  With one subdomain the RBMC estimator's traces are exact, so the
gradient from the estimator equals the one from the exact traces."""
import numpy as np
import pytest

import oracle as O
from oracle.gradient import exact_traces, gradient, log_posterior
from paper_2309_05435_amd.inputs import normals, obs_mask


def model(mx, my, T, frac, seed, theta):
    n = mx * my * T
    mask = obs_mask(n, frac, seed)
    h = 1.0 / (max(mx, my) - 1)
    return O.OracleModel(mx, my, T, h, *theta, mask)


CASES = [((5, 4, 3), 0.4, 41, (1.6, 0.2, 0.7, -0.5)),
         ((6, 6, 2), 0.25, 42, (2.2, -0.3, 0.5, 0.1)),
         ((4, 5, 4), 0.6, 43, (1.1, 0.5, 0.9, -0.9))]


@pytest.mark.parametrize("dims,frac,seed,theta", CASES)
def test_gradient_matches_finite_differences_of_the_log_posterior(dims, frac, seed, theta):
    M = model(*dims, frac, seed, theta)
    y = normals(M.n_obs, seed)
    g = gradient(M, y, exact_traces(M))["grad"]
    h = 1e-5
    fd = np.zeros(4)
    for j in range(4):
        tp, tm = list(theta), list(theta)
        tp[j] += h
        tm[j] -= h
        fd[j] = (log_posterior(model(*dims, frac, seed, tp), y)
                 - log_posterior(model(*dims, frac, seed, tm), y)) / (2 * h)
    scale = np.abs(gradient(M, y, exact_traces(M))["terms"]).sum(axis=1)
    np.testing.assert_allclose(g, fd, rtol=0, atol=1e-7 * scale.max())
    assert np.all(np.abs(g - fd) <= 1e-6 * np.maximum(scale, 1.0))


def test_single_subdomain_estimator_traces_give_the_exact_gradient():
    theta = (1.6, 0.2, 0.7, -0.5)
    M = model(5, 4, 3, 0.4, 44, theta)
    y = normals(M.n_obs, 44)
    lab = np.zeros(M.n, np.int32)
    x = normals((3, M.n), 45)
    tr = M.rbmc(lab, 1, 0, x, grad_mask=0b1111)["trace"]
    np.testing.assert_allclose(tr, exact_traces(M), rtol=1e-10)
    np.testing.assert_allclose(gradient(M, y, tr)["grad"], gradient(M, y, exact_traces(M))["grad"],
                               rtol=1e-9, atol=1e-9)


def test_without_observations_the_gradient_vanishes():
    """No data: the posterior of theta is its (flat) prior."""
    theta = (1.6, 0.2, 0.7, -0.5)
    M = model(5, 4, 3, 0.0, 46, theta)
    g = gradient(M, np.zeros(0), exact_traces(M))["grad"]
    np.testing.assert_allclose(g, 0.0, atol=1e-9)


# --------------------------------------------------------------------------
# with fixed effects (eq:hyperpar:3's Schur term) and the Alg. 6 iteration
# --------------------------------------------------------------------------

from oracle.gradient import alg6, gradient_fixed, log_posterior_fixed  # noqa: E402


def covariates(n_obs, nb, seed):
    a = normals((nb, n_obs), seed)
    if nb:
        a[0] = 1.0
    return a, 0.05 + np.abs(normals(nb, seed + 1))


@pytest.mark.parametrize("dims,frac,seed,theta,nb", [
    ((5, 4, 3), 0.4, 51, (1.6, 0.2, 0.7, -0.5), 2),
    ((4, 5, 4), 0.6, 52, (1.1, 0.5, 0.9, -0.9), 3)])
def test_fixed_effects_gradient_matches_finite_differences(dims, frac, seed, theta, nb):
    M = model(*dims, frac, seed, theta)
    y = normals(M.n_obs, seed)
    a, q = covariates(M.n_obs, nb, seed + 2)
    r = gradient_fixed(M, y, a, q, exact_traces(M))
    h = 1e-5
    fd = np.zeros(4)
    for j in range(4):
        tp, tm = list(theta), list(theta)
        tp[j] += h
        tm[j] -= h
        fd[j] = (log_posterior_fixed(model(*dims, frac, seed, tp), y, a, q)
                 - log_posterior_fixed(model(*dims, frac, seed, tm), y, a, q)) / (2 * h)
    scale = np.maximum(np.abs(r["terms"]).sum(axis=1), 1.0)
    assert np.all(np.abs(r["grad"] - fd) <= 1e-6 * scale), (r["grad"], fd)
    assert np.any(np.abs(r["terms"][:, 5]) > 1e-3)   # the Schur term matters here


def test_fixed_effects_gradient_without_covariates_is_the_plain_gradient():
    theta = (1.6, 0.2, 0.7, -0.5)
    M = model(5, 4, 3, 0.4, 53, theta)
    y = normals(M.n_obs, 53)
    tr = exact_traces(M)
    r0 = gradient(M, y, tr)
    r = gradient_fixed(M, y, np.zeros((0, M.n_obs)), np.zeros(0), tr)
    np.testing.assert_allclose(r["terms"][:, :5], r0["terms"], rtol=1e-12, atol=1e-10)
    assert not r["terms"][:, 5].any()


def test_alg6_reaches_the_mode_of_the_log_posterior():
    """On data drawn from the model, the iteration of Alg. 6 (diagonal
    Hessian from two first derivatives) stops where a general-purpose
    optimizer of the exact log posterior finds the mode.  log tau stays
    fixed: on a grid this small the data fix the marginal variance, a
    combination of kappa and tau, much better than either, and a diagonal
    Hessian crawls along that ridge."""
    from scipy.optimize import minimize
    dims, frac, seed, nb = (6, 6, 8), 0.8, 61, 2
    truth = np.array([1.9, 0.0, 0.5, -0.7])
    act = np.array([True, False, True, True])
    M0 = model(*dims, frac, seed, tuple(truth))
    obs = np.flatnonzero(M0.mask)
    a, q = covariates(len(obs), nb, seed + 2)
    Qu = np.kron(M0.csr(O.QT).dense(), M0.csr(O.QS).dense())
    u = np.linalg.solve(np.linalg.cholesky(Qu).T, normals(M0.n, seed + 3))
    y = u[obs] + a.T @ np.array([0.5, -0.3]) + np.exp(truth[3]) * normals(len(obs), seed + 4)

    def mk(th):
        return model(*dims, frac, seed, tuple(th))

    def full(v):
        th = truth.copy()
        th[act] = v
        return th

    def f(v):
        th = full(v)
        return 1e30 if abs(th[2]) >= 0.995 else -log_posterior_fixed(mk(th), y, a, q)

    best = full(minimize(f, truth[act], method="Nelder-Mead",
                         options=dict(xatol=1e-11, fatol=1e-14, maxiter=20000)).x)
    assert abs(best[2]) < 0.9   # an interior mode

    def grad_fn(M, y_, a_, q_, deterministic):
        return gradient_fixed(M, y_, a_, q_, exact_traces(M))["grad"]

    start = best + np.where(act, [0.08, -0.08, 0.04, 0.06], 0.0)
    path = alg6(mk, start, y, a, q, grad_fn, steps=60, max_step=0.1, active=act)
    assert len(path) < 61                                   # it converged
    th = path[-1]
    assert th[1] == truth[1]
    np.testing.assert_allclose(th, best, atol=1e-5)
    assert np.abs(grad_fn(mk(th), y, a, q, False)[act]).max() < 1e-6
