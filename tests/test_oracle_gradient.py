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
