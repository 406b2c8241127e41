"""Gradient of the log marginal posterior of the hyperparameters (Sec. 3.4,
eq:hyperpar:1-4), for the model without fixed effects and a flat prior on
theta = (log kappa, log tau, rho, log sigma): the plain FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the product path.

At x = mu(theta) the three Gaussian densities of eq:hyperpar:1 give, up to a
constant,
  log pi(theta | y) = 1/2 log|Q_y| + 1/2 log|Q_u| - 1/2 log|Q|
                      - 1/2 (y - A_u mu)^T Q_y (y - A_u mu) - 1/2 mu^T Q_u mu,
with Q_u = Q_t (x) Q_s, Q_y = sigma^-2 I, Q = Q_u + A_u^T Q_y A_u and
mu = Q^-1 A_u^T Q_y y.  Since mu makes the exponent of the joint density
stationary in x, its theta-derivative drops out of the quadratic terms, so
  d_j log pi = 1/2 d_j log|Q_y| + 1/2 tr(Q_u^-1 d_j Q_u) - 1/2 tr(Q^-1 d_j Q)
               - 1/2 r^T (d_j Q_y) r - 1/2 mu^T (d_j Q_u) mu,   r = y - A_u mu,
where tr(Q^-1 d_j Q) is what the RBMC estimator returns (eq:hyperpar:4) and
the other terms are computed here by their definitions (dense inverse of
Q_u for its trace: small models only).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mean import posterior_mean

# operator codes of the oracle model (Q, dQ/dlog kappa, dQ/dlog tau, dQ/drho)
_Q, _DQ = 0, (1, 2, 3)
_QS, _QT = 6, 7


def _sparse(M, which):
    c = M.csr(which)
    return sp.csr_matrix((c.v, c.ci, c.rp), shape=(c.nr, c.nc))


def _logdet_spd(A) -> float:
    """log det of a sparse SPD matrix from its LU factors (library LU)."""
    lu = spla.splu(sp.csc_matrix(A))
    return float(np.sum(np.log(np.abs(lu.U.diagonal()))) + np.sum(np.log(np.abs(lu.L.diagonal()))))


def log_posterior(M, y) -> float:
    """log pi(theta | y) up to its theta-independent constant."""
    tau_y = math.exp(-2.0 * M.theta[3])
    obs = np.flatnonzero(M.mask)
    Qu = sp.kron(_sparse(M, _QT), _sparse(M, _QS))
    Q = _sparse(M, _Q)
    mu = posterior_mean(M, y, np.zeros((0, len(obs))), np.zeros(0))["mu_u"]
    r = np.asarray(y, np.float64) - mu[obs]
    return (0.5 * len(obs) * math.log(tau_y) + 0.5 * _logdet_spd(Qu) - 0.5 * _logdet_spd(Q)
            - 0.5 * tau_y * float(r @ r) - 0.5 * float(mu @ (Qu @ mu)))


def exact_traces(M) -> np.ndarray:
    """tr(Q^-1 d_j Q), j = log kappa, log tau, rho, log sigma, by a dense inverse."""
    Qi = np.linalg.inv(M.csr(_Q).dense())
    return np.array([float(np.sum(Qi * M.csr(w).dense())) for w in (1, 2, 3, 4)])


def gradient(M, y, traces) -> dict:
    """d_j log pi(theta | y) with the given tr(Q^-1 d_j Q) (4 values).
    Returns dict(grad, terms (4 x 5: the five terms of each component), mu)."""
    tau_y = math.exp(-2.0 * M.theta[3])
    obs = np.flatnonzero(M.mask)
    n_obs = len(obs)
    mu = posterior_mean(M, y, np.zeros((0, n_obs)), np.zeros(0))["mu_u"]
    r = np.asarray(y, np.float64) - mu[obs]
    Qu = np.kron(M.csr(_QT).dense(), M.csr(_QS).dense())
    Qu_inv = np.linalg.inv(Qu)
    terms = np.zeros((4, 5))
    for j in range(4):
        # d_j Q_u: the prior's derivative (Q's minus that of A_u^T Q_y A_u,
        # which depends on log sigma only)
        dQu = M.csr(_DQ[j]).dense() if j < 3 else np.zeros_like(Qu)
        # d_j log|Q_y| and d_j Q_y: Q_y = exp(-2 log sigma) I
        dlogQy = -2.0 * n_obs if j == 3 else 0.0
        dQy = -2.0 * tau_y if j == 3 else 0.0
        terms[j] = [0.5 * dlogQy,
                    0.5 * float(np.sum(Qu_inv * dQu)),
                    -0.5 * float(traces[j]),
                    -0.5 * dQy * float(r @ r),
                    -0.5 * float(mu @ (dQu @ mu))]
    return dict(grad=terms.sum(axis=1), terms=terms, mu=mu)
