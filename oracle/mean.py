"""Posterior mean with fixed effects (Sec. 3.1, eq:mean:3-5) and the
fixed-effects term of the latent marginal variances (Sec. 3.2, eq:var:1):
the plain FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and by the oracle's own
gradient module, never by the product path.

The latent field is x = (u, beta) (eq:lgm:1): u on the space-time grid with
prior precision Q_u = Q_t (x) Q_s, beta with a diagonal prior precision
Q_beta.  The observations are y = A_u u + A_beta beta + noise, with Q_y =
tau_y I and tau_y = sigma^-2 (the model's D on the observed nodes); A_u
selects the observed nodes in ascending node order and A_beta (n_obs x
n_beta) holds the covariates.  Then Q_uu = Q_u + A_u^T Q_y A_u is the
model's Q.  The steps below follow eq:mean:3-5 in the paper's order, with a
sparse LU of Q_uu (a library primitive) for every solve with it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def blocks(M, a_beta, q_beta):
    """The blocks of eq:mean:3 and the pieces of A: (obs, tau_y, A_beta as
    n_obs x n_beta, Q_uu as CSC, Q_ubeta (n x n_beta), Q_betabeta)."""
    n = M.n
    obs = np.flatnonzero(M.mask)
    tau_y = float(np.exp(-2.0 * M.theta[3]))
    a = np.asarray(a_beta, np.float64).reshape(len(q_beta), len(obs)).T
    c = M.csr(0)                                           # the model's Q = Q_uu
    quu = sp.csr_matrix((c.v, c.ci, c.rp), shape=(n, n)).tocsc()
    qub = np.zeros((n, a.shape[1]))
    qub[obs] = tau_y * a                                   # A_u^T Q_y A_beta
    qbb = np.diag(np.asarray(q_beta, np.float64)) + tau_y * (a.T @ a)
    return obs, tau_y, a, quu, qub, qbb


def posterior_mean(M, y, a_beta, q_beta):
    """y: n_obs observations (ascending observed node); a_beta: n_beta rows of
    n_obs covariate values (covariate j contiguous); q_beta: n_beta prior
    precisions.  Returns dict(mu_u (n), mu_beta (n_beta), var_beta = S^-1,
    var_u_add = diag(Q_uu^-1 Q_ubeta S^-1 Q_betau Q_uu^-1) (n), solves)."""
    obs, tau_y, a, quu, qub, qbb = blocks(M, a_beta, q_beta)
    n, nb = M.n, a.shape[1]
    y = np.asarray(y, np.float64)
    lu = spla.splu(quu)
    b_u = np.zeros(n)
    b_u[obs] = tau_y * y                                   # A_u^T Q_y y
    b_b = tau_y * (a.T @ y)                                # A_beta^T Q_y y
    # eq:mean:5, first line: Q_uu^-1 (A_u^T Q_y y) and Q_uu^-1 Q_ubeta
    # (n_beta + 1 solves), the Schur complement S of Q_uu, then mu_beta
    w = lu.solve(b_u)
    W = lu.solve(qub) if nb else np.zeros((n, 0))
    S = qbb - qub.T @ W
    mu_b = np.linalg.solve(S, b_b - qub.T @ w) if nb else np.zeros(0)
    # second line: one more solve with Q_uu for mu_u
    mu_u = lu.solve(b_u - qub @ mu_b)
    # Var(beta) = S^-1; eq:var:1's second term with Q_uu^-1 Q_ubeta = W
    var_b = np.linalg.inv(S) if nb else np.zeros((0, 0))
    var_u_add = np.einsum("ij,jk,ik->i", W, var_b, W) if nb else np.zeros(n)
    return dict(mu_u=mu_u, mu_beta=mu_b, var_beta=var_b, var_u_add=var_u_add,
                solves=nb + 2)
