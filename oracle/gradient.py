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


def _joint(M, a_beta, q_beta):
    """The joint posterior precision of x = (u, beta) (eq:mean:3, first line)
    and A = [A_u A_beta], dense (small models)."""
    tau_y = math.exp(-2.0 * M.theta[3])
    obs = np.flatnonzero(M.mask)
    a = np.asarray(a_beta, np.float64).reshape(len(q_beta), len(obs)).T
    n, nb = M.n, a.shape[1]
    Au = np.zeros((len(obs), n))
    Au[np.arange(len(obs)), obs] = 1.0
    A = np.hstack([Au, a])
    Qx = np.zeros((n + nb, n + nb))
    Qx[:n, :n] = np.kron(M.csr(_QT).dense(), M.csr(_QS).dense())
    Qx[n:, n:] = np.diag(np.asarray(q_beta, np.float64))
    return Qx, A, tau_y


def log_posterior_fixed(M, y, a_beta, q_beta) -> float:
    """log pi(theta | y) with fixed effects (eq:hyperpar:1 at x = mu, dense):
    1/2 log|Q_y| + 1/2 log|Q_x| - 1/2 log|Q| - 1/2 r^T Q_y r - 1/2 mu^T Q_x mu,
    Q = Q_x + A^T Q_y A over x = (u, beta), mu = Q^-1 A^T Q_y y, r = y - A mu."""
    Qx, A, tau_y = _joint(M, a_beta, q_beta)
    y = np.asarray(y, np.float64)
    Q = Qx + tau_y * A.T @ A
    mu = np.linalg.solve(Q, tau_y * A.T @ y)
    r = y - A @ mu
    return (0.5 * len(y) * math.log(tau_y) + 0.5 * np.linalg.slogdet(Qx)[1]
            - 0.5 * np.linalg.slogdet(Q)[1] - 0.5 * tau_y * float(r @ r) - 0.5 * float(mu @ Qx @ mu))


def gradient_fixed(M, y, a_beta, q_beta, traces) -> dict:
    """d_j log pi(theta | y) with fixed effects, eq:hyperpar:3 for log|Q|:
    tr(Q_uu^-1 d_j Q_uu) (the given traces) + tr(S^-1 d_j S), with the Schur
    complement S = Q_bb - Q_bu W, W = Q_uu^-1 Q_ub, and
    d_j S = d_j Q_bb - (d_j Q_bu) W - W^T (d_j Q_ub) + W^T (d_j Q_uu) W
    (Q_ub = tau_y A_u^T A_beta, Q_bb = Q_beta + tau_y A_beta^T A_beta: their
    derivatives come from tau_y = exp(-2 log sigma) only).  The quadratic
    terms are those of the model without fixed effects at the joint mean
    (Q_beta does not depend on theta).  Returns dict(grad, terms (4 x 6: the
    five terms of gradient() and -1/2 tr(S^-1 d_j S)), mu_u, mu_beta)."""
    from .mean import blocks
    obs, tau_y, a, quu, qub, qbb = blocks(M, a_beta, q_beta)
    n_obs, nb = len(obs), a.shape[1]
    pm = posterior_mean(M, y, a_beta, q_beta)
    mu_u, mu_b = pm["mu_u"], pm["mu_beta"]
    r = np.asarray(y, np.float64) - mu_u[obs] - a @ mu_b
    W = spla.splu(quu).solve(qub) if nb else np.zeros((M.n, 0))
    S = qbb - qub.T @ W
    S_inv = np.linalg.inv(S) if nb else np.zeros((0, 0))
    Qu = np.kron(M.csr(_QT).dense(), M.csr(_QS).dense())
    Qu_inv = np.linalg.inv(Qu)
    terms = np.zeros((4, 6))
    for j in range(4):
        dQu = M.csr(_DQ[j]).dense() if j < 3 else np.zeros_like(Qu)
        dtau = -2.0 * tau_y if j == 3 else 0.0       # d_j tau_y
        dQuu = M.csr(_DQ[j] if j < 3 else 4).dense()  # d_j Q_uu = d_j Q
        dQub = (dtau / tau_y) * qub
        dQbb = dtau * (a.T @ a)
        dS = dQbb - dQub.T @ W - W.T @ dQub + W.T @ dQuu @ W
        terms[j] = [-float(n_obs) if j == 3 else 0.0,
                    0.5 * float(np.sum(Qu_inv * dQu)),
                    -0.5 * float(traces[j]),
                    -0.5 * dtau * float(r @ r),
                    -0.5 * float(mu_u @ (dQu @ mu_u)),
                    -0.5 * float(np.sum(S_inv * dS.T)) if nb else 0.0]
    return dict(grad=terms.sum(axis=1), terms=terms, mu_u=mu_u, mu_beta=mu_b)


def alg6(make_model, theta0, y, a_beta, q_beta, grad_fn, steps=50, h=1e-4, max_step=0.5,
         tol=1e-8, active=(True, True, True, True)):
    """The iteration of Alg. 6 / eq:hyperpar:2, theta <- theta - rho H^-1 g,
    with g the gradient and H the diagonal of second derivatives taken from
    two first derivatives per component, (g_j(theta + h e_j) - g_j(theta -
    h e_j)) / 2h, of the gradient without its stochastic part (grad_fn is
    called with deterministic=True for those).  rho = 1; a component whose
    second derivative is not negative takes a gradient-ascent step instead,
    and every component's step is capped at max_step (the paper leaves both
    choices open).  Components outside `active` stay at their start value.
    make_model(theta) builds the oracle model.  Returns the iterates (steps + 1
    rows at most)."""
    th = np.array(theta0, np.float64)
    act = np.asarray(active, bool)
    path = [th.copy()]
    for _ in range(steps):
        g = grad_fn(make_model(th), y, a_beta, q_beta, deterministic=False)
        H = np.full(4, -1.0)
        for j in np.flatnonzero(act):
            tp, tm = th.copy(), th.copy()
            tp[j] += h
            tm[j] -= h
            H[j] = (grad_fn(make_model(tp), y, a_beta, q_beta, deterministic=True)[j]
                    - grad_fn(make_model(tm), y, a_beta, q_beta, deterministic=True)[j]) / (2 * h)
        step = np.where(H < 0, -g / np.where(H < 0, H, 1.0), g)
        step = np.where(act, np.clip(step, -max_step, max_step), 0.0)
        th = th + step
        path.append(th.copy())
        if np.abs(step).max() < tol:
            break
    return np.array(path)
