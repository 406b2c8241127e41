"""Pins of the oracle's overlap probe (the n_l choice of Sec. 3.2.2 from one
covariance column, the probing Sec. 5 proposes), on the CPU.

Without observations the posterior is the prior Q_t (x) Q_s, whose covariance
column factorizes: along time it is the unit-variance AR(1) correlation
rho^|t - t_c| (Q_t^-1 = [rho^|i-j|]); within the centre's step it is the
column of Q_s^-1, known in closed form in the DCT-II eigenbasis of the
Neumann grid Laplacian (Q_s = tau (kappa^2 h^2 + l_a + l_b)^2 / h^2 in that
basis, eq:spde:4 with alpha = 2 and C = h^2 I).  With observations the
column is checked against a dense inverse."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2309_05435_amd.inputs import obs_mask


def neumann_eig(m):
    a = np.arange(m)
    lam = 2.0 - 2.0 * np.cos(np.pi * a / m)
    U = np.cos(np.pi * np.outer(np.arange(m) + 0.5, a) / m)
    U /= np.linalg.norm(U, axis=0)
    return lam, U


def lag_of(dist, ratio, eps):
    big = np.abs(ratio) > eps
    return 1 + (int(np.max(dist[big])) if big.any() else 0)


@pytest.mark.parametrize("mx,my,T,rho,range_,eps", [(14, 12, 21, 0.8, 0.3, 1e-2),
                                                    (16, 16, 9, 0.5, 0.15, 1e-3),
                                                    (10, 13, 30, 0.9, 0.5, 5e-2)])
def test_probe_without_observations_is_ar1_times_spatial_closed_form(mx, my, T, rho, range_,
                                                                      eps):
    h = 1.0 / (max(mx, my) - 1)
    kappa = math.sqrt(8) / range_
    log_tau = 0.4
    M = O.OracleModel(mx, my, T, h, math.log(kappa), log_tau, rho, 0.0,
                      np.zeros(mx * my * T, np.uint8))
    lags, ct, cs = O.probe_overlap(M, eps)
    tc, cx, cy = T // 2, mx // 2, my // 2
    dt = np.abs(np.arange(T) - tc)
    np.testing.assert_allclose(ct, rho ** dt, rtol=1e-9, atol=1e-12)
    lx, Ux = neumann_eig(mx)
    ly, Uy = neumann_eig(my)
    w = 1.0 / (kappa ** 2 * h ** 2 + lx[None, :] + ly[:, None]) ** 2  # [b (y), a (x)]
    col = np.einsum("xa,yb,ba->yx", Ux * Ux[cx][None, :], Uy * Uy[cy][None, :], w).reshape(-1)
    expect = col / col[cy * mx + cx]
    np.testing.assert_allclose(cs, expect, rtol=1e-8, atol=1e-11)
    iy, ix = np.divmod(np.arange(mx * my), mx)
    dist = np.abs(ix - cx) + np.abs(iy - cy)
    assert lags[0] == lag_of(dt, rho ** dt, eps)
    assert lags[1] == lag_of(dist, expect, eps)
    assert lags[2] == max(lags[0], (lags[1] + 1) // 2)


def test_probe_with_observations_matches_dense_inverse():
    mx, my, T = 8, 7, 6
    n = mx * my * T
    M = O.OracleModel(mx, my, T, 1.0 / 7, 1.9, 0.2, 0.85, -0.3, obs_mask(n, 0.4, 5))
    lags, ct, cs = O.probe_overlap(M, 1e-2)
    Sig = np.linalg.inv(M.csr(O.Q).dense())
    ns = mx * my
    c = (T // 2) * ns + (my // 2) * mx + mx // 2
    r = Sig[:, c] / Sig[c, c]
    np.testing.assert_allclose(ct, r[np.arange(T) * ns + (my // 2) * mx + mx // 2], rtol=1e-9,
                               atol=1e-12)
    np.testing.assert_allclose(cs, r[(T // 2) * ns:(T // 2 + 1) * ns], rtol=1e-9, atol=1e-12)


def test_probe_lags_grow_as_eps_shrinks():
    M = O.OracleModel(12, 12, 16, 1.0 / 11, 2.2, 0.0, 0.9, 0.0, obs_mask(12 * 12 * 16, 0.3, 9))
    prev = None
    for eps in (0.3, 0.1, 1e-2, 1e-3, 1e-4):
        lags, _, _ = O.probe_overlap(M, eps)
        if prev is not None:
            assert (lags >= prev).all()
        prev = lags
