"""Conditioning of the subdomain matrices Q_AA of a workload, and the parity
bars derived from it (test infrastructure).

Each Omega_p* is a product set T_A x R: n_l hops of Q's graph move at most
n_l time steps and, at the same time, n_l hops of the 13-point spatial
stencil.  Hence Q_AA = (Q_t)_{T_A} (x) (Q_s)_R + D_A with D_A >= 0
diagonal.  The eigenvalues of a Kronecker product of two SPD matrices are
the products of theirs, and adding D_A raises every eigenvalue by at most
max D = sigma^-2 (Weyl), so
    lambda_min(Q_AA) >= lambda_min((Q_t)_{T_A}) lambda_min((Q_s)_R),
    lambda_max(Q_AA) <= lambda_max((Q_t)_{T_A}) lambda_max((Q_s)_R) + sigma^-2,
and their ratio bounds cond_2(Q_AA) from above.  The extremes of the two
small factors are computed exactly: dense eigvalsh for the T_A x T_A time
factor, Lanczos (with shift-invert for the smallest) for the spatial one,
a principal submatrix of the global Q_s.

Bars.  Two backward-stable FP64 evaluations of the same entry of Q_AA^-1
(the library's factor and selected inverse, the oracle's Cholesky, sparse LU
or CG) carry relative errors of order u cond(Q_AA) each (u = 2^-53: the
usual digits-lost rule for a backward-stable inverse, a first-order
estimate, not a worst-case bound); the bar is BAR_C u max_p cond(Q_AA) with
BAR_C = 8.
"""
from __future__ import annotations

import numpy as np

import oracle as O

U64 = 2.0 ** -53
BAR_C = 8.0


def _piece(idx, length, parts):
    base, extra = divmod(length, parts)
    return idx * base + min(idx, extra), base + (1 if idx < extra else 0)


def _axis_key(start, length, m, reach):
    # the principal submatrix of Q_s on R depends on how far the box sits from
    # the domain edges only up to the reach of the grown region plus the stencil
    return min(start, reach), length, min(m - start - length, reach)


_CACHE: dict = {}


def cond_bound(wl) -> dict:
    """{'K': max_p bound on cond(Q_AA), 'parts': [(tile key, slab, |R|, T_A,
    lmin_s, lmax_s, lmin_t, lmax_t, K)]} over every subdomain shape of wl."""
    if repr(wl) not in _CACHE:
        _CACHE[repr(wl)] = _cond_bound(wl)
    return _CACHE[repr(wl)]


def _cond_bound(wl) -> dict:
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    lk, lt, rho, ls = wl.theta
    m, T = wl.m, wl.T
    Ms = O.OracleModel(m, m, 1, wl.h, lk, lt, rho, ls, np.zeros(m * m, np.uint8))
    c = Ms.csr(O.QS)
    Qs = sp.csr_matrix((c.v, c.ci, c.rp), shape=(c.nr, c.nc))
    Qt = O.OracleModel(1, 1, T, wl.h, lk, lt, rho, ls, np.zeros(T, np.uint8)).csr(O.QT).dense()
    reach = 2 * wl.n_l + 3
    spatial = {}
    for tx in range(wl.n_tiles):
        for ty in range(wl.n_tiles):
            x0, xl = _piece(tx, m, wl.n_tiles)
            y0, yl = _piece(ty, m, wl.n_tiles)
            kx, ky = _axis_key(x0, xl, m, reach), _axis_key(y0, yl, m, reach)
            key = min((kx, ky), (ky, kx))
            if key in spatial:
                continue
            g = np.arange(m * m)
            yy, xx = divmod(g, m)
            lab = np.ones(m * m, np.int32)
            lab[(xx >= x0) & (xx < x0 + xl) & (yy >= y0) & (yy < y0 + yl)] = 0
            st = Ms.subdomain_state(lab, 0, wl.n_l)
            R = np.flatnonzero((st == 1) | (st == 2))
            QR = sp.csc_matrix(Qs[R][:, R])
            if len(R) <= 400:
                ev = np.linalg.eigvalsh(QR.toarray())
                lo, hi = ev[0], ev[-1]
            else:
                hi = spla.eigsh(QR, k=1, which="LA", return_eigenvectors=False)[0]
                lo = spla.eigsh(QR, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
            spatial[key] = (len(R), float(lo), float(hi))
    parts, K = [], 0.0
    for slab in range(wl.n_tslabs):
        a, ln = _piece(slab, T, wl.n_tslabs)
        ta = np.arange(max(0, a - wl.n_l), min(T, a + ln + wl.n_l))
        ev = np.linalg.eigvalsh(Qt[np.ix_(ta, ta)])
        for key, (nr, lo, hi) in spatial.items():
            k = (ev[-1] * hi + np.exp(-2.0 * ls)) / (ev[0] * lo)
            parts.append((key, slab, nr, len(ta), lo, hi, float(ev[0]), float(ev[-1]), float(k)))
            K = max(K, float(k))
    return {"K": K, "parts": parts}


def parity_bar(wl) -> float:
    """Relative parity bar of diagonal entries: BAR_C u max_p cond(Q_AA)."""
    return BAR_C * U64 * cond_bound(wl)["K"]
