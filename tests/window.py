"""Oracle values at sizes where the whole oracle model is too large to build.

The estimator at node i of core p reads Q only through Q_AA and Q_AB, with
A = Omega_p* (the core grown by n_l hops of the graph of Q) and B = S_p (one
more hop).  One hop of Q moves at most one time step and at most two grid
steps in L1 distance (the 13-point stencil of Q_s), and an entry Q_jk is
fixed by the degrees of j and k in the grid graph and by the AR(1) row of its
time steps.  A window of the space-time grid that contains A and S with a
margin of two grid steps and one time step - built with the global h, theta
and observation mask - therefore has the same Q_AA and Q_AB, hence the same
(deterministic part, estimate) at node i.  Where the window reaches the
domain boundary it stops there, so boundary rows are the true ones.

The same holds for a row of Q x: a window with a margin of three grid steps
and one time step around the node gives that row exactly.
"""
from __future__ import annotations

import numpy as np

import oracle as O


def piece(idx: int, length: int, parts: int) -> tuple[int, int]:
    """(start, len) of piece idx when length is split into parts; the first
    (length mod parts) pieces get one extra element."""
    base, extra = divmod(length, parts)
    start = idx * base + min(idx, extra)
    return start, base + (1 if idx < extra else 0)


def core_box(wl, p: int):
    """((t0, t1), (x0, x1), (y0, y1)) half-open ranges of core p."""
    ntx = nty = wl.n_tiles
    tx = p % ntx
    ty = (p // ntx) % nty
    slab = p // (ntx * nty)
    t0, tl = piece(slab, wl.T, wl.n_tslabs)
    x0, xl = piece(tx, wl.m, ntx)
    y0, yl = piece(ty, wl.m, nty)
    return (t0, t0 + tl), (x0, x0 + xl), (y0, y0 + yl)


class Window:
    """A sub-grid [t0,t1) x [x0,x1) x [y0,y1) of a workload with its oracle model."""

    def __init__(self, wl, mask, tr, xr, yr):
        self.wl = wl
        self.t0, self.t1 = tr
        self.x0, self.x1 = xr
        self.y0, self.y1 = yr
        self.wt, self.wx, self.wy = self.t1 - self.t0, self.x1 - self.x0, self.y1 - self.y0
        tt, yy, xx = np.meshgrid(np.arange(self.t0, self.t1), np.arange(self.y0, self.y1),
                                 np.arange(self.x0, self.x1), indexing="ij")
        self.glob = (tt * wl.m * wl.m + yy * wl.m + xx).ravel()  # window order -> global id
        self.M = O.OracleModel(self.wx, self.wy, self.wt, wl.h, *wl.theta, mask[self.glob])

    def local(self, i: int) -> int:
        t, r = divmod(i, self.wl.m * self.wl.m)
        y, x = divmod(r, self.wl.m)
        return ((t - self.t0) * self.wy + (y - self.y0)) * self.wx + (x - self.x0)


def _clip(lo, hi, n):
    return max(0, lo), min(n, hi)


def core_window(wl, mask, p: int) -> Window:
    (t0, t1), (x0, x1), (y0, y1) = core_box(wl, p)
    ms = 2 * (wl.n_l + 1) + 2      # grid steps: Omega*, separator, margin
    mt = (wl.n_l + 1) + 1          # time steps
    return Window(wl, mask, _clip(t0 - mt, t1 + mt, wl.T), _clip(x0 - ms, x1 + ms, wl.m),
                  _clip(y0 - ms, y1 + ms, wl.m))


def estimator_entries(wl, mask, p: int, nodes, x: np.ndarray):
    """[(det, diag)] of the estimator at global nodes of core p (x: (n_k, n)
    samples): Omega_p* and S_p by the oracle's graph growth on the window
    model, then y = Q_AA^-1 e_i by a sparse direct solve (SuperLU) of the
    window's Q_AA, det = y_i, mu_k = y^T Q_AB x_B, diag = det + mean mu_k^2."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    w = core_window(wl, mask, p)
    (t0, t1), (x0, x1), (y0, y1) = core_box(wl, p)
    labels = np.ones(w.M.n, np.int32)
    tt, yy, xx = np.meshgrid(np.arange(w.t0, w.t1), np.arange(w.y0, w.y1),
                             np.arange(w.x0, w.x1), indexing="ij")
    inside = ((tt >= t0) & (tt < t1) & (yy >= y0) & (yy < y1) & (xx >= x0) & (xx < x1)).ravel()
    labels[inside] = 0
    state = w.M.subdomain_state(labels, 0, wl.n_l)
    A = np.flatnonzero((state == 1) | (state == 2))
    Bn = np.flatnonzero(state == 3)
    c = w.M.csr(O.Q)
    Q = sp.csr_matrix((c.v, c.ci, c.rp), shape=(c.nr, c.nc))
    lu = spla.splu(sp.csc_matrix(Q[A][:, A]))
    QAB = Q[A][:, Bn]
    xB = x[:, w.glob[Bn]]                      # (n_k, |B|)
    pos = {g: k for k, g in enumerate(A)}
    out = []
    for i in nodes:
        e = np.zeros(len(A))
        e[pos[w.local(i)]] = 1.0
        y = lu.solve(e)
        det = y[pos[w.local(i)]]
        mu = (QAB.T @ y) @ xB.T                # (n_k,)
        out.append((det, det + (np.mean(mu ** 2) if len(mu) else 0.0)))
    return out


# unit roundoff of FP64 and the constant of the per-entry bounds below
U64 = 2.0 ** -53
C_BOUND = 64.0


def estimator_entries_bounded(wl, mask, p: int, nodes, x: np.ndarray):
    """As estimator_entries, with a bound on the rounding error that any
    backward-stable FP64 evaluation of each value may carry, derived from the
    conditioning of Q_AA along e_i: a solve with (Q_AA + dQ) y~ = e_i,
    ||dQ|| <= c u ||Q_AA||, changes y_i by about y^T dQ y, so
      |d det| <= c u ||Q_AA|| ||y||^2,
    and mu_k = y^T r_k (r_k = Q_AB x_B) by about c u ||Q_AA|| ||y|| ||m_k||
    with m_k = Q_AA^-1 r_k, so the Monte Carlo term (1/n_k) sum mu_k^2 moves by
    at most (1/n_k) sum 2 |mu_k| c u ||Q_AA|| ||y|| ||m_k||.  ||Q_AA|| is taken
    as the largest absolute row sum (>= the 2-norm of a symmetric matrix) and
    c = 64.  Returns [(det, full, bound_det, bound_full)]; the parity bar for
    two such evaluations is the sum of their bounds, 2 x bound."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    w = core_window(wl, mask, p)
    (t0, t1), (x0, x1), (y0, y1) = core_box(wl, p)
    labels = np.ones(w.M.n, np.int32)
    tt, yy, xx = np.meshgrid(np.arange(w.t0, w.t1), np.arange(w.y0, w.y1),
                             np.arange(w.x0, w.x1), indexing="ij")
    inside = ((tt >= t0) & (tt < t1) & (yy >= y0) & (yy < y1) & (xx >= x0) & (xx < x1)).ravel()
    labels[inside] = 0
    state = w.M.subdomain_state(labels, 0, wl.n_l)
    A = np.flatnonzero((state == 1) | (state == 2))
    Bn = np.flatnonzero(state == 3)
    c = w.M.csr(O.Q)
    Q = sp.csr_matrix((c.v, c.ci, c.rp), shape=(c.nr, c.nc))
    QAA = Q[A][:, A]
    norm = float(abs(QAA).sum(axis=1).max())
    lu = spla.splu(sp.csc_matrix(QAA))
    QAB = Q[A][:, Bn]
    xB = x[:, w.glob[Bn]]                      # (n_k, |B|)
    R = np.asarray(QAB @ xB.T)                 # (|A|, n_k): r_k
    Mk = lu.solve(R)                           # m_k = Q_AA^-1 r_k
    mnorm = np.linalg.norm(Mk, axis=0)
    pos = {g: k for k, g in enumerate(A)}
    out = []
    for i in nodes:
        e = np.zeros(len(A))
        e[pos[w.local(i)]] = 1.0
        y = lu.solve(e)
        det = y[pos[w.local(i)]]
        mu = y @ R                             # (n_k,)
        ynorm = float(np.linalg.norm(y))
        bdet = C_BOUND * U64 * norm * ynorm ** 2
        bmc = (np.mean(2.0 * np.abs(mu) * C_BOUND * U64 * norm * ynorm * mnorm)
               if len(mu) else 0.0)
        full = det + (np.mean(mu ** 2) if len(mu) else 0.0)
        out.append((float(det), float(full), float(bdet), float(bdet + bmc)))
    return out


def estimator_entry(wl, mask, p: int, i: int, x: np.ndarray):
    return estimator_entries(wl, mask, p, [i], x)[0]


def q_row(wl, mask, which: int, i: int, x: np.ndarray) -> np.ndarray:
    """Row i of (operator `which`) @ x for each column of x ((n_k, n))."""
    t, r = divmod(i, wl.m * wl.m)
    y, xg = divmod(r, wl.m)
    w = Window(wl, mask, _clip(t - 1, t + 2, wl.T), _clip(xg - 3, xg + 4, wl.m),
               _clip(y - 3, y + 4, wl.m))
    xw = np.ascontiguousarray(x[:, w.glob])
    return w.M.apply(which, xw)[:, w.local(i)]
