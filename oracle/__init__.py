"""ctypes binding of the plain FP64 CPU oracle (``rbmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the benchmark's CPU-baseline leg; never by the product path.

The oracle follows the paper (arXiv 2309.05435) literally: explicit CSR
assembly of Q = Q_t (x) Q_s + A^T Q_y A (Sec. 2.1-2.3), overlap growth by
breadth-first search and the per-core estimator of Alg. 4 (diagonal) and of
Alg. 3 + eq:hyperpar:4 (traces), with Q_AA^-1 entries from a banded Cholesky
factor (the plain definition of the inverse).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C")
        lp = np.ctypeslib.ndpointer(np.int64, flags="C")
        up = np.ctypeslib.ndpointer(np.uint8, flags="C")
        L.orc_model_create.restype = P
        L.orc_model_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                       C.c_double, C.c_double, C.c_double, up]
        L.orc_model_destroy.argtypes = [P]
        L.orc_model_csr_dims.argtypes = [P, C.c_int, lp]
        L.orc_model_csr.argtypes = [P, C.c_int, lp, ip, dp]
        L.orc_grid_cores.argtypes = [C.c_int] * 6 + [ip]
        L.orc_subdomain_state.argtypes = [P, ip, C.c_int, C.c_int, up]
        L.orc_csr_subdomain_state.argtypes = [C.c_int, lp, ip, dp, ip, C.c_int, C.c_int, up]
        L.orc_csr_logdet.argtypes = [C.c_int, lp, ip, dp, C.POINTER(C.c_double)]
        L.orc_model_sample.argtypes = [P, C.c_int, dp, dp]
        L.orc_model_rhs.argtypes = [P, C.c_int, dp, dp]
        L.orc_model_rbmc.argtypes = [P, ip, C.c_int, C.c_int, C.c_int, dp, C.c_uint, dp, dp, dp,
                                     dp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.orc_csr_rbmc.argtypes = [C.c_int, lp, ip, dp, C.c_int, C.c_void_p, C.c_void_p,
                                   C.c_void_p, ip, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp,
                                   C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.orc_model_cg.argtypes = [P, C.c_void_p, dp, dp, C.c_double, C.c_int]
        L.orc_model_entry.argtypes = [P, ip, C.c_int, C.c_int, C.c_int, C.c_int, dp, C.c_double,
                                      C.c_int, dp]
        L.orc_model_apply.argtypes = [P, C.c_int, C.c_int, dp, dp]
        L.orc_model_nobs.argtypes = [P]
        _lib = L
    return _lib


# CSR selectors of OracleModel.csr()
Q, DQ_LOGKAPPA, DQ_LOGTAU, DQ_RHO, DQ_LOGSIGMA, F, QS, QT, G = range(9)


class CSR:
    def __init__(self, nr, nc, rp, ci, v):
        self.nr, self.nc, self.rp, self.ci, self.v = nr, nc, rp, ci, v

    def dense(self) -> np.ndarray:
        out = np.zeros((self.nr, self.nc))
        for r in range(self.nr):
            out[r, self.ci[self.rp[r]:self.rp[r + 1]]] += self.v[self.rp[r]:self.rp[r + 1]]
        return out

    def matvec(self, x: np.ndarray) -> np.ndarray:
        rows = np.repeat(np.arange(self.nr), np.diff(self.rp))
        return np.bincount(rows, weights=self.v * x[self.ci], minlength=self.nr)

    @staticmethod
    def from_dense(a: np.ndarray) -> "CSR":
        nr, nc = a.shape
        rp = np.zeros(nr + 1, np.int64)
        ci, v = [], []
        for r in range(nr):
            nz = np.nonzero(a[r])[0]
            ci.extend(nz.tolist())
            v.extend(a[r, nz].tolist())
            rp[r + 1] = rp[r] + len(nz)
        return CSR(nr, nc, rp, np.asarray(ci, np.int32), np.asarray(v, np.float64))


def grid_cores(mx, my, T, n_tslabs, n_tiles_x, n_tiles_y) -> np.ndarray:
    lab = np.zeros(mx * my * T, np.int32)
    lib().orc_grid_cores(mx, my, T, n_tslabs, n_tiles_x, n_tiles_y, lab)
    return lab


class OracleModel:
    """Q(theta) = Q_t (x) Q_s + A^T Q_y A on an mx x my grid with T steps."""

    def __init__(self, mx, my, T, h, log_kappa, log_tau, rho, log_sigma, mask):
        self.mx, self.my, self.T = mx, my, T
        self.theta = (log_kappa, log_tau, rho, log_sigma)
        self.n = mx * my * T
        self.mask = np.ascontiguousarray(mask, np.uint8)
        assert self.mask.shape == (self.n,)
        self._h = lib().orc_model_create(mx, my, T, h, log_kappa, log_tau, rho, log_sigma,
                                         self.mask)
        self.n_obs = lib().orc_model_nobs(self._h)

    @classmethod
    def from_workload(cls, wl, mask=None, theta=None):
        th = wl.theta if theta is None else theta
        return cls(wl.m, wl.m, wl.T, wl.h, *th, wl.mask() if mask is None else mask)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_model_destroy(self._h)
            self._h = None

    def csr(self, which: int) -> CSR:
        d = np.zeros(3, np.int64)
        lib().orc_model_csr_dims(self._h, which, d)
        rp = np.zeros(d[0] + 1, np.int64)
        ci = np.zeros(max(d[2], 1), np.int32)
        v = np.zeros(max(d[2], 1), np.float64)
        lib().orc_model_csr(self._h, which, rp, ci, v)
        return CSR(int(d[0]), int(d[1]), rp, ci[:d[2]], v[:d[2]])

    def sample(self, z: np.ndarray) -> np.ndarray:
        """Exact x = Q^-1 F z for each row of z (n_k x (n + n_obs))."""
        z = np.ascontiguousarray(z, np.float64)
        n_k = z.shape[0]
        assert z.shape[1] == self.n + self.n_obs
        x = np.zeros((n_k, self.n))
        info = lib().orc_model_sample(self._h, n_k, z, x)
        if info != 0:
            raise RuntimeError(f"oracle Cholesky breakdown at row {-info - 1}")
        return x

    def rhs(self, z: np.ndarray) -> np.ndarray:
        z = np.ascontiguousarray(z, np.float64)
        b = np.zeros((z.shape[0], self.n))
        lib().orc_model_rhs(self._h, z.shape[0], z, b)
        return b

    def apply(self, which: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
        c = self.csr(which)
        y = np.zeros((x.shape[0], c.nr))
        lib().orc_model_apply(self._h, which, x.shape[0], x, y)
        return y

    def subdomain_state(self, labels: np.ndarray, p: int, n_l: int) -> np.ndarray:
        st = np.zeros(self.n, np.uint8)
        lib().orc_subdomain_state(self._h, np.ascontiguousarray(labels, np.int32), p, n_l, st)
        return st

    def rbmc(self, labels, n_parts, n_l, x, grad_mask=0b111):
        """Returns dict(diag, diag_det, trace, trace_det, err_est)."""
        x = np.ascontiguousarray(np.atleast_2d(x), np.float64) if x is not None and len(x) else \
            np.zeros((0, self.n))
        n_k = x.shape[0]
        nd = bin(grad_mask).count("1")
        diag = np.zeros(self.n)
        diag_det = np.zeros(self.n)
        tr = np.zeros(max(nd, 1))
        trd = np.zeros(max(nd, 1))
        err = C.c_double(0)
        fail = C.c_int(-1)
        xx = x if n_k else np.zeros((1, self.n))
        st = lib().orc_model_rbmc(self._h, np.ascontiguousarray(labels, np.int32), n_parts, n_l,
                                  n_k, xx, grad_mask, diag, diag_det, tr, trd, C.byref(err),
                                  C.byref(fail))
        if st != 0:
            raise RuntimeError(f"oracle: Q_AA not SPD in part {fail.value}")
        return dict(diag=diag, diag_det=diag_det, trace=tr[:nd], trace_det=trd[:nd],
                    err_est=err.value)

    def cg(self, b, sel=None, rtol=1e-13, maxit=100000):
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros(self.n)
        s = None if sel is None else np.ascontiguousarray(sel, np.uint8)
        it = lib().orc_model_cg(self._h, None if s is None else s.ctypes.data, b, x, rtol, maxit)
        return x, it

    def entry(self, labels, p, n_l, i, x, rtol=1e-13, maxit=100000):
        """(det, diag) of the estimator at node i of core p, by CG on Q_AA."""
        x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
        out = np.zeros(2)
        it = lib().orc_model_entry(self._h, np.ascontiguousarray(labels, np.int32), p, n_l, i,
                                   x.shape[0], x, rtol, maxit, out)
        if it < 0:
            raise RuntimeError("oracle CG did not converge")
        return out[0], out[1]


def csr_rbmc(A: CSR, dQs, labels, n_parts, n_l, x):
    """Generic estimator on an explicit SPD matrix (e.g. the paper's AR(1) example)."""
    x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
    n = A.nr
    nd = len(dQs)
    keep = []
    rps = (C.c_void_p * max(nd, 1))()
    cis = (C.c_void_p * max(nd, 1))()
    vs = (C.c_void_p * max(nd, 1))()
    for j, d in enumerate(dQs):
        a, b, c = (np.ascontiguousarray(d.rp, np.int64), np.ascontiguousarray(d.ci, np.int32),
                   np.ascontiguousarray(d.v, np.float64))
        keep += [a, b, c]
        rps[j], cis[j], vs[j] = a.ctypes.data, b.ctypes.data, c.ctypes.data
    diag = np.zeros(n)
    diag_det = np.zeros(n)
    tr = np.zeros(max(nd, 1))
    trd = np.zeros(max(nd, 1))
    err = C.c_double(0)
    fail = C.c_int(-1)
    st = lib().orc_csr_rbmc(n, np.ascontiguousarray(A.rp, np.int64),
                            np.ascontiguousarray(A.ci, np.int32),
                            np.ascontiguousarray(A.v, np.float64), nd, C.cast(rps, C.c_void_p),
                            C.cast(cis, C.c_void_p), C.cast(vs, C.c_void_p),
                            np.ascontiguousarray(labels, np.int32), n_parts, n_l, x.shape[0], x,
                            diag, diag_det, tr, trd, C.byref(err), C.byref(fail))
    if st != 0:
        raise RuntimeError(f"oracle: Q_AA not SPD in part {fail.value}")
    return dict(diag=diag, diag_det=diag_det, trace=tr[:nd], trace_det=trd[:nd], err_est=err.value)


def csr_state(A: CSR, labels, p, n_l) -> np.ndarray:
    st = np.zeros(A.nr, np.uint8)
    lib().orc_csr_subdomain_state(A.nr, np.ascontiguousarray(A.rp, np.int64),
                                  np.ascontiguousarray(A.ci, np.int32),
                                  np.ascontiguousarray(A.v, np.float64),
                                  np.ascontiguousarray(labels, np.int32), p, n_l, st)
    return st


def csr_logdet(A: CSR) -> float:
    out = C.c_double(0)
    info = lib().orc_csr_logdet(A.nr, np.ascontiguousarray(A.rp, np.int64),
                                np.ascontiguousarray(A.ci, np.int32),
                                np.ascontiguousarray(A.v, np.float64), C.byref(out))
    if info != 0:
        raise RuntimeError("oracle: matrix not SPD")
    return out.value


def probe_overlap(M: OracleModel, eps: float, rtol: float = 1e-13):
    """The overlap choice of Sec. 3.2.2 (n_l = the lag at which the correlation
    falls to about zero, separately in time and space) from one covariance
    column, as Sec. 5 proposes probing the posterior range.

    y = Q^-1 e_c at the centre node c = (T // 2, my // 2, mx // 2), by the
    oracle's conjugate gradients on the whole Q.  Ratios y_j / y_c:
      time:  at (t, my // 2, mx // 2) for every step t;
      space: at every node of step T // 2.
    lag = the smallest distance d >= 1 (steps; L1 grid distance) such that
    every ratio at distance >= d has magnitude <= eps.  Suggested hops:
    max(time lag, ceil(space lag / 2)), one hop of Q's graph covering one step
    and up to two grid steps.  Returns (lags, corr_time, corr_space)."""
    mx, my, T = M.mx, M.my, M.T
    ns = mx * my
    tc, cx, cy = T // 2, mx // 2, my // 2
    c = tc * ns + cy * mx + cx
    e = np.zeros(M.n)
    e[c] = 1.0
    y, _ = M.cg(e, rtol=rtol)
    r = y / y[c]
    corr_time = r[np.arange(T) * ns + cy * mx + cx]
    corr_space = r[tc * ns:(tc + 1) * ns].copy()
    dt = np.abs(np.arange(T) - tc)
    lag_t = 1 + max([int(d) for d, v in zip(dt, corr_time) if abs(v) > eps], default=0)
    iy, ix = np.divmod(np.arange(ns), mx)
    dist = np.abs(ix - cx) + np.abs(iy - cy)
    big = np.abs(corr_space) > eps
    lag_s = 1 + (int(dist[big].max()) if big.any() else 0)
    return np.array([lag_t, lag_s, max(lag_t, (lag_s + 1) // 2)]), corr_time, corr_space


def alg2(M: OracleModel, labels, n_parts, x):
    """The non-overlapping estimator (Alg. 2): cores Omega_p (labels >= 0)
    separated by S (label -1).  Core nodes: (Q_pp^-1)_ii plus the Monte
    Carlo variance of Q_pp^-1 Q_pS x_S (the overlapping estimator with n_l = 0,
    whose S_p = N(Omega_p) lies in S); separator nodes: Var(x_S)_i from the
    zero-mean samples, (1/n_k) sum_k x_k[i]^2.  Returns the diagonal."""
    x = np.ascontiguousarray(np.atleast_2d(x), np.float64) if x is not None and len(x) else \
        np.zeros((0, M.n))
    d = M.rbmc(labels, n_parts, 0, x, grad_mask=0)["diag"].copy()
    sep = np.asarray(labels) < 0
    d[sep] = (x[:, sep] ** 2).mean(axis=0) if x.shape[0] else 0.0
    return d
