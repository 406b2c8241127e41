"""Thin ctypes binding of librbmc.so (the C ABI declared in include/rbmc.h).

Argument marshalling only: every step of the estimator runs in the HIP
library.  PyTorch provides device memory and the HIP stream.  Loading fails
loudly when the built library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbmc.so")

RBMC_OK, RBMC_W_NOT_CONVERGED = 0, 1
RBMC_E_ARG, RBMC_E_NOT_SPD, RBMC_E_OOM, RBMC_E_DEVICE, RBMC_E_UNSUPPORTED = -1, -2, -3, -4, -5
RBMC_FP64, RBMC_MIXED = 0, 1
RBMC_PC_BJ, RBMC_PC_BJ_LEARNED, RBMC_PC_SPECTRAL = 0, 1, 2
RBMC_SEL_AUTO, RBMC_SEL_BLOCKTRI, RBMC_SEL_KRON = 0, 1, 2
RBMC_GRAD_LOGKAPPA, RBMC_GRAD_LOGTAU, RBMC_GRAD_RHO, RBMC_GRAD_LOGSIGMA = 1, 2, 4, 8
(RBMC_OP_Q, RBMC_OP_DQ_LOGKAPPA, RBMC_OP_DQ_LOGTAU, RBMC_OP_DQ_RHO, RBMC_OP_DQ_LOGSIGMA,
 RBMC_OP_F) = range(6)

# every symbol include/rbmc.h declares
EXPORTS = ["rbmc_ctx_create", "rbmc_ctx_destroy", "rbmc_model_create", "rbmc_model_destroy",
           "rbmc_model_set_theta", "rbmc_apply_op", "rbmc_sample", "rbmc_estimate_from_samples",
           "rbmc_estimate", "rbmc_estimate_batched", "rbmc_plan_query", "rbmc_ctx_profile",
           "rbmc_ctx_profile_read", "rbmc_precond_train", "rbmc_precond_apply",
           "rbmc_precond_get_weights", "rbmc_precond_set_weights", "rbmc_precond_info",
           "rbmc_ctx_get_tune", "rbmc_ctx_set_tune", "rbmc_autotune", "rbmc_last_error",
           "rbmc_normals", "rbmc_apply_op_noalloc", "rbmc_solve", "rbmc_probe_overlap",
           "rbmc_posterior_mean", "rbmc_grad_log_posterior"]
RBMC_MAX_FIXED_EFFECTS = 32
RBMC_PC_NWEIGHTS = 15120
# (cin, cout) of the learned correction's four convolutions, in weight order
PC_LAYERS = [(2, 16), (16, 16), (16, 16), (16, 1)]
(RBMC_KF_GEMM, RBMC_KF_SPD_INVERSE, RBMC_KF_SPMM, RBMC_KF_RSTENCIL, RBMC_KF_PANELS,
 RBMC_KF_GEMM_MIXED, RBMC_KF_GEMM_SMALL, RBMC_KF_INV_SMALL, RBMC_KF_OFFDIAG, RBMC_KF_DCT,
 RBMC_KF_KRON_REDUCE, RBMC_KF_SPEC_SOLVE, RBMC_KF_MC, RBMC_KF_TMIX, RBMC_KF_COUNT) = range(15)
KF_NAMES = ["gemm", "spd_inverse", "spmm", "rstencil", "panels", "gemm_mixed", "gemm_small",
            "inv_small", "offdiag", "dct", "kron_reduce", "spec_solve", "mc", "tmix"]


class rbmc_kernel_stats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("alg_flops", C.c_double),
                ("alg_bytes", C.c_double)]


class rbmc_model_desc(C.Structure):
    _fields_ = [("mx", C.c_int32), ("my", C.c_int32), ("T", C.c_int32), ("h", C.c_double),
                ("log_kappa", C.c_double), ("log_tau", C.c_double), ("rho", C.c_double),
                ("log_sigma", C.c_double), ("obs_mask", C.POINTER(C.c_uint8))]


class rbmc_decomp_desc(C.Structure):
    _fields_ = [("n_tslabs", C.c_int32), ("n_tiles_x", C.c_int32), ("n_tiles_y", C.c_int32),
                ("overlap_hops", C.c_int32), ("pc_tslabs", C.c_int32), ("pc_tiles_x", C.c_int32),
                ("pc_tiles_y", C.c_int32), ("separators", C.c_int32)]


class rbmc_est_opts(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("pcg_maxit", C.c_int32), ("pcg_rtol", C.c_double),
                ("precision", C.c_int32), ("precond", C.c_int32), ("grad_mask", C.c_uint32),
                ("sample_chunk", C.c_int32), ("method", C.c_int32)]


class rbmc_train_opts(C.Structure):
    _fields_ = [("n_pairs", C.c_int32), ("epochs", C.c_int32), ("batch", C.c_int32),
                ("lr", C.c_float), ("seed", C.c_uint64)]


class rbmc_tune(C.Structure):
    _fields_ = [("small_k", C.c_int32), ("small_tiles", C.c_int32), ("wide_from", C.c_int32)]


class rbmc_tune_report(C.Structure):
    _fields_ = [("best", rbmc_tune), ("best_ms", C.c_double), ("default_ms", C.c_double),
                ("from_cache", C.c_int32), ("n_candidates", C.c_int32),
                ("cache_written", C.c_int32)]


class rbmc_pc_info(C.Structure):
    _fields_ = [("ready", C.c_int32), ("usable", C.c_int32), ("val_ratio", C.c_double),
                ("trial_it_bj", C.c_int32), ("trial_it_learned", C.c_int32),
                ("trial_s_bj", C.c_double), ("trial_s_learned", C.c_double)]


class rbmc_report(C.Structure):
    _fields_ = [("t_sample", C.c_double), ("t_factor", C.c_double), ("t_select", C.c_double),
                ("t_correct", C.c_double), ("t_total", C.c_double), ("pcg_it_max", C.c_int32),
                ("pcg_it_mean", C.c_double), ("max_rel_residual", C.c_double),
                ("err_estimate", C.c_double), ("peak_bytes", C.c_int64),
                ("fail_subdomain", C.c_int32), ("fail_block", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                               "python paper_2309_05435_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.rbmc_ctx_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
        L.rbmc_ctx_destroy.argtypes = [vp]
        L.rbmc_ctx_destroy.restype = None
        L.rbmc_model_create.argtypes = [vp, C.POINTER(rbmc_model_desc),
                                        C.POINTER(rbmc_decomp_desc), C.POINTER(vp)]
        L.rbmc_model_destroy.argtypes = [vp]
        L.rbmc_model_destroy.restype = None
        L.rbmc_model_set_theta.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
        L.rbmc_apply_op.argtypes = [vp, C.c_int, vp, vp, C.c_int32]
        L.rbmc_apply_op_noalloc.argtypes = [vp, C.c_int, vp, vp, C.c_int32]
        L.rbmc_sample.argtypes = [vp, C.POINTER(rbmc_est_opts), vp, vp, C.POINTER(rbmc_report)]
        L.rbmc_solve.argtypes = [vp, C.POINTER(rbmc_est_opts), vp, vp, C.POINTER(rbmc_report)]
        L.rbmc_probe_overlap.argtypes = [vp, C.POINTER(rbmc_est_opts), C.c_double, vp, vp, vp]
        L.rbmc_posterior_mean.argtypes = [vp, C.POINTER(rbmc_est_opts), vp, C.c_int32, vp, vp,
                                          vp, vp, vp, vp, C.POINTER(rbmc_report)]
        L.rbmc_grad_log_posterior.argtypes = [vp, C.POINTER(rbmc_est_opts), vp, vp, C.c_uint64,
                                              vp, vp, vp, C.POINTER(rbmc_report)]
        L.rbmc_estimate_from_samples.argtypes = [vp, C.POINTER(rbmc_est_opts), vp, vp,
                                                 C.POINTER(C.c_double), C.POINTER(rbmc_report)]
        L.rbmc_estimate.argtypes = [vp, C.POINTER(rbmc_est_opts), vp, C.c_uint64, vp,
                                    C.POINTER(C.c_double), C.POINTER(rbmc_report)]
        L.rbmc_estimate_batched.argtypes = [vp, C.c_int32, C.POINTER(vp),
                                            C.POINTER(rbmc_est_opts), C.POINTER(vp),
                                            C.POINTER(vp), C.POINTER(C.POINTER(C.c_double)),
                                            C.POINTER(rbmc_report)]
        L.rbmc_plan_query.argtypes = [C.POINTER(rbmc_model_desc), C.POINTER(rbmc_decomp_desc),
                                      C.c_int32, vp, vp]
        L.rbmc_ctx_profile.argtypes = [vp, C.c_int]
        L.rbmc_ctx_profile_read.argtypes = [vp, C.c_int, C.POINTER(rbmc_kernel_stats)]
        L.rbmc_precond_train.argtypes = [vp, C.POINTER(rbmc_est_opts), C.POINTER(rbmc_train_opts),
                                         vp, C.c_int32, C.POINTER(C.c_float),
                                         C.POINTER(rbmc_report)]
        L.rbmc_precond_apply.argtypes = [vp, vp, vp, vp, C.c_int32]
        L.rbmc_precond_get_weights.argtypes = [vp, C.POINTER(C.c_float)]
        L.rbmc_precond_info.argtypes = [vp, C.POINTER(rbmc_pc_info)]
        L.rbmc_ctx_get_tune.argtypes = [vp, C.POINTER(rbmc_tune)]
        L.rbmc_ctx_set_tune.argtypes = [vp, C.POINTER(rbmc_tune)]
        L.rbmc_autotune.argtypes = [vp, C.c_int32, C.POINTER(vp), C.POINTER(rbmc_est_opts),
                                    C.POINTER(vp), C.c_char_p, C.POINTER(rbmc_tune_report)]
        L.rbmc_precond_set_weights.argtypes = [vp, C.POINTER(C.c_float)]
        L.rbmc_normals.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_int64, vp]
        L.rbmc_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("rbmc_ctx_destroy", "rbmc_model_destroy", "rbmc_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class RbmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rbmc status {status}: {msg}")
        self.status = status


def check(st):
    if st < 0:
        raise RbmcError(st, lib().rbmc_last_error().decode())
    return st


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ---- thin wrappers with the C names ----------------------------------------

def rbmc_ctx_create(device: int = 0, stream=None):
    out = C.c_void_p()
    check(lib().rbmc_ctx_create(device, stream, C.byref(out)))
    return out


def rbmc_ctx_destroy(ctx):
    lib().rbmc_ctx_destroy(ctx)


def rbmc_model_create(ctx, desc: rbmc_model_desc, decomp: rbmc_decomp_desc):
    out = C.c_void_p()
    check(lib().rbmc_model_create(ctx, C.byref(desc), C.byref(decomp), C.byref(out)))
    return out


def rbmc_model_destroy(m):
    lib().rbmc_model_destroy(m)


def rbmc_model_set_theta(m, log_kappa, log_tau, rho, log_sigma):
    return check(lib().rbmc_model_set_theta(m, log_kappa, log_tau, rho, log_sigma))


def rbmc_apply_op(m, op, x, y, n_rhs):
    return check(lib().rbmc_apply_op(m, op, _ptr(x), _ptr(y), n_rhs))


def rbmc_apply_op_noalloc(m, op, x, y, n_rhs):
    """Enqueued on the context stream, not synchronized."""
    return check(lib().rbmc_apply_op_noalloc(m, op, _ptr(x), _ptr(y), n_rhs))


def rbmc_probe_overlap(m, opts, eps, T=0, ns=0):
    """(status, lags [time, space, suggested hops], corr_time (T), corr_space
    (ns)); the profiles are returned when T and ns are given."""
    import numpy as np
    lags = np.zeros(3, np.int32)
    ct = np.zeros(T) if T else None
    cs = np.zeros(ns) if ns else None
    ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)  # noqa: E731
    st = check(lib().rbmc_probe_overlap(m, C.byref(opts), C.c_double(eps), ptr(lags), ptr(ct),
                                        ptr(cs)))
    return st, lags, ct, cs


def rbmc_posterior_mean(m, opts, y, n_beta, a_beta, q_beta, mu_u, var_u_add=None):
    """(status, mu_beta, var_beta, report); y, a_beta, mu_u, var_u_add are
    device tensors, q_beta host values."""
    import numpy as np
    q = np.ascontiguousarray(q_beta, np.float64).reshape(n_beta)
    mb = np.zeros(n_beta)
    vb = np.zeros((n_beta, n_beta))
    rep = rbmc_report()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p) if a.size else None  # noqa: E731
    st = check(lib().rbmc_posterior_mean(m, C.byref(opts), _ptr(y), n_beta, _ptr(a_beta), ptr(q),
                                         _ptr(mu_u), ptr(mb), ptr(vb), _ptr(var_u_add),
                                         C.byref(rep)))
    return st, mb, vb, rep


def rbmc_grad_log_posterior(m, opts, y, x=None, seed=0, mu_out=None):
    """(status, grad (4), terms (4 x 5), report); y, x, mu_out device tensors."""
    import numpy as np
    g = np.zeros(4)
    terms = np.zeros((4, 5))
    rep = rbmc_report()
    st = check(lib().rbmc_grad_log_posterior(m, C.byref(opts), _ptr(y), _ptr(x), C.c_uint64(seed),
                                             g.ctypes.data_as(C.c_void_p),
                                             terms.ctypes.data_as(C.c_void_p), _ptr(mu_out),
                                             C.byref(rep)))
    return st, g, terms, rep


def rbmc_solve(m, opts, b, x):
    rep = rbmc_report()
    st = check(lib().rbmc_solve(m, C.byref(opts), _ptr(b), _ptr(x), C.byref(rep)))
    return st, rep


def rbmc_sample(m, opts, z, x):
    rep = rbmc_report()
    st = check(lib().rbmc_sample(m, C.byref(opts), _ptr(z), _ptr(x), C.byref(rep)))
    return st, rep


def rbmc_estimate_from_samples(m, opts, x, diag_out, n_trace):
    rep = rbmc_report()
    tr = (C.c_double * max(n_trace, 1))()
    st = check(lib().rbmc_estimate_from_samples(m, C.byref(opts), _ptr(x), _ptr(diag_out),
                                                tr if n_trace else None, C.byref(rep)))
    return st, list(tr)[:n_trace], rep


def rbmc_estimate(m, opts, z, seed, diag_out, n_trace):
    rep = rbmc_report()
    tr = (C.c_double * max(n_trace, 1))()
    st = check(lib().rbmc_estimate(m, C.byref(opts), _ptr(z), seed, _ptr(diag_out),
                                   tr if n_trace else None, C.byref(rep)))
    return st, list(tr)[:n_trace], rep


def rbmc_estimate_batched(ctx, models, opts, zs, diag_outs, n_trace):
    """models: model handles of one context; zs, diag_outs: device tensors per model."""
    nm = len(models)
    vp = C.c_void_p
    mh = (vp * max(nm, 1))(*[m.value for m in models])
    zp = (vp * max(nm, 1))(*[None if z is None else z.data_ptr() for z in zs])
    dp = (vp * max(nm, 1))(*[d.data_ptr() for d in diag_outs])
    trs = [(C.c_double * max(n_trace, 1))() for _ in range(nm)]
    tp = (C.POINTER(C.c_double) * max(nm, 1))(
        *[C.cast(t, C.POINTER(C.c_double)) for t in trs])
    rep = rbmc_report()
    st = check(lib().rbmc_estimate_batched(ctx, nm, mh, C.byref(opts), zp, dp,
                                           tp if n_trace else None, C.byref(rep)))
    return st, [list(t)[:n_trace] for t in trs], rep


def rbmc_precond_train(m, pcg_opts, train_opts, z, n_train):
    loss = (C.c_float * (train_opts.epochs + 1))()
    rep = rbmc_report()
    st = check(lib().rbmc_precond_train(m, C.byref(pcg_opts), C.byref(train_opts), _ptr(z),
                                        n_train, loss, C.byref(rep)))
    return st, list(loss), rep


def rbmc_precond_apply(m, r, u, y, n_rhs):
    return check(lib().rbmc_precond_apply(m, _ptr(r), _ptr(u), _ptr(y), n_rhs))


def rbmc_precond_get_weights(m):
    import numpy as np
    w = np.zeros(RBMC_PC_NWEIGHTS, np.float32)
    check(lib().rbmc_precond_get_weights(m, w.ctypes.data_as(C.POINTER(C.c_float))))
    return w


def rbmc_ctx_get_tune(ctx):
    t = rbmc_tune()
    check(lib().rbmc_ctx_get_tune(ctx, C.byref(t)))
    return t


def rbmc_ctx_set_tune(ctx, small_k, small_tiles, wide_from):
    return check(lib().rbmc_ctx_set_tune(ctx, C.byref(rbmc_tune(small_k, small_tiles, wide_from))))


def rbmc_autotune(ctx, models, opts, zs, cache_path=None):
    """models: model handles of one context; zs: per model (n + n_obs) x n_k device
    tensors (None entries when n_k = 0).  Returns an rbmc_tune_report."""
    nm = len(models)
    vp = C.c_void_p
    mh = (vp * max(nm, 1))(*[m.value for m in models])
    zp = (vp * max(nm, 1))(*[None if z is None else z.data_ptr() for z in zs])
    rep = rbmc_tune_report()
    check(lib().rbmc_autotune(ctx, nm, mh, C.byref(opts), zp,
                              cache_path.encode() if cache_path else None, C.byref(rep)))
    return rep


def rbmc_precond_info(m):
    info = rbmc_pc_info()
    check(lib().rbmc_precond_info(m, C.byref(info)))
    return info


def rbmc_precond_set_weights(m, w):
    import numpy as np
    w = np.ascontiguousarray(w, np.float32)
    assert w.shape == (RBMC_PC_NWEIGHTS,)
    return check(lib().rbmc_precond_set_weights(m, w.ctypes.data_as(C.POINTER(C.c_float))))


def rbmc_normals(ctx, seed, offset, count, out):
    """out: device float64 tensor with at least count entries."""
    return check(lib().rbmc_normals(ctx, seed, offset, count, _ptr(out)))


def rbmc_plan_query(desc, decomp, p, label_out=None, state_out=None):
    """label_out / state_out: numpy int32 / uint8 arrays of length n (host)."""
    lp = None if label_out is None else label_out.ctypes.data_as(C.c_void_p)
    sp = None if state_out is None else state_out.ctypes.data_as(C.c_void_p)
    return check(lib().rbmc_plan_query(C.byref(desc), C.byref(decomp), p, lp, sp))


def rbmc_ctx_profile(ctx, enable: bool):
    return check(lib().rbmc_ctx_profile(ctx, 1 if enable else 0))


def rbmc_ctx_profile_read(ctx, family: int) -> dict:
    st = rbmc_kernel_stats()
    check(lib().rbmc_ctx_profile_read(ctx, family, C.byref(st)))
    return {f: getattr(st, f) for f, _ in st._fields_}


# ---- convenience ------------------------------------------------------------

def make_desc(mx, my, T, h, theta, mask):
    """mask: numpy uint8 array (kept alive by the returned tuple)."""
    import numpy as np
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    d = rbmc_model_desc(mx, my, T, h, theta[0], theta[1], theta[2], theta[3],
                        mask.ctypes.data_as(C.POINTER(C.c_uint8)))
    return d, mask


def make_opts(n_samples, pcg_maxit=2000, pcg_rtol=1e-8, grad_mask=0b111,
              precision=RBMC_FP64, precond=RBMC_PC_BJ, method=RBMC_SEL_AUTO, sample_chunk=0):
    return rbmc_est_opts(n_samples, pcg_maxit, pcg_rtol, precision, precond, grad_mask,
                         sample_chunk, method)


def make_train_opts(n_pairs=2000, epochs=5, batch=8, lr=1e-3, seed=1):
    return rbmc_train_opts(n_pairs, epochs, batch, lr, seed)


def popcount(mask: int) -> int:
    return bin(mask).count("1")


class Model:
    """Owns a context + model; inputs/outputs are torch tensors on the device."""

    def __init__(self, wl, mask=None, theta=None, device: int = 0, decomp=None, pc="workload",
                 shape=None):
        """pc: block-Jacobi blocks (slabs, tiles_x, tiles_y); "workload" takes the
        workload's setting, None or () the cores.  shape: (mx, my) for a grid
        other than the workload's m x m (mask then drawn for mx my T nodes)."""
        if isinstance(pc, str):
            pc = getattr(wl, "pc", None)
        import torch
        self.wl = wl
        self.torch = torch
        self.dev = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.dev).cuda_stream
        self.ctx = rbmc_ctx_create(device, C.c_void_p(stream))
        mx, my = shape if shape else (wl.m, wl.m)
        if mask is None:
            from .inputs import obs_mask
            mask = wl.mask() if not shape else obs_mask(mx * my * wl.T, wl.obs_frac,
                                                        wl.mask_seed)
        th = wl.theta if theta is None else theta
        self.desc, self._mask = make_desc(mx, my, wl.T, wl.h, th, mask)
        if decomp is None:
            decomp = (wl.n_tslabs, wl.n_tiles, wl.n_tiles, wl.n_l)
        decomp = tuple(decomp) + (tuple(pc) if pc else ())
        self.decomp = rbmc_decomp_desc(*decomp)
        self.m = rbmc_model_create(self.ctx, self.desc, self.decomp)
        self.n = mx * my * wl.T
        self.n_obs = int(self._mask.sum())

    def close(self):
        if getattr(self, "m", None):
            rbmc_model_destroy(self.m)
            self.m = None
        if getattr(self, "ctx", None):
            rbmc_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def apply(self, op, x):
        x = x.contiguous()
        n_rhs = x.shape[0]
        y = self.torch.empty((n_rhs, self.n), dtype=self.torch.float64, device=self.dev)
        rbmc_apply_op(self.m, op, x, y, n_rhs)
        return y

    def sample(self, z, rtol=1e-8, maxit=5000, precond=RBMC_PC_BJ, precision=RBMC_FP64):
        z = z.contiguous()
        x = self.torch.empty((z.shape[0], self.n), dtype=self.torch.float64, device=self.dev)
        st, rep = rbmc_sample(self.m, make_opts(z.shape[0], maxit, rtol, precision=precision,
                                                precond=precond), z, x)
        return x, st, rep

    def solve(self, b, rtol=1e-8, maxit=5000, precond=RBMC_PC_BJ):
        """x with Q x_k = b_k for the rows b_k of b ((n_rhs, n) device tensor)."""
        b = b.contiguous()
        x = self.torch.empty((b.shape[0], self.n), dtype=self.torch.float64, device=self.dev)
        st, rep = rbmc_solve(self.m, make_opts(b.shape[0], maxit, rtol, precond=precond), b, x)
        return x, st, rep

    def posterior_mean(self, y, a_beta, q_beta, rtol=1e-8, maxit=5000, precond=RBMC_PC_BJ,
                       var_u_add=True):
        """(mu_u, mu_beta, var_beta, var_u_add or None, status, report) of
        rbmc_posterior_mean; y (n_obs) and a_beta ((n_beta, n_obs)) device
        tensors, q_beta host values."""
        nb = len(q_beta)
        mu = self.torch.empty(self.n, dtype=self.torch.float64, device=self.dev)
        va = self.torch.empty_like(mu) if var_u_add else None
        st, mb, vb, rep = rbmc_posterior_mean(
            self.m, make_opts(1, maxit, rtol, precond=precond), y.contiguous(), nb,
            a_beta.contiguous() if nb else None, q_beta, mu, va)
        return mu, mb, vb, va, st, rep

    def grad_log_posterior(self, y, x=None, n_samples=None, seed=0, rtol=1e-8, maxit=5000,
                           precond=RBMC_PC_BJ, method=RBMC_SEL_AUTO, sample_chunk=0):
        """(grad, terms, mu, status, report) of rbmc_grad_log_posterior; x a
        (n_k, n) device tensor of samples, or None with n_samples > 0 for
        device normals from seed."""
        nk = (0 if x is None else x.shape[0]) if n_samples is None else n_samples
        mu = self.torch.empty(self.n, dtype=self.torch.float64, device=self.dev)
        st, g, terms, rep = rbmc_grad_log_posterior(
            self.m, make_opts(nk, maxit, rtol, grad_mask=0b1111, precond=precond, method=method,
                              sample_chunk=sample_chunk),
            y.contiguous(), None if x is None else x.contiguous(), seed, mu)
        return g, terms, mu, st, rep

    def probe_overlap(self, eps=1e-3, rtol=1e-12, maxit=2000, precond=RBMC_PC_BJ):
        """(status, lags, corr_time, corr_space) of rbmc_probe_overlap."""
        T = self.wl.T
        return rbmc_probe_overlap(self.m, make_opts(1, maxit, rtol, precond=precond), eps, T,
                                  self.n // T)

    def estimate_from_samples(self, x, grad_mask=0b111, method=RBMC_SEL_AUTO,
                              precision=RBMC_FP64):
        n_k = 0 if x is None else x.shape[0]
        diag = self.torch.empty(self.n, dtype=self.torch.float64, device=self.dev)
        st, tr, rep = rbmc_estimate_from_samples(
            self.m, make_opts(n_k, grad_mask=grad_mask, method=method, precision=precision),
            None if x is None else x.contiguous(), diag, popcount(grad_mask))
        return diag, tr, st, rep

    def estimate(self, z, grad_mask=0b111, rtol=1e-8, maxit=5000, precond=RBMC_PC_BJ,
                 method=RBMC_SEL_AUTO, precision=RBMC_FP64, sample_chunk=0, n_samples=None,
                 seed=0):
        """z: (n_k, n + n_obs) device tensor, or None for device normals drawn
        from seed (then n_samples gives n_k)."""
        diag = self.torch.empty(self.n, dtype=self.torch.float64, device=self.dev)
        nk = z.shape[0] if z is not None else n_samples
        opts = make_opts(nk, maxit, rtol, grad_mask, precision, precond, method, sample_chunk)
        st, tr, rep = rbmc_estimate(self.m, opts, None if z is None else z.contiguous(), seed,
                                    diag, popcount(grad_mask))
        return diag, tr, st, rep


class ModelSet:
    """Many models in one context, estimated together by rbmc_estimate_batched
    (or one by one with rbmc_estimate, for comparison)."""

    def __init__(self, wls, device: int = 0, pc="workload"):
        import torch
        self.torch = torch
        self.wls = list(wls)
        self.dev = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.dev).cuda_stream
        self.ctx = rbmc_ctx_create(device, C.c_void_p(stream))
        self.models, self._keep, self.n, self.n_obs = [], [], [], []
        for wl in self.wls:
            p = getattr(wl, "pc", None) if isinstance(pc, str) else pc
            desc, mask = make_desc(wl.m, wl.m, wl.T, wl.h, wl.theta, wl.mask())
            dc = rbmc_decomp_desc(*((wl.n_tslabs, wl.n_tiles, wl.n_tiles, wl.n_l) +
                                    (tuple(p) if p else ())))
            self.models.append(rbmc_model_create(self.ctx, desc, dc))
            self._keep.append((desc, mask, dc))
            self.n.append(wl.m * wl.m * wl.T)
            self.n_obs.append(int(mask.sum()))

    def close(self):
        for m in getattr(self, "models", []):
            rbmc_model_destroy(m)
        self.models = []
        if getattr(self, "ctx", None):
            rbmc_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def _diags(self):
        return [self.torch.empty(n, dtype=self.torch.float64, device=self.dev) for n in self.n]

    def estimate(self, zs, grad_mask=0b111, rtol=1e-8, maxit=5000):
        """zs: per model (n_k, n + n_obs) device tensors (same n_k)."""
        zs = [z.contiguous() for z in zs]
        diags = self._diags()
        st, trs, rep = rbmc_estimate_batched(
            self.ctx, self.models, make_opts(zs[0].shape[0], maxit, rtol, grad_mask), zs, diags,
            popcount(grad_mask))
        return diags, trs, st, rep

    def estimate_each(self, zs, grad_mask=0b111, rtol=1e-8, maxit=5000):
        diags, trs, sts, reps = self._diags(), [], [], []
        for m, z, d in zip(self.models, zs, diags):
            st, tr, rep = rbmc_estimate(m, make_opts(z.shape[0], maxit, rtol, grad_mask),
                                        z.contiguous(), 0, d, popcount(grad_mask))
            trs.append(tr)
            sts.append(st)
            reps.append(rep)
        return diags, trs, sts, reps
