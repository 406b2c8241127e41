"""Throughput benchmark of the RBMC hot path on one MI355X.

A step is one full estimate at <= 1% error on the 512 x 512 x 48 space-time
workload (n = 12,582,912; 5% observed; 3 time slabs x 8 x 8 tiles of 64 x 64
= 192 subdomains with 2 hops of overlap; PCG to 1e-8; traces for log kappa,
log tau, rho and log sigma): rebuild Q(theta), form the selected entries of
every subdomain inverse, then per pass of samples draw z on the device,
sample x = Q^-1 F z by PCG, and run the correction solves and the
diagonal/trace accumulation.  The sample count is the smallest multiple of
the pass size (256) whose plug-in error, predicted from a 200-sample
estimate, is <= 0.90%.
Prints one JSON line.  After the timed steps (each leg only while the
wall-time budget allows): the stated setting (200 samples), the true error
at uniformly drawn nodes against exact (Q^-1)_ii from PCG solves, the CPU
oracle on a bounded sample, the plain FP64 block-Jacobi method, the batched
uneven models.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6    # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix


# the HIP kernel behind each instrumented family
KERNEL_OF = {"gemm": "k_gemm_f64<0>", "gemm_small": "k_gemm_f64s", "gemm_mixed": "k_gemm_mx",
             "inv_small": "k_inv128", "spmm": "k_space_time_op", "rstencil": "k_rstencil",
             "panels": "k_panels", "spd_inverse": "gauss_jordan", "offdiag": "k_offdiag",
             "dct": "k_dct_fft", "kron_reduce": "k_kron_reduce", "spec_solve": "k_spec_solve_reg",
             "mc": "k_mc", "tmix": "k_kron_tmix"}


def kernel_file_tag(kern: str) -> str:
    """k_gemm_f64<1> -> k_gemm_f64_1 (profile file names)."""
    return kern.replace("<", "_").replace(">", "")


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2309_05435_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_file_tag(kernel)}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("sources_hash") != kernel_sources_hash():
        return None
    return d.get("bytes_per_launch")


def calibration_copy(nbytes: int, reps: int = 3):
    """A plain device-to-device copy of nbytes, reps times: under rocprofv3
    --pmc its FETCH_SIZE / WRITE_SIZE per dispatch give the counter's scale."""
    import torch
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n * 8, "reps": reps}), flush=True)


def _counter_per_dispatch(path: str, counter: str):
    """{kernel name: [KiB per dispatch, ...]} from a rocprofv3 counter CSV."""
    import csv
    out = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def write_traffic(paths, workload: str, copy_bytes: int, commands):
    """HBM bytes per launch of each library kernel from two counter runs of the
    bench (FETCH_SIZE, WRITE_SIZE) and two of the calibration copy, each
    scaled by (known copy bytes) / (counter reading of the copy)."""
    f_main, w_main, f_copy, w_copy = (_counter_per_dispatch(p, c) for p, c in zip(
        paths, ("FETCH_SIZE", "WRITE_SIZE", "FETCH_SIZE", "WRITE_SIZE")))

    def copy_kib(d):
        vals = [v for k, vs in d.items() if "copyBuffer" in k for v in vs]
        big = [v for v in vals if v * 1024 > copy_bytes / 2]
        return sum(big) / len(big)

    s_fetch = copy_bytes / (copy_kib(f_copy) * 1024)
    s_write = copy_bytes / (copy_kib(w_copy) * 1024)
    written = []
    for fam, kern in KERNEL_OF.items():
        # the stencil family times Q p with the fused dot: k_space_time_op<0, true>
        if kern == "k_space_time_op":
            pat = re.compile(r"(^|[\s:])k_space_time_op<0, true>\(")
        elif "<" in kern:
            pat = re.compile(r"(^|[\s:])" + re.escape(kern) + r"\(")
        else:
            pat = re.compile(r"(^|[\s:])" + re.escape(kern) + r"[<(]")
        fk = [k for k in f_main if pat.search(k)]
        wk = [k for k in w_main if pat.search(k)]
        if not fk or not wk:
            continue
        fv = [v for k in fk for v in f_main[k]]
        wv = [v for k in wk for v in w_main[k]]
        fb = sum(fv) / len(fv) * 1024 * s_fetch
        wb = sum(wv) / len(wv) * 1024 * s_write
        rec = {"kernel": kern, "workload": workload, "dispatches": len(fv),
               "bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb,
               "write_bytes_per_launch": wb, "scale_fetch": s_fetch, "scale_write": s_write,
               "calibration_copy_bytes": copy_bytes, "sources_hash": kernel_sources_hash(),
               "commands": commands}
        path = os.path.join(ROOT, "profiles", f"traffic_{kernel_file_tag(kern)}_{workload}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        written.append(path)
    print(json.dumps({"written": written}))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_entry(wl):
    """The CPU oracle on a bounded sample of the workload: the estimator at one
    node of an interior subdomain (slab 1, tile (3, 3)): conjugate gradients on
    Q_AA to the workload's tolerance (one column of Q_AA^-1) and the Monte
    Carlo part from the same column, with the oracle's threads on all host
    cores.  The oracle builds Q only on a window of the grid holding A and its
    separator (the estimator at a node reads Q through Q_AA and Q_AB only).
    Its whole-subdomain path (banded Cholesky of the 102,880-node Q_AA, then
    one banded solve per core row) takes far longer than this bound allows;
    the rate below is per entry, scaled to entries/s."""
    import numpy as np
    import oracle as O
    p = (1 * wl.n_tiles + 3) * wl.n_tiles + 3
    base, extra = divmod(wl.T, wl.n_tslabs)
    sl = p // (wl.n_tiles * wl.n_tiles)
    t0 = sl * base + min(sl, extra)
    t1 = t0 + base + (1 if sl < extra else 0)
    tx = p % wl.n_tiles
    ty = (p // wl.n_tiles) % wl.n_tiles
    side = wl.m // wl.n_tiles
    x0, y0 = tx * side, ty * side
    ms, mt = 2 * (wl.n_l + 1) + 2, wl.n_l + 2
    wt0, wt1 = max(0, t0 - mt), min(wl.T, t1 + mt)
    wx0, wx1 = max(0, x0 - ms), min(wl.m, x0 + side + ms)
    wy0, wy1 = max(0, y0 - ms), min(wl.m, y0 + side + ms)
    tt, yy, xx = np.meshgrid(np.arange(wt0, wt1), np.arange(wy0, wy1), np.arange(wx0, wx1),
                             indexing="ij")
    glob = (tt * wl.m * wl.m + yy * wl.m + xx).ravel()
    M = O.OracleModel(wx1 - wx0, wy1 - wy0, wt1 - wt0, wl.h, *wl.theta, wl.mask()[glob])
    inside = ((tt >= t0) & (tt < t1) & (yy >= y0) & (yy < y0 + side) & (xx >= x0) &
              (xx < x0 + side)).ravel()
    labels = np.where(inside, 0, 1).astype(np.int32)
    x = np.random.default_rng(1).standard_normal((wl.n_k, M.n))
    i = int(np.flatnonzero(inside)[inside.sum() // 2])
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    t = time.perf_counter()
    M.entry(labels, 0, wl.n_l, i, x, rtol=wl.rtol)
    dt = time.perf_counter() - t
    return {"value": 1.0 / dt, "unit": "entries/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": (f"one diagonal entry of the {wl.m}x{wl.m}x{wl.T} workload (a node at the "
                       f"centre of interior core {p}): oracle conjugate gradients on its Q_AA "
                       f"(window model of {M.n} nodes) to {wl.rtol:g} plus the Monte Carlo part "
                       f"for {wl.n_k} samples, {dt:.1f} s; all n = {wl.n} entries would take "
                       f"n times as long ({wl.n * dt / 86400.0:.0f} days); sampling excluded "
                       f"(per entry about 1e-3 of this cost)")}


def cpu_baseline(wl, m_sample: int):
    """The CPU oracle, as it stands, on the same workload with the spatial grid
    reduced to m_sample^2 (full pipeline: exact sampling + estimator)."""
    import oracle as O
    sub = wl.replace(m=m_sample)
    M = O.OracleModel.from_workload(sub)
    lab = O.grid_cores(sub.m, sub.m, sub.T, sub.n_tslabs, sub.n_tiles, sub.n_tiles)
    z = sub.z()
    t0 = time.perf_counter()
    x = M.sample(z)
    M.rbmc(lab, sub.n_tslabs * sub.n_tiles * sub.n_tiles, sub.n_l, x, 0b111)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": sub.n / dt, "unit": "entries/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": (f"full oracle pipeline (banded-Cholesky sampling + estimator) on the "
                       f"same workload with the grid reduced to {m_sample}x{m_sample} "
                       f"(n={sub.n}, {sub.n_k} samples), {dt:.1f} s")}


def tune_dict(r):
    return {"small_k": r.best.small_k, "small_tiles": r.best.small_tiles,
            "wide_from": r.best.wide_from, "ms": r.best_ms,
            "default_ms": r.default_ms if not r.from_cache else None,
            "from_cache": bool(r.from_cache), "candidates": r.n_candidates}


def batched_leg(n_models: int, tune_cache=None, per_model=True):
    """The uneven-model workload (grids 16^2-48^2, T 8-24, 2-8 slabs, 1-step
    overlap, 100 samples): all models in one rbmc_estimate_batched call against
    the same models estimated one call each (unless per_model is False).  Each
    timing follows a warm-up."""
    import torch

    from paper_2309_05435_amd import binding as B
    from paper_2309_05435_amd.inputs import batched_models

    torch.cuda.empty_cache()  # the library allocates beside torch's cache
    wls = batched_models(n_models)
    ms = B.ModelSet(wls)
    zs = [torch.from_numpy(wl.z()).to("cuda") for wl in wls]
    tune = None
    if tune_cache is not None:
        tr_ = B.rbmc_autotune(ms.ctx, ms.models,
                              B.make_opts(wls[0].n_k, pcg_maxit=5000, pcg_rtol=wls[0].rtol),
                              zs, tune_cache)
        tune = tune_dict(tr_)
    n_tot = sum(ms.n)
    res = {"workload": f"{n_models} uneven models, sum n = {n_tot}", "n_models": n_models,
           "n_samples": wls[0].n_k, "tune": tune}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    def reset_theta():
        for m, wl in zip(ms.models, wls):
            B.rbmc_model_set_theta(m, *wl.theta)

    def run_batched():
        reset_theta()
        return ms.estimate(zs, rtol=wls[0].rtol)

    def run_each():
        reset_theta()
        return ms.estimate_each(zs, rtol=wls[0].rtol)

    sec_b, (db, tb, st, rep) = timed(run_batched)
    per, speedup, dev = None, None, None
    if per_model:
        sec_e, (de, te, sts, reps) = timed(run_each)
        dev = max(float(((a - b).abs() / b.abs()).max()) for a, b in zip(db, de))
        per = {"value": n_tot / sec_e, "ms_per_step": sec_e * 1e3}
        speedup = sec_e / sec_b
    res.update({"value": n_tot / sec_b, "unit": "entries/s", "ms_per_step": sec_b * 1e3,
                "per_model_calls": per, "speedup": speedup, "max_rel_diff_vs_per_model": dev,
                "err_estimate": rep.err_estimate, "pcg_iters_max": rep.pcg_it_max,
                "phase_s": {k: getattr(rep, k) for k in ("t_sample", "t_factor", "t_select",
                                                         "t_correct", "t_total")},
                "device_bytes": rep.peak_bytes})
    ms.close()
    del zs
    torch.cuda.empty_cache()
    return res


def main():
    t_start = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tile512")
    ap.add_argument("--samples", type=int, default=0,
                    help="samples of the timed estimate (0: the smallest multiple of the pass "
                         "size whose plug-in error, predicted from the workload's own sample "
                         "count, is <= 0.90%%)")
    ap.add_argument("--pass-samples", type=int, default=256,
                    help="samples per pass of the timed estimate (0: the workload's count); "
                         "a multiple of 128 fills the matrix-core tiles of the products "
                         "with Y and Z (measured: 256 per pass 4%% faster per sample than 200)")
    ap.add_argument("--budget-s", type=float, default=600.0,
                    help="wall-time budget: legs after the timed steps run only if their "
                         "projected end stays within it")
    ap.add_argument("--legs",
                    default="stated,mixed,probe,mean,grad,alg2,true_error,cpu,plain,batched",
                    help="legs after the timed steps, in order (subset of stated,mixed,probe,"
                         "mean,grad,alg2,true_error,cpu,plain,batched; empty for none)")
    ap.add_argument("--true-error-nodes", type=int, default=256)
    ap.add_argument("--pc", default="1,32,32",
                    help="block-Jacobi blocks 'slabs,tiles_x,tiles_y' of the plain leg, or 'cores'")
    ap.add_argument("--plain-est-s", type=float, default=150.0,
                    help="projected duration of the plain block-Jacobi leg (budget check)")
    ap.add_argument("--cpu-sample-m", type=int, default=24,
                    help="grid side of the CPU oracle leg for workloads other than tile512")
    ap.add_argument("--batched-models", type=int, default=256)
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched workload and print its JSON")
    ap.add_argument("--no-per-model", action="store_true",
                    help="batched workload without the one-call-per-model comparison")
    ap.add_argument("--calibration-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched leg: keep the default launch shapes")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2309_05435_amd",
                                                          "tune_cache.txt"),
                    help="autotuner cache file (read, and appended to when a workload is new)")
    ap.add_argument("--traffic-from", nargs=4, metavar="CSV",
                    help="write profiles/traffic_*.json from the counter CSVs of the bench "
                         "(FETCH_SIZE, WRITE_SIZE) and of the calibration copy (same order)")
    ap.add_argument("--commands", default="", help="commands recorded with --traffic-from")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args.traffic_from, args.workload, args.calibration_copy,
                      args.commands)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibration_copy:
        calibration_copy(args.calibration_copy)
        return
    if args.batched_only:
        print(json.dumps(batched_leg(args.batched_models,
                                     None if args.no_autotune else args.tune_cache,
                                     per_model=not args.no_per_model)), flush=True)
        return

    from paper_2309_05435_amd import binding as B
    from paper_2309_05435_amd.inputs import WORKLOADS, normals

    wl = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    legs = [v for v in args.legs.split(",") if v]

    def say(msg):
        print(f"[{time.perf_counter() - t_start:7.1f} s] {msg}", file=sys.stderr, flush=True)

    # ---- the path: spectral-preconditioned PCG sampler (FP64 residuals and
    # dots), Kronecker form of the subdomain inverses, FP64, z drawn on the
    # device from the workload's seed; samples in passes of the workload's
    # sample count
    grad = 0b1111
    seed = wl.z_seed
    chunk = args.pass_samples or wl.n_k
    gm = B.Model(wl)
    diag = torch.empty(gm.n, dtype=torch.float64, device="cuda")
    theta = wl.theta

    def opts_for(nk, passes=True, precision=B.RBMC_FP64):
        return B.make_opts(nk, pcg_maxit=500, pcg_rtol=wl.rtol, grad_mask=grad,
                           precision=precision, precond=B.RBMC_PC_SPECTRAL,
                           method=B.RBMC_SEL_KRON,
                           sample_chunk=chunk if passes and nk > chunk else 0)

    def estimate(opts):
        # rebuilding Q(theta) invalidates every factor: each estimate factors again
        B.rbmc_model_set_theta(gm.m, *theta)
        return B.rbmc_estimate(gm.m, opts, None, seed, diag, B.popcount(grad))

    # the stated setting (the workload's own sample count) first: it loads the
    # code and sizes the workspaces, and its plug-in error sets the sample
    # count of the timed estimate (the error falls as n_k^-1/2).  The target
    # 0.90% leaves room for the plug-in estimate reading 5-7% below the true
    # error measured at uniformly drawn nodes on this workload
    _, _, rep0 = estimate(opts_for(wl.n_k, passes=False))
    err0 = rep0.err_estimate
    nk = args.samples or max(wl.n_k, int(math.ceil(wl.n_k * (err0 / 0.0090) ** 2 / chunk)) * chunk)
    say(f"stated setting: {wl.n_k} samples, plug-in error {err0:.4f}; timed estimate: {nk} "
        f"samples in {nk // chunk} passes")
    opts = opts_for(nk)
    for i in range(args.warmup):
        estimate(opts)
        say(f"warm-up estimate {i + 1} of {args.warmup} done")
    torch.cuda.synchronize()
    B.rbmc_ctx_profile(gm.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(args.steps):
        st, tr, rep = estimate(opts)
        reps.append(rep.as_dict())
        say(f"timed estimate {i + 1} of {args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = {B.KF_NAMES[f]: B.rbmc_ctx_profile_read(gm.ctx, f) for f in range(B.RBMC_KF_COUNT)}
    B.rbmc_ctx_profile(gm.ctx, False)
    d_head = diag.clone()
    ms = (t1 - t0) * 1000.0 / args.steps
    value = gm.n / (ms / 1000.0)
    flop_fams = ("gemm", "gemm_small", "gemm_mixed", "inv_small")

    def roofline(fam):
        s = stats[fam]
        per_launch = 1.0 / max(s["launches"], 1)
        if fam in flop_fams:
            peak = PEAK_FP32_TFLOPS if fam == "gemm_mixed" else PEAK_FP64_TFLOPS
            achieved = s["alg_flops"] / (s["total_ms"] * 1e-3) / 1e12
            r = {"bound": "alu" if fam == "inv_small" else "mfma", "achieved": achieved,
                 "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                 "alg_flops_per_launch": s["alg_flops"] * per_launch}
        else:
            achieved = s["alg_bytes"] / (s["total_ms"] * 1e-3) / 1e9
            r = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": achieved / PEAK_HBM_GBS,
                 "alg_bytes_per_launch": s["alg_bytes"] * per_launch}
        r["traffic"] = traffic_for(KERNEL_OF[fam], wl.name)
        r["kernel"] = KERNEL_OF[fam]
        r["family"] = fam
        r["launches_per_step"] = s["launches"] // max(args.steps, 1)
        r["avg_launch_ms"] = s["total_ms"] * per_launch
        r["ms_per_step"] = s["total_ms"] / max(args.steps, 1)
        return r

    # dominant single kernel: the largest speed-of-light time per step
    # (algorithmic flops / peak, or bytes / HBM peak).  The inversion family is
    # a composite of several kernels whose products are counted under the GEMM
    # families.
    def ideal_ms(fam):
        s = stats[fam]
        if fam in flop_fams:
            peak = PEAK_FP32_TFLOPS if fam == "gemm_mixed" else PEAK_FP64_TFLOPS
            return s["alg_flops"] / (peak * 1e12) * 1e3
        return s["alg_bytes"] / (PEAK_HBM_GBS * 1e9) * 1e3

    singles = [k for k in stats if k != "spd_inverse" and stats[k]["launches"] > 0]
    dom = max(singles, key=ideal_ms)
    roof = roofline(dom)
    roof["ideal_ms_per_step"] = ideal_ms(dom) / max(args.steps, 1)
    others = {k: dict(roofline(k), ideal_ms_per_step=ideal_ms(k) / max(args.steps, 1))
              for k in singles if k != dom}
    last = reps[-1]
    err = last["err_estimate"]
    out = {
        "metric": "diag(Q^-1) entries/sec at <=1% rel err; PCG iters; learned+mixed vs plain",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": f"{wl.m}x{wl.m}", "T": wl.T, "n": gm.n,
                   "n_obs": gm.n_obs, "n_samples": nk, "samples_per_pass": chunk,
                   "passes": nk // chunk, "stated_n_samples": wl.n_k,
                   "n_tslabs": wl.n_tslabs, "n_tiles": wl.n_tiles, "overlap_hops": wl.n_l,
                   "subdomains": wl.n_tslabs * wl.n_tiles * wl.n_tiles, "pcg_rtol": wl.rtol,
                   "precision": "fp64", "precond": "spectral (Q_t x Q_s + mean(D) I)",
                   "selected_inverse": "kronecker-woodbury",
                   "traces": "logkappa,logtau,rho,logsigma",
                   "z": f"device normals (Philox4x32-10), seed {seed}"},
        "pcg_iters": {"mean": last["pcg_it_mean"], "max": last["pcg_it_max"]},
        "err_estimate": err,
        "accuracy_gate_1pct": bool(err <= 0.01),
        "phase_s": {k: last[k] for k in ("t_sample", "t_factor", "t_select", "t_correct",
                                         "t_total")},
        "device_bytes": last["peak_bytes"],
        "kernel_ms_per_step": {k: v["total_ms"] / args.steps for k, v in stats.items()},
        "roofline": roof,
        "rooflines_other_kernels": others,
        "cpu_baseline": None,
    }
    say(f"timed: {value:.0f} entries/s, {ms:.0f} ms per estimate of {nk} samples, plug-in "
        f"error {err:.4f}")

    def budget_ok(est_s, name):
        left = args.budget_s - (time.perf_counter() - t_start)
        if est_s <= left:
            return True
        out.setdefault("skipped_legs", {})[name] = (
            f"projected {est_s:.0f} s, {max(left, 0):.0f} s left of the {args.budget_s:.0f} s budget")
        say(f"skipping leg {name}: projected {est_s:.0f} s, {left:.0f} s left")
        return False

    d_stated = d_mixed = d_alg2 = d_alg2_timed = None
    for leg in legs:
        if leg == "stated":
            if not budget_ok(3.0 * rep0.t_total, "stated") or not gm.m:
                continue
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, _, rs = estimate(opts_for(wl.n_k, passes=False))
            torch.cuda.synchronize()
            sec = time.perf_counter() - ta
            d_stated = diag.clone()
            out["stated_setting"] = {
                "n_samples": wl.n_k, "value": gm.n / sec, "ms_per_estimate": sec * 1e3,
                "err_estimate": rs.err_estimate, "accuracy_gate_1pct": bool(rs.err_estimate <= 0.01),
                "pcg_iters": {"mean": rs.pcg_it_mean, "max": rs.pcg_it_max},
                "phase_s": {k: getattr(rs, k) for k in ("t_sample", "t_factor", "t_correct",
                                                        "t_total")}}
            say(f"stated setting: {sec:.2f} s, plug-in error {rs.err_estimate:.4f}")
        elif leg == "mixed":
            # the timed estimate under RBMC_MIXED (the correction products on
            # the FP32 matrix cores, the sampler in FP64): same sample count,
            # passes and z
            if not budget_ok(2.2 * ms / 1000.0, "mixed") or not gm.m:
                continue
            om = opts_for(nk, precision=B.RBMC_MIXED)
            estimate(om)  # warm-up: loads the mixed kernels
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, trm, rm = estimate(om)
            torch.cuda.synchronize()
            sec = time.perf_counter() - ta
            d_mixed = diag.clone()
            rel_d = (d_mixed - d_head).abs() / d_head
            out["mixed"] = {
                "n_samples": nk, "value": gm.n / sec, "ms_per_estimate": sec * 1e3,
                "speedup_vs_fp64": ms / (sec * 1e3),
                "precision": "mixed (FP32 matrix-core correction products)",
                "err_estimate": rm.err_estimate,
                "pcg_iters": {"mean": rm.pcg_it_mean, "max": rm.pcg_it_max},
                "phase_s": {k: getattr(rm, k) for k in ("t_sample", "t_factor", "t_correct",
                                                        "t_total")},
                "diag_rel_diff_vs_fp64": {"mean": float(rel_d.mean()),
                                          "max": float(rel_d.max())},
                "trace_rel_diff_vs_fp64": [abs(a - b) / abs(b) for a, b in zip(trm, tr)]}
            say(f"mixed: {sec:.2f} s ({ms / (sec * 1e3):.3f}x), {rm.pcg_it_max} PCG "
                f"iterations, diag vs FP64 mean {float(rel_d.mean()):.2e}")
        elif leg == "probe":
            # the overlap suggested by the posterior correlation range at the
            # domain centre (one solve), against the workload's n_l
            if not budget_ok(30.0, "probe") or not gm.m:
                continue
            torch.cuda.synchronize()
            ta = time.perf_counter()
            pr = {}
            for eps in (1e-1, 1e-2, 1e-3):
                st, lags, _, _ = B.rbmc_probe_overlap(
                    gm.m, B.make_opts(1, 500, 1e-12, precond=B.RBMC_PC_SPECTRAL), eps)
                pr[f"{eps:g}"] = {"time_lag": int(lags[0]), "space_lag": int(lags[1]),
                                  "suggested_overlap_hops": int(lags[2])}
            sec = time.perf_counter() - ta
            out["probe"] = {"workload_overlap_hops": wl.n_l, "by_eps": pr, "seconds": sec,
                            "solve_rtol": 1e-12}
            say(f"probe: {pr} in {sec:.1f} s (workload n_l = {wl.n_l})")
        elif leg == "mean":
            # the posterior mean with four fixed effects (an intercept and
            # three seeded covariates; Sec. 3.1) and the fixed-effects variance
            # term, on the timed model, spectral preconditioner, the
            # workload's tolerance
            if not budget_ok(30.0, "mean") or not gm.m:
                continue
            import numpy as np
            try:
                nbeta = 4
                y = torch.from_numpy(normals(gm.n_obs, seed + 11)).cuda()
                a = normals((nbeta, gm.n_obs), seed + 12)
                a[0] = 1.0
                a = torch.from_numpy(a).cuda()
                q = np.full(nbeta, 0.01)
                secs = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    ta = time.perf_counter()
                    mu, mb, vb, va, st, rm = gm.posterior_mean(
                        y, a, q, rtol=wl.rtol, maxit=500, precond=B.RBMC_PC_SPECTRAL)
                    torch.cuda.synchronize()
                    secs.append(time.perf_counter() - ta)
                out["mean"] = {"n_beta": nbeta, "seconds_median": float(np.median(secs)),
                               "seconds": secs, "value": gm.n / float(np.median(secs)),
                               "unit": "posterior-mean entries/s (with diag(Var(u)) term)",
                               "pcg_rtol": wl.rtol, "pcg_iters": rm.pcg_it_max,
                               "solve_columns": nbeta + 1, "status": st,
                               "mu_beta": [float(v) for v in mb],
                               "var_beta_diag": [float(v) for v in np.diag(vb)]}
                del mu, va, y, a
                say(f"mean: {np.median(secs) * 1e3:.1f} ms per call, {rm.pcg_it_max} PCG "
                    f"iterations, mu_beta {mb}")
            except Exception as ex:  # recorded, the other legs still run
                out["mean"] = {"error": repr(ex)}
                say(f"mean: failed: {ex!r}")
        elif leg == "grad":
            # the gradient of log pi(theta | y) (no fixed effects, flat prior;
            # Sec. 3.4) with the configuration's samples drawn on the device:
            # the posterior mean, the estimator's traces, the mu terms
            if not budget_ok(30.0, "grad") or not gm.m:
                continue
            import numpy as np
            try:
                y = torch.from_numpy(normals(gm.n_obs, seed + 11)).cuda()
                kw = dict(n_samples=wl.n_k, seed=seed, rtol=wl.rtol, maxit=500,
                          precond=B.RBMC_PC_SPECTRAL, method=B.RBMC_SEL_KRON)
                gm.grad_log_posterior(y, **kw)  # warm-up
                torch.cuda.synchronize()
                ta = time.perf_counter()
                g, terms, mu, st, rg = gm.grad_log_posterior(y, **kw)
                torch.cuda.synchronize()
                sec = time.perf_counter() - ta
                out["grad"] = {"n_samples": wl.n_k, "seconds": sec, "status": st,
                               "theta": ["log_kappa", "log_tau", "rho", "log_sigma"],
                               "grad": [float(v) for v in g],
                               "terms": [[float(v) for v in row] for row in terms],
                               "pcg_iters": rg.pcg_it_max, "err_estimate": rg.err_estimate}
                del mu, y
                say(f"grad: {sec:.2f} s, gradient {g}")
            except Exception as ex:  # recorded, the other legs still run
                out["grad"] = {"error": repr(ex)}
                say(f"grad: failed: {ex!r}")
        elif leg == "alg2":
            import numpy as np
            # the non-overlapping variant (Alg. 2: separator layers between the
            # same slabs and tiles, plain Monte Carlo on them) at the
            # configuration's sample count, diagonal only; its own model
            if not budget_ok(90.0, "alg2"):
                continue
            if gm.m:
                gm.close()
            torch.cuda.empty_cache()
            ga = B.Model(wl, decomp=(wl.n_tslabs, wl.n_tiles, wl.n_tiles, 0, 0, 0, 0, 1),
                         pc=None)
            da = torch.empty(ga.n, dtype=torch.float64, device="cuda")
            lab = np.zeros(ga.n, np.int32)
            B.rbmc_plan_query(ga.desc, ga.decomp, 0, label_out=lab)
            res = {}
            # the configuration's samples, then the timed estimate's (passes of chunk)
            for key, nka in (("stated", wl.n_k), ("timed", nk)):
                oa = B.make_opts(nka, pcg_maxit=500, pcg_rtol=wl.rtol, grad_mask=0,
                                 precond=B.RBMC_PC_SPECTRAL, method=B.RBMC_SEL_KRON,
                                 sample_chunk=chunk if nka > chunk else 0)
                if key == "stated":
                    B.rbmc_estimate(ga.m, oa, None, seed, da, 0)  # warm-up: loads and sizes
                torch.cuda.synchronize()
                ta = time.perf_counter()
                _, _, ra = B.rbmc_estimate(ga.m, oa, None, seed, da, 0)
                torch.cuda.synchronize()
                sec = time.perf_counter() - ta
                res[key] = {"n_samples": nka, "value": ga.n / sec, "ms_per_estimate": sec * 1e3,
                            "err_estimate": ra.err_estimate}
                if key == "stated":
                    d_alg2 = da.clone()
                else:
                    d_alg2_timed = da.clone()
                say(f"alg2, {nka} samples: {sec:.2f} s, plug-in error {ra.err_estimate:.4f}")
            out["alg2"] = dict(res["stated"], separator_nodes=int((lab < 0).sum()),
                               overlap_estimate_err_estimate=out.get("stated_setting", {})
                               .get("err_estimate"), at_timed_samples=res["timed"])
            out["alg2_timed"] = res["timed"]
            ga.close()
            del da
            torch.cuda.empty_cache()
        elif leg == "true_error":
            if not budget_ok(60.0, "true_error"):
                continue
            # exact (Q^-1)_ii at uniformly drawn nodes: PCG solves Q y = e_i to
            # 1e-12 with the spectral preconditioner, exact = y_i
            # (a model of its own: the timed model's context holds the estimate's
            # workspaces, sized to the free device memory)
            import numpy as np
            if gm.m:
                gm.close()
            torch.cuda.empty_cache()
            gs = B.Model(wl)
            rng = np.random.default_rng(seed + 7)
            nodes = np.sort(rng.choice(gs.n, size=args.true_error_nodes, replace=False))
            exact = np.empty(len(nodes))
            it_max = 0
            ta = time.perf_counter()
            for b0 in range(0, len(nodes), 64):
                nb = nodes[b0:b0 + 64]
                E = torch.zeros((len(nb), gs.n), dtype=torch.float64, device="cuda")
                E[torch.arange(len(nb)), torch.from_numpy(nb).cuda()] = 1.0
                y, st, rs = gs.solve(E, rtol=1e-12, maxit=2000, precond=B.RBMC_PC_SPECTRAL)
                it_max = max(it_max, rs.pcg_it_max)
                exact[b0:b0 + len(nb)] = y[torch.arange(len(nb)), torch.from_numpy(nb).cuda()] \
                    .cpu().numpy()
                del E, y
            sec = time.perf_counter() - ta
            te = {"nodes": len(nodes), "node_seed": seed + 7, "solve_rtol": 1e-12,
                  "solve_pcg_iters_max": it_max, "seconds": sec}
            for name, d in (("timed", d_head), ("stated", d_stated), ("mixed", d_mixed),
                            ("alg2", d_alg2), ("alg2_timed", d_alg2_timed)):
                if d is None:
                    continue
                est = d[torch.from_numpy(nodes).cuda()].cpu().numpy()
                rel = np.abs(est - exact) / exact
                te[name] = {"mean_rel_err": float(rel.mean()),
                            "stderr": float(rel.std(ddof=1) / math.sqrt(len(rel))),
                            "max_rel_err": float(rel.max()),
                            "plugin_err": err if name == "timed" else
                            out.get({"stated": "stated_setting"}.get(name, name), {})
                            .get("err_estimate")}
            out["true_error"] = te
            out["accuracy_gate_1pct_true"] = bool(te["timed"]["mean_rel_err"] <= 0.01)
            gs.close()
            torch.cuda.empty_cache()
            say(f"true error at {len(nodes)} nodes: {te['timed']['mean_rel_err']:.4f} "
                f"(+- {te['timed']['stderr']:.4f}), {sec:.1f} s")
        elif leg == "cpu":
            if not budget_ok(90.0, "cpu"):
                continue
            out["cpu_baseline"] = (cpu_baseline_entry(wl) if wl.name == "tile512"
                                   else cpu_baseline(wl, args.cpu_sample_m))
            say("cpu baseline done")
        elif leg == "plain":
            if not budget_ok(args.plain_est_s, "plain"):
                continue
            # the plain method: FP64, block-Jacobi PCG (whole time chains of
            # spatial tiles, factored block-tridiagonally), same z, same subdomain
            # method, the workload's own sample count; its own model (the timed
            # model's workspaces released)
            if gm.m:
                gm.close()
            torch.cuda.empty_cache()
            pc = None if args.pc == "cores" else tuple(int(v) for v in args.pc.split(","))
            mp = B.Model(wl, pc=pc)
            op = B.make_opts(wl.n_k, pcg_maxit=5000, pcg_rtol=wl.rtol, grad_mask=grad,
                             precond=B.RBMC_PC_BJ, method=B.RBMC_SEL_KRON)
            dp = torch.empty(mp.n, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, trp, rp = B.rbmc_estimate(mp.m, op, None, seed, dp, B.popcount(grad))
            torch.cuda.synchronize()
            sec = time.perf_counter() - ta
            per_pass = rp.t_sample + rp.t_correct
            proj = rp.t_factor + (nk // chunk) * per_pass
            out["plain"] = {
                "n_samples": wl.n_k, "value": mp.n / sec, "ms_per_estimate": sec * 1e3,
                "precision": "fp64", "precond": "block-jacobi",
                "pc_blocks": list(pc) if pc else "cores",
                "pcg_iters": {"mean": rp.pcg_it_mean, "max": rp.pcg_it_max},
                "phase_s": {k: getattr(rp, k) for k in ("t_sample", "t_factor", "t_correct",
                                                        "t_total")},
                "err_estimate": rp.err_estimate,
                "max_rel_diff_diag_vs_stated": (float(((dp - d_stated).abs() / d_stated).max())
                                                if d_stated is not None else None),
                "speedup_of_stated_setting": (sec / (out["stated_setting"]["ms_per_estimate"]
                                                     / 1000.0)
                                              if "stated_setting" in out else None),
                "projected_s_at_timed_samples": proj,
                "projected_value_at_timed_samples": mp.n / proj,
                "projection": "factor once + passes x (sampling + correction) of this run"}
            say(f"plain leg: {sec:.1f} s, {rp.pcg_it_max} PCG iterations")
            mp.close()
            del dp
            torch.cuda.empty_cache()
        elif leg == "batched":
            if not budget_ok(60.0, "batched"):
                continue
            if gm.m:
                gm.close()
            torch.cuda.empty_cache()
            try:
                out["batched"] = batched_leg(args.batched_models,
                                             None if args.no_autotune else args.tune_cache)
            except B.RbmcError as e:  # e.g. device memory: report, keep the main line
                out["batched"] = {"error": str(e)}
            say("batched leg done")
    out["wall_s"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)


def learned_leg(wl, pc=(4, 2, 2), n_train=8, n_cols=32):
    """The learned correction of the block-Jacobi preconditioner on the same
    grid with tiled blocks (4 slabs x 2 x 2 tiles: block Jacobi alone needs
    several hundred iterations, the most room for a correction): training
    (pairs from n_train columns, a quarter held out), its acceptance trial,
    then n_cols samples with block Jacobi alone and with the trained
    correction applied (forced, whatever the trial decided)."""
    import torch
    from paper_2309_05435_amd import binding as B
    from paper_2309_05435_amd.inputs import normals
    gm = B.Model(wl, pc=pc)
    zt = torch.from_numpy(normals((n_train, gm.n + gm.n_obs), 71)).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, loss, rep = B.rbmc_precond_train(
        gm.m, B.make_opts(n_train, 20000, wl.rtol),
        B.make_train_opts(n_pairs=1000, epochs=8, batch=8, lr=2e-3, seed=3), zt, n_train)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    info = B.rbmc_precond_info(gm.m)
    B.rbmc_precond_set_weights(gm.m, B.rbmc_precond_get_weights(gm.m))  # force use
    z = torch.from_numpy(normals((n_cols, gm.n + gm.n_obs), 72)).to("cuda")
    x = torch.empty((n_cols, gm.n), dtype=torch.float64, device="cuda")
    runs = {}
    for name, pcv in (("block_jacobi", B.RBMC_PC_BJ), ("learned", B.RBMC_PC_BJ_LEARNED)):
        o = B.make_opts(n_cols, 20000, wl.rtol, precond=pcv)
        B.rbmc_sample(gm.m, o, z, x)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        _, rp = B.rbmc_sample(gm.m, o, z, x)
        torch.cuda.synchronize()
        runs[name] = {"pcg_iters_max": rp.pcg_it_max, "sampler_s": time.perf_counter() - ta,
                      "max_rel_residual": rp.max_rel_residual}
    gm.close()
    return {"pc_blocks": list(pc), "train_s": t_train, "train_ratios": loss[:-1],
            "heldout_energy_ratio": info.val_ratio, "accepted": bool(info.usable),
            "trial_iters": [info.trial_it_bj, info.trial_it_learned],
            "trial_s": [info.trial_s_bj, info.trial_s_learned], "n_samples": n_cols, **runs}


if __name__ == "__main__":
    main()
