"""Throughput benchmark of the RBMC hot path on one MI355X.

A step is one full estimate on the 64 x 64 x 32 space-time workload
(n = 131,072, 500 samples, 16 time slabs, 2-hop overlap, PCG to 1e-8):
rebuild Q(theta), sample x = Q^-1 F z by block-Jacobi PCG, factor every
overlapping subdomain, form the selected inverse entries, the correction solves and
the trace/diagonal accumulation.  Inputs (z) are resident in HBM before the
timed region.  Prints one JSON line.

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
KERNEL_OF = {"gemm": "k_gemm_f64", "gemm_small": "k_gemm_f64s", "gemm_mixed": "k_gemm_mx",
             "inv_small": "k_inv128", "spmm": "k_space_time_op", "rstencil": "k_rstencil",
             "panels": "k_panels", "spd_inverse": "gauss_jordan", "offdiag": "k_offdiag"}


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
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
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
        tail = r"<0, true>\(" if kern == "k_space_time_op" else r"[<(]"
        pat = re.compile(r"(^|[\s:])" + re.escape(kern) + tail)
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
        path = os.path.join(ROOT, "profiles", f"traffic_{kern}_{workload}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        written.append(path)
    print(json.dumps({"written": written}))


def cpu_baseline(wl, m_sample: int):
    """The CPU oracle, as it stands, on the same workload with the spatial grid
    reduced to m_sample^2 (full pipeline: exact sampling + estimator)."""
    import numpy as np
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
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="slab64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-m", type=int, default=24)
    ap.add_argument("--pc", default="workload",
                    help="block-Jacobi blocks 'slabs,tiles_x,tiles_y', 'cores', or 'workload' "
                         "(the workload's tuned shape)")
    ap.add_argument("--no-gate", action="store_true",
                    help="skip the run at the sample count that reaches <= 1%% error")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the run with block-Jacobi blocks equal to the cores")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-model batched workload")
    ap.add_argument("--batched-models", type=int, default=256)
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched workload and print its JSON")
    ap.add_argument("--no-per-model", action="store_true",
                    help="batched workload without the one-call-per-model comparison")
    ap.add_argument("--calibration-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (no rbmc_autotune before timing)")
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

    import numpy as np
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
    from paper_2309_05435_amd.inputs import WORKLOADS

    wl = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.pc == "workload":
        pc = wl.pc
    elif args.pc == "cores":
        pc = None
    else:
        pc = tuple(int(v) for v in args.pc.split(","))
    gm = B.Model(wl, pc=pc)
    z = torch.from_numpy(wl.z()).to("cuda")
    diag = torch.empty(gm.n, dtype=torch.float64, device="cuda")
    grad = 0b111
    opts = B.make_opts(wl.n_k, pcg_maxit=5000, pcg_rtol=wl.rtol, grad_mask=grad)
    theta = wl.theta

    def step():
        # rebuilding Q(theta) invalidates every factor: each step factors again
        B.rbmc_model_set_theta(gm.m, *theta)
        return B.rbmc_estimate(gm.m, opts, z, 0, diag, B.popcount(grad))

    def timed_once(model, n_k, zz, reps=1):
        """warm-up call, then `reps` timed calls; returns (seconds per call, report)."""
        o = B.make_opts(n_k, pcg_maxit=5000, pcg_rtol=wl.rtol, grad_mask=grad)
        d = torch.empty(model.n, dtype=torch.float64, device="cuda")
        B.rbmc_model_set_theta(model.m, *theta)
        B.rbmc_estimate(model.m, o, zz, 0, d, B.popcount(grad))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            B.rbmc_model_set_theta(model.m, *theta)
            _, _, rp = B.rbmc_estimate(model.m, o, zz, 0, d, B.popcount(grad))
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, rp.as_dict()

    tune = None
    if not args.no_autotune:
        # launch shapes chosen by the autotuner (end-to-end timing of this
        # workload, or its cached choice), outside the timed steps
        tr_ = B.rbmc_autotune(gm.ctx, [gm.m], opts, [z], args.tune_cache)
        tune = tune_dict(tr_)
    for i in range(args.warmup):
        step()
        print(f"warm-up step {i + 1} of {args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    B.rbmc_ctx_profile(gm.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(args.steps):
        st, tr, rep = step()
        reps.append(rep.as_dict())
        print(f"step {i + 1} of {args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = {B.KF_NAMES[f]: B.rbmc_ctx_profile_read(gm.ctx, f) for f in range(B.RBMC_KF_COUNT)}
    B.rbmc_ctx_profile(gm.ctx, False)
    ms = (t1 - t0) * 1000.0 / args.steps
    value = gm.n / (ms / 1000.0)

    def roofline(fam):
        s = stats[fam]
        per_launch = 1.0 / max(s["launches"], 1)
        if fam in ("gemm", "gemm_small", "gemm_mixed", "inv_small"):
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
        r["launches_per_step"] = s["launches"] // max(args.steps, 1)
        r["avg_launch_ms"] = s["total_ms"] * per_launch
        return r

    # dominant single kernel: the largest speed-of-light time per step
    # (algorithmic flops / peak, or bytes / HBM peak).  Event times do not rank
    # kernels here: three streams overlap, and a kernel's event time includes
    # waiting for compute units held by the other streams (the 128-order
    # register inversion takes 70 us alone, 4-5 times that in the overlapped
    # step).  The inversion family is a composite of several kernels whose
    # products are counted under the GEMM families.
    def ideal_ms(fam):
        s = stats[fam]
        if fam in ("gemm", "gemm_small", "gemm_mixed", "inv_small"):
            peak = PEAK_FP32_TFLOPS if fam == "gemm_mixed" else PEAK_FP64_TFLOPS
            return s["alg_flops"] / (peak * 1e12) * 1e3
        return s["alg_bytes"] / (PEAK_HBM_GBS * 1e9) * 1e3

    singles = [k for k in stats if k != "spd_inverse" and stats[k]["launches"] > 0]
    dom = max(singles, key=ideal_ms)
    roof = roofline(dom)
    roof["ideal_ms_per_step"] = ideal_ms(dom) / max(args.steps, 1)
    others = {KERNEL_OF[k]: dict(roofline(k), ideal_ms_per_step=ideal_ms(k) / max(args.steps, 1))
              for k in singles if k != dom}

    last = reps[-1]
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
                   "n_obs": gm.n_obs, "n_samples": wl.n_k, "n_tslabs": wl.n_tslabs,
                   "n_tiles": wl.n_tiles, "overlap_hops": wl.n_l, "pcg_rtol": wl.rtol,
                   "precision": "fp64", "precond": "block-jacobi",
                   "pc_blocks": list(pc) if pc else "cores", "traces": "logkappa,logtau,rho"},
        "pcg_iters": {"mean": last["pcg_it_mean"], "max": last["pcg_it_max"]},
        "err_estimate": last["err_estimate"],
        "accuracy_gate_1pct": bool(last["err_estimate"] <= 0.01),
        "phase_s": {k: last[k] for k in ("t_sample", "t_factor", "t_select", "t_correct",
                                         "t_total")},
        "kernel_ms_per_step": {k: v["total_ms"] / args.steps for k, v in stats.items()},
        "roofline": roof,
        "rooflines_other_kernels": others,
        "cpu_baseline": None,
        "tune": tune,
    }
    if not args.no_variants:
        # RBMC_MIXED on the same model and samples: FP32 matrix-core products in
        # the correction solves; error stated against the FP64 run
        d64 = diag.clone()
        t64 = list(tr)
        om = B.make_opts(wl.n_k, pcg_maxit=5000, pcg_rtol=wl.rtol, grad_mask=grad,
                         precision=B.RBMC_MIXED)
        dm = torch.empty_like(diag)
        B.rbmc_model_set_theta(gm.m, *theta)
        B.rbmc_estimate(gm.m, om, z, 0, dm, B.popcount(grad))
        torch.cuda.synchronize()
        B.rbmc_ctx_profile(gm.ctx, True)
        ta = time.perf_counter()
        B.rbmc_model_set_theta(gm.m, *theta)
        _, trm, rpm = B.rbmc_estimate(gm.m, om, z, 0, dm, B.popcount(grad))
        torch.cuda.synchronize()
        sec = time.perf_counter() - ta
        sm = {B.KF_NAMES[f]: B.rbmc_ctx_profile_read(gm.ctx, f) for f in range(B.RBMC_KF_COUNT)}
        B.rbmc_ctx_profile(gm.ctx, False)
        g = sm["gemm_mixed"]
        out["variant_mixed"] = {
            "value": gm.n / sec, "ms_per_step": sec * 1e3,
            "max_rel_err_diag_vs_fp64": float(((dm - d64).abs() / d64).max()),
            "mean_rel_err_diag_vs_fp64": float(((dm - d64).abs() / d64).mean()),
            "rel_err_traces_vs_fp64": [abs(a - b) / abs(b) for a, b in zip(trm, t64)],
            "pcg_iters": {"mean": rpm.pcg_it_mean, "max": rpm.pcg_it_max},
            "phase_s": {k: getattr(rpm, k) for k in ("t_sample", "t_factor", "t_select",
                                                     "t_correct", "t_total")},
            "kernel_ms": {k: v["total_ms"] for k, v in sm.items()},
            "gemm_mixed_tflops": (g["alg_flops"] / (g["total_ms"] * 1e-3) / 1e12
                                  if g["total_ms"] > 0 else None),
            "gemm_mixed_peak_tflops": PEAK_FP32_TFLOPS}
    gm.close()
    del z
    torch.cuda.empty_cache()
    if not args.no_gate:
        # the plug-in error falls as 1/sqrt(n_k): the sample count for <= 1% (with margin)
        err = last["err_estimate"]
        if err <= 0.0095:
            out["accuracy_gate"] = {"n_samples": wl.n_k, "value": value, "err_estimate": err}
        else:
            nk_g = int(math.ceil(wl.n_k * (err / 0.0095) ** 2 / 100.0)) * 100
            mg = B.Model(wl, pc=pc)
            zg = torch.from_numpy(wl.z(nk_g)).to("cuda")
            sec, rp = timed_once(mg, nk_g, zg)
            out["accuracy_gate"] = {"n_samples": nk_g, "value": gm.n / sec, "ms_per_step": sec * 1e3,
                                    "err_estimate": rp["err_estimate"],
                                    "met": bool(rp["err_estimate"] <= 0.01),
                                    "pcg_iters": {"mean": rp["pcg_it_mean"], "max": rp["pcg_it_max"]}}
            mg.close()
            del zg
            torch.cuda.empty_cache()
    if not args.no_variants and pc is not None:
        # the preconditioner blocks equal to the cores (16 slabs of 2 steps)
        mv = B.Model(wl, pc=None)
        zv = torch.from_numpy(wl.z()).to("cuda")
        sec, rp = timed_once(mv, wl.n_k, zv)
        out["variant_pc_cores"] = {"value": mv.n / sec, "ms_per_step": sec * 1e3,
                                   "pcg_iters": {"mean": rp["pcg_it_mean"], "max": rp["pcg_it_max"]}}
        mv.close()
    if not args.no_variants:
        try:
            out["variant_learned"] = learned_leg(wl)
        except B.RbmcError as e:
            out["variant_learned"] = {"error": str(e)}
    if not args.no_batched:
        try:
            out["batched"] = batched_leg(args.batched_models,
                                         None if args.no_autotune else args.tune_cache)
        except B.RbmcError as e:  # e.g. device memory: report, keep the main line
            out["batched"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_m)
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
