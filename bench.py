"""Throughput benchmark of the RBMC hot path on one MI355X.

A step is one full estimate on the 64 x 64 x 32 space-time workload
(n = 131,072, 500 samples, 16 time slabs, 2-hop overlap, PCG to 1e-8):
rebuild Q(theta), sample x = Q^-1 F z by block-Jacobi PCG, factor every
overlapping subdomain, run the Takahashi sweep, the correction solves and
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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6    # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


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


def batched_leg(n_models: int):
    """The uneven-model workload (grids 16^2-48^2, T 8-24, 2-8 slabs, 1-step
    overlap, 100 samples): all models in one rbmc_estimate_batched call against
    the same models estimated one call each.  Each timing follows a warm-up."""
    import torch

    from paper_2309_05435_amd import binding as B
    from paper_2309_05435_amd.inputs import batched_models

    wls = batched_models(n_models)
    ms = B.ModelSet(wls)
    zs = [torch.from_numpy(wl.z()).to("cuda") for wl in wls]
    n_tot = sum(ms.n)
    res = {"workload": f"{n_models} uneven models, sum n = {n_tot}", "n_models": n_models,
           "n_samples": wls[0].n_k}

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
    sec_e, (de, te, sts, reps) = timed(run_each)
    dev = max(float(((a - b).abs() / b.abs()).max()) for a, b in zip(db, de))
    res.update({"value": n_tot / sec_b, "unit": "entries/s", "ms_per_step": sec_b * 1e3,
                "per_model_calls": {"value": n_tot / sec_e, "ms_per_step": sec_e * 1e3},
                "speedup": sec_e / sec_b, "max_rel_diff_vs_per_model": dev,
                "err_estimate": rep.err_estimate, "pcg_iters_max": rep.pcg_it_max,
                "phase_s": {k: getattr(rep, k) for k in ("t_sample", "t_factor", "t_takahashi",
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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    B.rbmc_ctx_profile(gm.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        st, tr, rep = step()
        reps.append(rep.as_dict())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = {B.KF_NAMES[f]: B.rbmc_ctx_profile_read(gm.ctx, f) for f in range(B.RBMC_KF_COUNT)}
    B.rbmc_ctx_profile(gm.ctx, False)
    ms = (t1 - t0) * 1000.0 / args.steps
    value = gm.n / (ms / 1000.0)

    # dominant kernel family by device time
    dom = max(stats, key=lambda k: stats[k]["total_ms"])
    s = stats[dom]
    if dom in ("gemm", "spd_inverse"):
        achieved = s["alg_flops"] / (s["total_ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS}
    else:
        achieved = s["alg_bytes"] / (s["total_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    roof["kernel"] = dom
    roof["launches"] = s["launches"] // max(args.steps, 1)
    roof["avg_launch_ms"] = s["total_ms"] / max(s["launches"], 1)
    roof["traffic"] = traffic_for(dom, wl.name)

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
        "phase_s": {k: last[k] for k in ("t_sample", "t_factor", "t_takahashi", "t_correct",
                                         "t_total")},
        "kernel_ms_per_step": {k: v["total_ms"] / args.steps for k, v in stats.items()},
        "roofline": roof,
        "cpu_baseline": None,
    }
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
    if not args.no_batched:
        out["batched"] = batched_leg(args.batched_models)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
