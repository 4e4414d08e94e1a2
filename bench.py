"""Benchmark of the REXII shifted-solve path on one MI355X.

One step = one complete u = exp(tA) f (all poles: coefficients, every shifted
solve, the weighted FP64 sum, reconstruction) for the 512 x 512 linear
rotating shallow-water workload: centred differences, g = H = 1, f_c = 10,
t rho = 1000, initial height a sum of 16 seeded Gaussian bumps, zero initial
velocity; FP32 inner Krylov iterations with FP64 residuals, refinement,
weights and pole sum (tol 1e-6).  Inputs are resident in HBM before the
timed region.

Prints one JSON line (see the keys at the bottom).  Also reported:
  * the all-FP64 path on the same workload (one untimed-warm run),
  * roofline of the dominant kernel (k_pass_f32: one COCG step or FP64
    residual round of every live solve), timed with HIP events on the
    stream it runs on,
  * the CPU oracle's per-mode REXII on a bounded sample of poles.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-pt·pole solves/s + HBM GB/s at rel-L2 ≤1e-6 vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
D = 512
TRHO = 1000.0
FC = 10.0
NBUMPS = 16
SEED = 2


def workload():
    from paper_2008_11607_amd import inputs
    from paper_2008_11607_amd import rexii
    f = inputs.gaussian_bumps(D, nbumps=NBUMPS, seed=SEED)
    rho = rexii.rho(D, D, fc=FC)
    return f, rho, TRHO / rho


def cpu_baseline(f, t, budget_s=12.0):
    """The oracle's per-mode REXII (one batched 3x3 solve per pole over all
    D^2 Fourier modes, numpy), on the leading poles of the same pole set
    until the time budget is spent."""
    from oracle import coeffs as oc
    from oracle import lrsw
    from oracle import rexii_modes as rm
    op = lrsw.LRSW(D, D, fc=FC)
    c = oc.api_coeffs(t, lrsw.rho(op), h=0.5, tol=1e-6)
    done = 0
    t0 = time.perf_counter()
    step = 8
    while time.perf_counter() - t0 < budget_s and done < len(c["z"]):
        sl = slice(done, done + step)
        rm.rexii_direct(op, f, t, c["z"][sl], c["w"][sl])
        done += len(c["z"][sl])
    el = time.perf_counter() - t0
    return {"value": done * D * D / el, "unit": "grid-pt·pole solves/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle per-mode REXII (exact 3x3 solve per pole and Fourier mode, numpy, single "
                      f"thread) on the first {done} of {len(c['z'])} poles of the same 512x512 workload, "
                      f"{el:.1f} s"}


def copy_calibration(nbytes=1 << 30, reps=8):
    """A copy of known size (nbytes read + nbytes written per launch): the
    per-dispatch FETCH_SIZE / WRITE_SIZE it reports scale the counters of
    the solver kernels to bytes."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison run")
    ap.add_argument("--slots", type=int, default=-1,
                    help="concurrent solves; -1 (default) autotunes on the first call and caches the choice")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 8 times (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the pole-sharded multi-GPU "
              "form is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2008_11607_amd import rexii
    from oracle import expm_modes as em
    from oracle import lrsw

    f, rho, t = workload()
    fd = torch.from_numpy(f).cuda()
    # pole_batch=-1: slot count autotuned on the first (warm-up) call, cached
    opts = dict(fc=FC, precision="mixed", tol=1e-6, profile=1, pole_batch=args.slots)
    for _ in range(args.warmup):
        rexii.apply(fd, t, **opts)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        u, rep = rexii.apply(fd, t, **opts)
        reps.append(rep)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1000.0 * el / args.steps
    P = reps[0]["P"]
    value = D * D * P / (el / args.steps)

    op = lrsw.LRSW(D, D, fc=FC)
    ref = em.expm_closed_real(op, f, t)
    err = em.rel_l2(u.cpu().numpy(), ref)

    k_l = sum(r["kernel_launches"] for r in reps)
    k_ms = sum(r["kernel_ms"] for r in reps)
    k_b = sum(r["kernel_bytes"] for r in reps)
    achieved = (k_b / k_l) / (k_ms / k_l * 1e-3) / 1e9
    alg_gbs = sum(r["alg_bytes"] for r in reps) / el / 1e9

    out = {
        "metric": METRIC, "value": value, "unit": "grid-pt·pole solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "lrsw-fd-512x512-trho1000-16bumps", "D": D, "t_rho": TRHO, "f_c": FC,
                   "precision": "mixed (FP32 inner COCG, FP64 residual/refinement/pole sum)", "tol": 1e-6,
                   "P": P, "solves": reps[0]["solves"], "h": 0.5, "slots": reps[0]["slots"]},
        "rel_l2_vs_oracle": err,
        "hbm_gbs_alg": alg_gbs,
        "krylov": {"total_iters": reps[0]["total_iters"], "max_iters": reps[0]["max_iters"],
                   "max_refine": reps[0]["max_refine"], "kappa_sum": reps[0]["kappa_sum"],
                   "pole_tol": reps[0]["pole_tol"], "max_rel_residual": reps[0]["max_rel_residual"]},
        "roofline": {"bound": "hbm", "kernel": "k_pass_f32", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "avg_launch_ms": k_ms / k_l, "launches": k_l,
                     "alg_bytes_per_launch": k_b / k_l,
                     "kernel_time_share": k_ms * 1e-3 / el},
    }
    if not args.no_fp64:
        rexii.apply(fd, t, fc=FC, precision="fp64", tol=1e-10, pole_batch=-1)   # tune
        t1 = time.perf_counter()
        u64, r64 = rexii.apply(fd, t, fc=FC, precision="fp64", tol=1e-10, pole_batch=-1)
        torch.cuda.synchronize()
        e64 = time.perf_counter() - t1
        out["fp64"] = {"value": D * D * r64["P"] / e64, "ms": 1000 * e64, "P": r64["P"],
                       "rel_l2_vs_oracle": em.rel_l2(u64.cpu().numpy(), ref),
                       "total_iters": r64["total_iters"], "max_iters": r64["max_iters"]}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(f, t)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
