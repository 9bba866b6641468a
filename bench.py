"""Benchmark: omega-point solves per second of the batched mixed-precision solve on one MI355X.

Workload (cnt20k): armchair (10,10) carbon nanotube, 500 periods = 20 000 atoms, jitter 0.01 A
(seed 2), graphene parameters (eps_F = 0.4 eV, tau = 170 a.u., d = 12, s = 1.1), 64 frequencies
uniform in 0.05-1.0 eV x 3 field polarisations = 192 systems sharing one stored T. One step = one
wfq_solve over all 192 systems: FP32 T products inside restarted GMRES(50) with FP64 refinement to
relative FP64 residual 1e-8. T and L are built (and resident in HBM) before the timed region.

Printed (one JSON line): solves/s, p50/p99 per-system completion latency inside a step, the
largest relative difference of q against the FP64 solve on the same GPU, the per-frequency FP64
baseline (one system per solve, same library), the roofline figures of the dominant kernel (FP32
MFMA block product, timed with HIP events on the library's stream) and the CPU oracle timed on a
bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}   # TFLOP/s, dense MFMA (MI355X)
HBM_PEAK = 8000.0                                        # GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cnt20k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference", action="store_true", help="skip the FP64 comparison runs")
    ap.add_argument("--precision", default=None)
    return ap.parse_args()


def cpu_baseline(wl, sys_index):
    """The oracle as it stands: FP64 restarted GMRES on one system of the workload (host cores)."""
    from oracle import wfq_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    P = O.Problem(wl.xyz, wl.params)
    t_build = time.perf_counter() - t0
    a, k = divmod(sys_index, len(wl.dirs))
    t0 = time.perf_counter()
    x, info = P.solve_gmres(wl.omegas_eV[a], wl.dirs[k], wl.restart, wl.tol)
    t_solve = time.perf_counter() - t0
    return dict(value=1.0 / t_solve, unit="solves/s", cores=cores, kind="oracle",
                sample=f"1 of {wl.n_systems} systems (omega={wl.omegas_eV[a]:.4f} eV, dir {k}), FP64 GMRES"
                       f"({wl.restart}) to {wl.tol:g}; solve {t_solve:.1f} s ({info['iters']} iterations), "
                       f"matrix build {t_build:.1f} s not included",
                solve_s=t_solve, build_s=t_build, iters=info["iters"])


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps(dict(error="this build runs on one GPU only; --gpus must be 1")))
        sys.exit(2)
    import torch
    import wfq_inputs as wi
    from paper_2103_00438_amd import wfq

    wl = wi.workload(args.workload)
    prec = args.precision or wl.precision
    store = ("fp64", "fp32", "bf16") if prec == "bf16" else ("fp64", "fp32")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    h = wfq.wfq_build(wl.xyz, wl.params, store=store, device=0)
    build_s = time.perf_counter() - t0
    opts = dict(restart=wl.restart, precision=prec, algorithm=wl.algorithm)
    # the library's autotuner picks the block-product shape per column count (outside the timed region)
    t0 = time.perf_counter()
    ncols = sorted({c for c in (16, 32, 64, 96, 128, 192, 256, 320, 384, 512, 640, 768) if c <= 2 * wl.n_systems}
                   | {2 * wl.n_systems})
    tune = wfq.wfq_tune(h, prec, ncols, reps=2)
    if prec != "fp64":
        wfq.wfq_tune(h, "fp64", ncols, reps=2)   # shapes of the FP64 refinement products
    tune_s = time.perf_counter() - t0

    for _ in range(args.warmup):
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=False, **opts)
    wfq.wfq_kernel_stats(h, reset=True)
    torch.cuda.synchronize()
    outs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs.append(wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, timing=True, **opts))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = wfq.wfq_kernel_stats(h)
    S = wl.n_systems
    value = S * args.steps / elapsed
    last = outs[-1]
    lat = np.array([r["t_done_ms"] for r in last["info"]])
    iters = np.array([r["iters"] for r in last["info"]])
    statuses = sorted(set(r["status"] for r in last["info"]))
    relres_max = max(r["relres"] for r in last["info"])

    dom = {"fp32": "tx_gemm_f32", "fp64": "tx_gemm_f64", "bf16": "tx_gemm_bf16"}[prec]
    st = stats[dom]
    achieved = st["flops"] / (st["ms"] / 1e3) / 1e12 if st["ms"] > 0 else 0.0
    roofline = dict(bound="mfma", achieved=achieved, peak=PEAKS[prec], unit="TFLOP/s",
                    frac=achieved / PEAKS[prec], traffic=None, kernel=dom,
                    launches=st["launches"], avg_launch_ms=st["ms"] / max(1, st["launches"]),
                    avg_flops_per_launch=st["flops"] / max(1, st["launches"]))
    breakdown = {k: dict(ms=round(v["ms"], 3), launches=v["launches"],
                         gbps=(v["bytes"] / (v["ms"] / 1e3) / 1e9) if v["ms"] > 0 else None)
                 for k, v in stats.items() if v["launches"]}

    extra = {}
    if not args.no_reference:
        # the same systems with FP64 T inside the iterations (same GPU, same library): accuracy of
        # the mixed result, and the batched FP64 rate
        t0 = time.perf_counter()
        ref = wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, restart=wl.restart, precision="fp64")
        t_ref = time.perf_counter() - t0
        qm, qr = last["q"], ref["q"]
        err = np.linalg.norm(qm - qr, axis=2) / np.linalg.norm(qr, axis=2)
        am, ar = last["alpha"], ref["alpha"]
        aerr = np.abs(am - ar).max(axis=2) / np.abs(ar).max(axis=2)
        # per-frequency FP64 baseline: one system per solve, sampled
        samp = [0, S // 4, S // 2, 3 * S // 4, S - 1]
        t0 = time.perf_counter()
        for s in samp:
            a, k = divmod(s, len(wl.dirs))
            wfq.wfq_solve(h, wl.omegas_eV[a:a + 1], wl.dirs[k:k + 1], wl.tol, want_q=False,
                          restart=wl.restart, precision="fp64")
        t_pf = (time.perf_counter() - t0) / len(samp)
        extra = dict(max_rel_err_q_vs_fp64=float(err.max()), max_rel_err_alpha_vs_fp64=float(aerr.max()),
                     fp64_batched_solves_per_s=S / t_ref,
                     fp64_per_frequency_solves_per_s=1.0 / t_pf,
                     speedup_vs_fp64_per_frequency=value * t_pf,
                     per_frequency_sample=f"{len(samp)} systems, one per solve")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, S // 2)

    line = dict(
        metric="omega-point solves/s at rel. err 1e-6 (mixed vs FP64, same GPU); p50/p99 latency",
        value=value, unit="solves/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=elapsed / args.steps * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype={"fp32": "fp32-ir-fp64", "bf16": "bf16-ir-fp64", "fp64": "fp64"}[prec], data="synthetic",
        config=dict(workload=wl.name, n_atoms=wl.n, n_systems=S, n_omega=len(wl.omegas_eV), n_dir=len(wl.dirs),
                    precision=prec, algorithm=wl.algorithm, restart=wl.restart, tol=wl.tol,
                    description=wl.description),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        iters_mean=float(iters.mean()), iters_max=int(iters.max()), relres_max=relres_max,
        statuses=statuses, build_s=build_s, tune_s=tune_s,
        tuned={str(c): v for c, v in zip(tune["ncols"], tune["chosen"])},
        roofline=roofline, cpu_baseline=cpu, kernels=breakdown, **extra)
    print(json.dumps(line))
    h.close()


if __name__ == "__main__":
    main()
