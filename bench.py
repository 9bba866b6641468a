"""Benchmark: omega-point solves per second of the batched mixed-precision solve on one MI355X.

Default workload (cnt20k): armchair (10,10) carbon nanotube, 500 periods = 20 000 atoms, jitter
0.01 A (seed 2), graphene parameters (eps_F = 0.4 eV, tau = 170 a.u., d = 12, s = 1.1), 64
frequencies uniform in 0.05-1.0 eV x 3 field polarisations = 192 systems sharing one stored T.
One step = one wfq_solve over all 192 systems: FP32 T products inside restarted GMRES(50) with FP64
refinement to relative FP64 residual 1e-8. T and L are built (and resident in HBM) before the timed
region.

Printed (one JSON line): solves/s, p50/p99 per-system completion latency inside a step, the largest
relative difference of q against the FP64 solve on the same GPU, the per-frequency FP64 baseline
(one system per solve, same library), the roofline figures of the dominant kernel (timed with HIP
events on the library's stream) and the CPU oracle timed on a bounded sample.

Other workloads (--workload): disk600 (single-system latency), fcc120k (BF16 T, 120k atoms),
sheet1m (matrix-free T, 10^6 atoms), serve_mix (Poisson stream of jobs through wfq_serve).
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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}   # TFLOP/s, dense MFMA (MI355X)
HBM_GBPS = 8000.0                                         # GB/s, HBM3E (MI355X)
METRIC = "omega-point solves/s at rel. err 1e-6 (mixed vs FP64, same GPU); p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=2,
                    help="untimed solves first (small structures: the first sight of a step chunk runs "
                         "eagerly, the second captures it as a HIP graph, later ones replay it)")
    ap.add_argument("--workload", default="cnt20k")
    ap.add_argument("--algorithm", default=None, help="gmres, qmr or msgmres (one shared basis per direction)")
    ap.add_argument("--shift-dim", type=int, default=0, help="msgmres: largest shared-basis dimension (0 = 400)")
    ap.add_argument("--restart", type=int, default=0,
                    help="override the workload's GMRES restart length / QMR check interval")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference", action="store_true", help="skip the FP64 comparison runs")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the leg with warm starts across neighbouring frequencies")
    ap.add_argument("--no-multishift", action="store_true", help="skip the multi-shift FP64 run of the same systems")
    ap.add_argument("--no-block-jacobi", action="store_true",
                    help="skip the leg with block-Jacobi right preconditioning (64-atom diagonal blocks)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB on the device 4 times (calibrates the HBM byte counters) and report GB/s")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in block-product shapes")
    ap.add_argument("--ref-systems", type=int, default=0,
                    help="compare only this many systems against FP64 (0 = all)")
    ap.add_argument("--jobs", type=int, default=40, help="serve_mix: number of jobs in the stream")
    ap.add_argument("--max-iter", type=int, default=5000, help="cap on inner iterations per system")
    return ap.parse_args()


def cores_used():
    try:
        from threadpoolctl import threadpool_info
        return max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def host_info():
    """The host the CPU baseline ran on: CPU model, logical CPUs and memory."""
    model, mem_gb = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), mem_gb=mem_gb)


def cpu_baseline(wl, sys_index):
    """The oracle as it stands: FP64 restarted GMRES on one system of the workload (host cores)."""
    from oracle import wfq_oracle as O
    t0 = time.perf_counter()
    P = O.Problem(wl.xyz, wl.params)
    t_build = time.perf_counter() - t0
    a, k = divmod(sys_index, len(wl.dirs))
    t0 = time.perf_counter()
    x, info = P.solve_gmres(wl.omegas_eV[a], wl.dirs[k], wl.restart, wl.tol)
    t_solve = time.perf_counter() - t0
    return dict(value=1.0 / t_solve, unit="solves/s", cores=cores_used(), kind="oracle", host=host_info(),
                sample=f"1 of {wl.n_systems} systems (omega={wl.omegas_eV[a]:.4f} eV, dir {k}), FP64 GMRES"
                       f"({wl.restart}) to {wl.tol:g}; solve {t_solve:.1f} s ({info['iters']} iterations), "
                       f"matrix build {t_build:.1f} s not included",
                solve_s=t_solve, build_s=t_build, iters=info["iters"])


def cpu_baseline_matrix_free(wl, iters_per_solve, n_rows=256):
    """The oracle's pairwise (matrix-free) rows of T x on a sample of rows, scaled to solves/s."""
    from oracle import wfq_oracle as O
    xyz = O.angstrom_to_bohr(wl.xyz)
    eta = np.full(len(xyz), wl.params["eta"])
    x = np.random.default_rng(0).standard_normal(len(xyz))
    rows = np.arange(n_rows) * (len(xyz) // n_rows)
    t0 = time.perf_counter()
    for s in range(0, n_rows, 16):
        O.coulomb_rows(xyz, eta, rows[s:s + 16]) @ x
    t = time.perf_counter() - t0
    per_product = t / n_rows * len(xyz) * 2          # 2 real columns per complex system
    return dict(value=1.0 / (per_product * iters_per_solve), unit="solves/s", cores=cores_used(), kind="oracle", host=host_info(),
                sample=f"{n_rows} rows of the matrix-free T x ({n_rows * len(xyz):.3g} pairs, {t:.1f} s); "
                       f"extrapolated to one system = {iters_per_solve:.0f} products of 2 real columns "
                       f"(the GPU's mean iteration count); L and vector work ignored",
                pairs_per_s=n_rows * len(xyz) / t)


def kernel_table(stats):
    return {k: dict(ms=round(v["ms"], 3), launches=v["launches"],
                    gbps=(v["bytes"] / (v["ms"] / 1e3) / 1e9) if v["ms"] > 0 else None)
            for k, v in stats.items() if v["launches"]}


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter summary of this workload
    (profiles/*.md; FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size); None when there
    is none or the kernel source changed since the counters were taken."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as f:
            m = re.search(r"<!-- traffic (\{.*\}) -->", f.read())
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec.get("workload") != workload or rec.get("kernel") != kernel:
            continue
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["bytes_per_launch"]
    return None


def roofline_of(stats, prec, otf, n, workload=None):
    if otf:
        # Per pair the kernel evaluates T_ij on the vector ALUs (about 10 lane-slots for a far pair:
        # 3 sub, 1 mul, 2 fma and a quarter-rate rsqrt; about 38 near the diagonal) and accumulates
        # 2 * 32 flops per 32-column block on the FP32 matrix cores (64 flops per SIMD-cycle). With the
        # far-field path the matrix-core work is the larger one, so the roofline is the FP32 MFMA peak
        # on the flops of the column blocks actually present (2 n^2 ncol per launch).
        key = "tx_otf_f32" if prec == "fp32" else "tx_otf_f64"
        st = stats[key]
        ncol_avg = st["flops"] / max(1, st["launches"]) / (2.0 * n * n)
        pairs = n * n * math.ceil(ncol_avg / 32)
        avg_s = st["ms"] / max(1, st["launches"]) / 1e3
        achieved = st["flops"] / max(1, st["launches"]) / avg_s / 1e12 if avg_s > 0 else 0.0
        peak = PEAKS["fp32" if prec == "fp32" else "fp64"]
        return dict(bound="mfma", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                    traffic=measured_traffic(workload, key), kernel=key, launches=st["launches"],
                    avg_launch_ms=st["ms"] / max(1, st["launches"]),
                    pairs_per_launch=pairs, pairs_per_s=pairs / avg_s if avg_s > 0 else 0.0)
    # the T-product class that took the most time (systems may have escalated to another precision)
    classes = {"tx_gemm_f32": "fp32", "tx_gemm_f64": "fp64", "tx_gemm_bf16": "bf16", "tx_skinny": None}
    dom = max(classes, key=lambda k: stats.get(k, {}).get("ms", 0.0))
    if dom == "tx_skinny":
        # narrow products dominate (one column per direction in multi-shift mode): HBM-bound, T read once
        st = stats["tx_skinny"]
        avg_s = st["ms"] / max(1, st["launches"]) / 1e3
        achieved = st["bytes"] / max(1, st["launches"]) / avg_s / 1e9 if avg_s > 0 else 0.0
        return dict(bound="hbm", achieved=achieved, peak=HBM_GBPS, unit="GB/s", frac=achieved / HBM_GBPS,
                    traffic=measured_traffic(workload, "tx_skinny"), kernel="tx_skinny", launches=st["launches"],
                    avg_launch_ms=st["ms"] / max(1, st["launches"]),
                    avg_bytes_per_launch=st["bytes"] / max(1, st["launches"]))
    st = stats[dom]
    prec = classes[dom]
    achieved = st["flops"] / (st["ms"] / 1e3) / 1e12 if st["ms"] > 0 else 0.0
    return dict(bound="mfma", achieved=achieved, peak=PEAKS[prec], unit="TFLOP/s", frac=achieved / PEAKS[prec],
                traffic=measured_traffic(workload, dom), kernel=dom, launches=st["launches"], avg_launch_ms=st["ms"] / max(1, st["launches"]),
                avg_flops_per_launch=st["flops"] / max(1, st["launches"]))


def bench_batched(args, wl, wfq, torch):
    prec = args.precision or wl.precision
    algo = args.algorithm or wl.algorithm
    otf = wl.t_mode == "otf"
    store = ("fp64", "fp32", "bf16") if prec == "bf16" else ("fp64", "fp32")
    t0 = time.perf_counter()
    h = wfq.wfq_build(wl.xyz, wl.params, t_mode=wl.t_mode, store=store, device=0)
    build_s = time.perf_counter() - t0
    opts = dict(restart=wl.restart, precision=prec, algorithm=algo, progress=wl.n > 50000, max_iter=args.max_iter,
                shift_dim=args.shift_dim)
    # FP64 references: the same solver, except that multi-shift is checked against batched GMRES
    ref_algo = "gmres" if algo == "msgmres" else algo
    tune = None
    tune_s = 0.0
    S = wl.n_systems
    if not otf and not args.no_tune:
        # the library's autotuner picks the block-product shape per column count (outside the timed region)
        t0 = time.perf_counter()
        big = wl.n > 50000
        grid = (64, 128, 256, 384, 512, 768) if big else (16, 32, 64, 96, 128, 160, 192, 224, 256, 288, 320, 352, 384, 512, 640, 768)
        ncols = sorted({c for c in grid if c <= 2 * S} | {2 * S})
        reps = 1 if big else 2
        tune = wfq.wfq_tune(h, prec, ncols, reps=reps)
        if prec == "bf16":
            wfq.wfq_tune(h, "fp32", ncols, reps=reps)   # systems that escalate continue in FP32
        if prec != "fp64" and not big:
            wfq.wfq_tune(h, "fp64", ncols, reps=reps)   # shapes of the FP64 refinement products
        tune_s = time.perf_counter() - t0

    for _ in range(args.warmup):
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, **opts)
    wfq.wfq_kernel_stats(h, reset=True)
    torch.cuda.synchronize()
    # Per-kernel HIP events cost a few microseconds per launch: negligible for large workloads
    # (timed in the measured steps), dominant for small latency-bound ones, which are timed without
    # them and get the kernel table from one extra instrumented solve.
    events_in_steps = otf or wl.n > 50000
    outs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs.append(wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, timing=events_in_steps, **opts))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if not events_in_steps:
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=False, timing=True, **opts)
    stats = wfq.wfq_kernel_stats(h)
    value = S * args.steps / elapsed
    last = outs[-1]
    lat = np.array([r["t_done_ms"] for r in last["info"]])
    iters = np.array([r["iters"] for r in last["info"]])
    statuses = sorted(set(r["status"] for r in last["info"]))
    relres_max = max(r["relres"] for r in last["info"])
    prec_end = sorted(set(r["precision"] for r in last["info"]))
    roofline = roofline_of(stats, prec, otf, wl.n, wl.name)

    extra = {}
    if otf and not args.ref_systems:
        # a matrix-free FP64 solve of even one 10^6-atom system takes minutes: the check is the FP64
        # residual every result already carries (recomputed with FP64 elements on the fly) and the
        # error estimate relres x cond(R)
        extra = dict(fp64_reference_systems=0,
                     err_est_max=float(max(r["err_est"] for r in last["info"])),
                     fp64_check="relres of every system recomputed with FP64 matrix-free T")
    elif not args.no_reference and prec != "fp64":
        # the same systems with FP64 T inside the iterations (same GPU, same library)
        sel = list(range(S))
        # very large or matrix-free workloads: a sample of systems, each solved alone (which is also
        # the per-frequency FP64 baseline)
        nref = args.ref_systems or (2 if wl.n > 50000 else 0)
        if nref and nref < S:
            sel = [int(round(v)) for v in np.linspace(0, S - 1, nref)] if nref > 1 else [S // 2]
        t0 = time.perf_counter()
        qref = np.zeros((len(sel), wl.n), dtype=complex)
        aref = np.zeros((len(sel), 3), dtype=complex)
        if len(sel) == S:
            ref = wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, restart=wl.restart,
                                precision="fp64", algorithm=ref_algo, progress=wl.n > 50000)
            qref = ref["q"].reshape(S, wl.n)
            aref = ref["alpha"].reshape(S, 3)
        else:
            for q, s in enumerate(sel):
                a, k = divmod(s, len(wl.dirs))
                r1 = wfq.wfq_solve(h, wl.omegas_eV[a:a + 1], wl.dirs[k:k + 1], wl.tol, want_q=True,
                                   restart=wl.restart, precision="fp64", algorithm=ref_algo, progress=wl.n > 50000)
                qref[q] = r1["q"][0, 0]
                aref[q] = r1["alpha"][0, 0]
        t_ref = time.perf_counter() - t0
        qm = last["q"].reshape(S, wl.n)[sel]
        am = last["alpha"].reshape(S, 3)[sel]
        err = np.linalg.norm(qm - qref, axis=1) / np.linalg.norm(qref, axis=1)
        aerr = np.abs(am - aref).max(axis=1) / np.abs(aref).max(axis=1)
        extra = dict(max_rel_err_q_vs_fp64=float(err.max()), max_rel_err_alpha_vs_fp64=float(aerr.max()),
                     fp64_reference_systems=len(sel), fp64_reference_s=t_ref)
        if len(sel) == S:
            extra["fp64_batched_solves_per_s"] = S / t_ref
        # per-frequency FP64 baseline: one system per solve
        if len(sel) < S:
            t_pf = t_ref / len(sel)
            samp_note = f"the {len(sel)} reference system(s) above, one per solve"
        else:
            samp = [0, S // 4, S // 2, 3 * S // 4, S - 1]
            t0 = time.perf_counter()
            for s in samp:
                a, k = divmod(s, len(wl.dirs))
                wfq.wfq_solve(h, wl.omegas_eV[a:a + 1], wl.dirs[k:k + 1], wl.tol, want_q=False,
                              restart=wl.restart, precision="fp64", algorithm=ref_algo, progress=wl.n > 50000)
            t_pf = (time.perf_counter() - t0) / len(samp)
            samp_note = f"{len(samp)} systems, one per solve"
        extra.update(fp64_per_frequency_solves_per_s=1.0 / t_pf, speedup_vs_fp64_per_frequency=value * t_pf,
                     per_frequency_sample=samp_note)
    cpu = None
    if not otf and algo != "msgmres" and not args.no_multishift and wl.n <= 50000:
        # the next step of the method on the same systems: one real Krylov basis per field direction
        # shared by every frequency (multi-shift GMRES, FP64 T throughout), two warm-ups and one timed run
        msopts = dict(restart=wl.restart, precision="fp64", algorithm="msgmres", max_iter=args.max_iter)
        for _ in range(2):
            wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, **msopts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, **msopts)
        torch.cuda.synchronize()
        t_ms = time.perf_counter() - t0
        wfq.wfq_kernel_stats(h, reset=True)
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=False, timing=True, **msopts)
        ms_stats = wfq.wfq_kernel_stats(h)
        ms_line = dict(value=S / t_ms, unit="solves/s", ms_per_step=t_ms * 1e3, dtype="fp64",
                       iters_mean=float(np.mean([r["iters"] for r in ms["info"]])),
                       iters_max=int(max(r["iters"] for r in ms["info"])),
                       relres_max=max(r["relres"] for r in ms["info"]),
                       statuses=sorted(set(r["status"] for r in ms["info"])),
                       roofline=roofline_of(ms_stats, "fp64", False, wl.n, f"{wl.name}_multishift"),
                       kernels=kernel_table(ms_stats))
        if "fp64_reference_systems" in extra and extra["fp64_reference_systems"] == S:
            qms = ms["q"].reshape(S, wl.n)
            ms_line["max_rel_err_q_vs_fp64_batched"] = float(
                (np.linalg.norm(qms - qref, axis=1) / np.linalg.norm(qref, axis=1)).max())
        extra["multishift_fp64"] = ms_line
    if not otf and algo == "gmres" and not args.no_warm_start and len(wl.omegas_eV) >= 3 and wl.n <= 50000:
        # warm starts across neighbouring frequencies (the same options as the timed steps): one
        # warm-up and one timed run
        wopts = dict(opts, warm_start=True)
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, **wopts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ws = wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, **wopts)
        torch.cuda.synchronize()
        t_ws = time.perf_counter() - t0
        ws_line = dict(value=S / t_ws, unit="solves/s", ms_per_step=t_ws * 1e3, dtype=prec,
                       iters_mean=float(np.mean([r["iters"] for r in ws["info"]])),
                       iters_max=int(max(r["iters"] for r in ws["info"])),
                       relres_max=max(r["relres"] for r in ws["info"]),
                       statuses=sorted(set(r["status"] for r in ws["info"])))
        if "fp64_reference_systems" in extra and extra["fp64_reference_systems"] == S:
            qws = ws["q"].reshape(S, wl.n)
            ws_line["max_rel_err_q_vs_fp64_batched"] = float(
                (np.linalg.norm(qws - qref, axis=1) / np.linalg.norm(qref, axis=1)).max())
        extra["warm_start"] = ws_line
    if not otf and algo == "gmres" and not args.no_block_jacobi and wl.n <= 50000:
        # block-Jacobi right preconditioning (the same options as the timed steps): one warm-up and
        # one timed run
        bopts = dict(opts, block_jacobi=True)
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, **bopts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bj = wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, **bopts)
        torch.cuda.synchronize()
        t_bj = time.perf_counter() - t0
        wfq.wfq_kernel_stats(h, reset=True)
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=False, timing=True, **bopts)
        bj_stats = wfq.wfq_kernel_stats(h)
        bj_line = dict(value=S / t_bj, unit="solves/s", ms_per_step=t_bj * 1e3, dtype=prec,
                       iters_mean=float(np.mean([r["iters"] for r in bj["info"]])),
                       iters_max=int(max(r["iters"] for r in bj["info"])),
                       relres_max=max(r["relres"] for r in bj["info"]),
                       statuses=sorted(set(r["status"] for r in bj["info"])),
                       kernels=kernel_table(bj_stats))
        if "fp64_reference_systems" in extra and extra["fp64_reference_systems"] == S:
            qbj = bj["q"].reshape(S, wl.n)
            bj_line["max_rel_err_q_vs_fp64_batched"] = float(
                (np.linalg.norm(qbj - qref, axis=1) / np.linalg.norm(qref, axis=1)).max())
        extra["block_jacobi"] = bj_line

    if not args.no_cpu_baseline:
        if otf or wl.n > 50000:
            cpu = cpu_baseline_matrix_free(wl, float(iters.mean()))
        else:
            cpu = cpu_baseline(wl, S // 2)

    line = dict(
        metric=METRIC, value=value, unit="solves/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=elapsed / args.steps * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype={"fp32": "fp32-ir-fp64", "bf16": "bf16-ir-fp64", "fp64": "fp64"}[prec], data="synthetic",
        config=dict(workload=wl.name, n_atoms=wl.n, n_systems=S, n_omega=len(wl.omegas_eV), n_dir=len(wl.dirs),
                    precision=prec, algorithm=algo, restart=wl.restart, tol=wl.tol, t_mode=wl.t_mode,
                    description=wl.description),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        iters_mean=float(iters.mean()), iters_max=int(iters.max()), relres_max=relres_max,
        statuses=statuses, final_precisions=prec_end, build_s=build_s, tune_s=tune_s,
        tuned={str(c): v for c, v in zip(tune["ncols"], tune["chosen"])} if tune else None,
        roofline=roofline, cpu_baseline=cpu, kernels=kernel_table(stats), **extra)
    h.close()
    return line


def bench_latency(args, wl, wfq, torch):
    """disk600: one small system; latency of a single solve."""
    h = wfq.wfq_build(wl.xyz, wl.params, device=0)
    opts = dict(restart=wl.restart, precision=wl.precision, algorithm=args.algorithm or wl.algorithm)
    for _ in range(max(1, args.warmup)):
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, **opts)
    reps = max(20, args.steps)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        t1 = time.perf_counter()
        out = wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, **opts)
        lat.append((time.perf_counter() - t1) * 1e3)
    elapsed = time.perf_counter() - t0
    bj = None
    if not args.no_block_jacobi:
        # the same solve with block-Jacobi right preconditioning (64-atom diagonal blocks)
        bopts = dict(opts, block_jacobi=True)
        for _ in range(max(1, args.warmup)):
            wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, **bopts)
        blat = []
        for _ in range(reps):
            t1 = time.perf_counter()
            bo = wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, **bopts)
            blat.append((time.perf_counter() - t1) * 1e3)
        bj = dict(p50_ms=float(np.percentile(blat, 50)), p99_ms=float(np.percentile(blat, 99)),
                  iters=bo["info"][0]["iters"], relres=bo["info"][0]["relres"])
    from oracle import wfq_oracle as O
    P = O.Problem(wl.xyz, wl.params)
    t1 = time.perf_counter()
    P.solve_lu(wl.omegas_eV[0], wl.dirs[0])
    t_lu = time.perf_counter() - t1
    t1 = time.perf_counter()
    _, info = P.solve_gmres(wl.omegas_eV[0], wl.dirs[0], wl.restart, wl.tol)
    t_gm = time.perf_counter() - t1
    line = dict(metric=METRIC, value=reps / elapsed, unit="solves/s", n_gpus=1, steps=reps, warmup=args.warmup,
                ms_per_step=elapsed / reps * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="fp64", data="synthetic",
                config=dict(workload=wl.name, n_atoms=wl.n, n_systems=1, precision="fp64", restart=wl.restart,
                            tol=wl.tol, description=wl.description),
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                iters=out["info"][0]["iters"], relres=out["info"][0]["relres"], block_jacobi=bj,
                cpu_baseline=dict(value=1.0 / t_gm, unit="solves/s", cores=cores_used(), kind="oracle", host=host_info(),
                                  sample=f"the same system: FP64 GMRES({wl.restart}) {t_gm * 1e3:.1f} ms "
                                         f"({info['iters']} iterations); dense LU {t_lu * 1e3:.1f} ms"))
    h.close()
    return line


def bench_serve(args, wl, wfq, torch):
    """serve_mix: a seeded Poisson stream of spectrum jobs through the request loop."""
    import wfq_inputs as wi
    jobs = wi.serve_mix_jobs(n_jobs=args.jobs)
    prec = args.precision or wl.precision
    algo = args.algorithm or wl.algorithm
    srv = wfq.wfq_serve(wl.tol, max_jobs=4, max_queue=4096, restart=wl.restart, precision=prec, algorithm=algo)
    t0 = time.perf_counter()
    tickets = []
    for j in jobs:
        delay = j["arrival"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(wfq.wfq_submit(srv, j["xyz"], j["params"], j["omegas_eV"], j["dirs"]))
    res = [wfq.wfq_wait(srv, t) for t in tickets]
    elapsed = time.perf_counter() - t0
    st = wfq.wfq_serve_stats(srv)
    wfq.wfq_serve_stop(srv)
    lat = np.array([r["timing"]["latency_ms"] for r in res])
    queue = np.array([r["timing"]["t_admit_ms"] - r["timing"]["t_submit_ms"] for r in res])
    systems = sum(r["timing"]["n_systems"] for r in res)
    ok = sum(r["status"] == 0 for r in res)
    n_atoms = [len(j["xyz"]) for j in jobs]
    line = dict(metric=METRIC, value=systems / elapsed, unit="solves/s", n_gpus=1, steps=len(jobs), warmup=0,
                ms_per_step=elapsed / len(jobs) * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype={"fp32": "fp32-ir-fp64", "bf16": "bf16-ir-fp64", "fp64": "fp64"}[prec], data="synthetic",
                config=dict(workload=wl.name, jobs=len(jobs), rate_per_s=20.0, n_atoms_min=int(min(n_atoms)),
                            n_atoms_max=int(max(n_atoms)), systems=systems, tol=wl.tol, precision=prec,
                            algorithm=algo, max_jobs=4, description=wl.description),
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                queue_p50_ms=float(np.percentile(queue, 50)), queue_p99_ms=float(np.percentile(queue, 99)),
                jobs_ok=int(ok), busy_frac=st["busy_frac"], max_resident=st["max_resident"],
                wall_s=elapsed, offered_span_s=jobs[-1]["arrival"])
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps(dict(error="this build runs on one GPU only; --gpus must be 1")))
        sys.exit(2)
    import torch
    import wfq_inputs as wi
    from paper_2103_00438_amd import wfq

    torch.cuda.set_device(torch.device("cuda:0"))
    if args.copy_probe:
        a = torch.ones(64 * 1024 * 1024, device="cuda:0")      # 256 MiB of float32
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 4
        print(json.dumps(dict(copy_bytes=2 * a.numel() * 4, copy_gbps=2 * a.numel() * 4 / dt / 1e9)))
        return
    wl = wi.workload(args.workload)
    if args.restart > 0:
        wl.restart = args.restart
    if wl.name == "disk600":
        line = bench_latency(args, wl, wfq, torch)
    elif wl.name == "serve_mix":
        line = bench_serve(args, wl, wfq, torch)
    else:
        line = bench_batched(args, wl, wfq, torch)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
