"""Benchmark: omega-point solves per second on one MI355X.

Default workload (fcc120k): FCC metal sphere, a = 4.09 A, R = 78.8 A, 119 879 atoms, jitter 0.02 A
(seed 3), metal parameters (tau = 170 a.u., d = 12, s = 1.1, W from the Drude sum-rule closure), 128
frequencies uniform in 1.5-4.5 eV x 3 field polarisations = 384 systems sharing one T. One step =
one wfq_solve over all 384 systems to relative FP64 residual 1e-7: multi-shift GMRES (one Krylov
basis of L T per field direction shared by the 128 frequencies, FP64 throughout; the narrow T
products recompute T's elements on the vector ALUs), then the FP64 residual check of every system.
T (FP64 copy, for the residual check) and L are built and resident in HBM before the timed region.

Printed (one JSON line): solves/s, p50/p99 per-system completion latency inside a step, iterations,
the largest relative difference of q against per-frequency FP64 GMRES(100) solves of sampled systems
on the same GPU (which are also the per-frequency baseline), a per-frequency QMR leg, the roofline of
the dominant kernel (HIP events on the library's stream) and the C++ CPU oracle timed on a bounded
sample.

Other workloads (--workload): cnt20k (FP32 T inside FP64 refinement, batched GMRES(50), 20 000
atoms), disk600 (single-system latency), disk600_spectrum, sheet1m (matrix-free T, 10^6 atoms),
serve_mix (Poisson stream of jobs through wfq_serve).
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
# FP64 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one FP64 operation per lane per
# clock; an FMA counts as one operation here)
VALU_F64_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
METRIC = "omega-point solves/s at rel. err 1e-6 (mixed vs FP64, same GPU); p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=2,
                    help="untimed solves first (small structures: the first sight of a step chunk runs "
                         "eagerly, the second captures it as a HIP graph, later ones replay it)")
    ap.add_argument("--workload", default="fcc120k")
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
    ap.add_argument("--ni-study", action="store_true",
                    help="per-frequency full-GMRES iteration counts against sigma_k (one JSON line per structure)")
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


def cpu_baseline(wl, n_samples=5, budget_s=40.0):
    """The C++ FP64 oracle (stored T, OpenMP over the host's cores): restarted GMRES on a stratified
    sample of the workload's systems (evenly spaced over frequency, cycling through the field
    directions), stopping early once budget_s of solve time is spent."""
    from oracle import cpp_oracle
    t0 = time.perf_counter()
    P = cpp_oracle.CppProblem(wl.xyz, wl.params)
    t_build = time.perf_counter() - t0
    S = wl.n_systems
    idx = [int(round(v)) for v in np.linspace(0, len(wl.omegas_eV) - 1, n_samples)]
    done, t_solve, iters = [], 0.0, []
    for q, a in enumerate(idx):
        k = q % len(wl.dirs)
        t1 = time.perf_counter()
        _, info = P.solve_gmres(wl.omegas_eV[a], wl.dirs[k], wl.restart, wl.tol)
        t_solve += time.perf_counter() - t1
        done.append(f"{wl.omegas_eV[a]:.3f} eV/dir {k}")
        iters.append(info["iters"])
        if t_solve > budget_s:
            break
    return dict(value=len(done) / t_solve, unit="solves/s", cores=cpp_oracle.threads(), kind="oracle",
                host=host_info(),
                sample=f"{len(done)} of {S} systems ({', '.join(done)}), C++ oracle FP64 GMRES({wl.restart}) to "
                       f"{wl.tol:g} with stored FP64 T; solve {t_solve:.1f} s, iterations {iters}; matrix build "
                       f"{t_build:.1f} s not included",
                solve_s=t_solve, build_s=t_build, iters=iters)


def cpu_baseline_rows(wl, iters_per_solve, target_s=15.0):
    """The C++ FP64 oracle's matrix-free T product (every element recomputed, OpenMP over the host's
    cores) timed on sampled rows, scaled to one solve of iters_per_solve products of 2 real columns."""
    from oracle import cpp_oracle
    P = cpp_oracle.CppProblem(wl.xyz, wl.params, dense_T=False, build_L=False)
    X = np.random.default_rng(0).standard_normal((wl.n, 2))
    n_rows, t = 256, 0.0
    while True:
        rows = (np.arange(n_rows) * (wl.n // n_rows)).astype(np.int64)
        t0 = time.perf_counter()
        P.apply_T_rows(rows, X)
        t = time.perf_counter() - t0
        if t > target_s / 4 or n_rows >= wl.n:
            break
        n_rows = min(wl.n, int(n_rows * max(2.0, target_s / 4 / max(t, 1e-3))))
    pairs_per_s = n_rows * wl.n / t
    per_product = wl.n * wl.n / pairs_per_s
    return dict(value=1.0 / (per_product * iters_per_solve), unit="solves/s", cores=cpp_oracle.threads(),
                kind="oracle", host=host_info(),
                sample=f"{n_rows} rows of the C++ oracle's matrix-free T x, 2 columns ({n_rows * wl.n:.3g} pair "
                       f"evaluations in {t:.1f} s), extrapolated to one system = {iters_per_solve:.0f} products "
                       f"(the per-frequency GMRES({wl.restart}) iteration count on the GPU); L and vector work "
                       f"ignored",
                pairs_per_s=pairs_per_s)


def cpu_baseline_matrix_free(wl, iters_per_solve, n_rows=256):
    """The oracle's pairwise (matrix-free) rows of T x on a sample of rows, scaled to solves/s."""
    return cpu_baseline_rows(wl, iters_per_solve, target_s=10.0)


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
    classes = {"tx_gemm_f32": "fp32", "tx_gemm_f64": "fp64", "tx_gemm_bf16": "bf16", "tx_skinny": None,
               "tx_skinny_f32": None, "tx_otf_narrow": None}
    dom = max(classes, key=lambda k: stats.get(k, {}).get("ms", 0.0))
    if dom == "tx_otf_narrow":
        # narrow products with every element recomputed: bound by the FP64 vector ALUs. Work per
        # element: 3 differences, 3 operations for r^2, the reciprocal square root, 4 for its Newton
        # step, and one multiply-add per column and row; from 65 536 atoms each element serves both
        # of its rows (n^2 / 2 evaluations) - the library's count; peak: one FP64 operation per lane
        # per clock
        st = stats["tx_otf_narrow"]
        avg_s = st["ms"] / max(1, st["launches"]) / 1e3
        achieved = st["flops"] / max(1, st["launches"]) / avg_s / 1e12 if avg_s > 0 else 0.0
        return dict(bound="alu", achieved=achieved, peak=VALU_F64_TOPS, unit="TOP/s", frac=achieved / VALU_F64_TOPS,
                    traffic=measured_traffic(workload, "tx_otf_narrow"), kernel="tx_otf_narrow",
                    launches=st["launches"], avg_launch_ms=st["ms"] / max(1, st["launches"]),
                    avg_ops_per_launch=st["flops"] / max(1, st["launches"]),
                    pairs_per_s=n * n / avg_s if avg_s > 0 else 0.0)
    if dom in ("tx_skinny", "tx_skinny_f32"):
        # narrow products dominate (one column per direction in multi-shift mode): HBM-bound, T read once
        st = stats[dom]
        avg_s = st["ms"] / max(1, st["launches"]) / 1e3
        achieved = st["bytes"] / max(1, st["launches"]) / avg_s / 1e9 if avg_s > 0 else 0.0
        return dict(bound="hbm", achieved=achieved, peak=HBM_GBPS, unit="GB/s", frac=achieved / HBM_GBPS,
                    traffic=measured_traffic(workload, dom), kernel=dom, launches=st["launches"],
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
    if not otf and algo == "gmres" and not args.no_warm_start and len(wl.omegas_eV) >= 3 and wl.n <= 50000:
        # subspace recycling (the same options, recycle space of the 4 nearest solved frequencies):
        # one warm-up and one timed run; iteration totals against the warm starts and q0 = 0
        ropts = dict(opts, recycle=4)
        wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=False, **ropts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = wfq.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=True, **ropts)
        torch.cuda.synchronize()
        t_rc = time.perf_counter() - t0
        n_rc = int(sum(r["iters"] for r in rc["info"]))
        rc_line = dict(value=S / t_rc, unit="solves/s", ms_per_step=t_rc * 1e3, dtype=prec, recycle=4,
                       iters_total=n_rc, iters_total_warm_start=int(sum(r["iters"] for r in ws["info"])),
                       iters_total_zero_start=int(sum(r["iters"] for r in last["info"])),
                       iters_max=int(max(r["iters"] for r in rc["info"])),
                       relres_max=max(r["relres"] for r in rc["info"]),
                       statuses=sorted(set(r["status"] for r in rc["info"])))
        if "fp64_reference_systems" in extra and extra["fp64_reference_systems"] == S:
            qrc = rc["q"].reshape(S, wl.n)
            rc_line["max_rel_err_q_vs_fp64_batched"] = float(
                (np.linalg.norm(qrc - qref, axis=1) / np.linalg.norm(qref, axis=1)).max())
        extra["recycle"] = rc_line
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
            cpu = cpu_baseline(wl)

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


def bench_multishift(args, wl, wfq, torch):
    """Large structures solved by multi-shift GMRES in FP64 (fcc120k): one shared basis per field
    direction, the narrow products recomputing T's elements; the FP64 copy of T serves the final
    residual check. Per-frequency FP64 GMRES(restart) and QMR solves of sampled systems give the
    reference, the per-frequency baseline and the two solvers' legs."""
    prec = args.precision or wl.precision
    shift_dim = args.shift_dim or wl.extra.get("shift_dim", 0)
    S = wl.n_systems
    nd = len(wl.dirs)
    t0 = time.perf_counter()
    h = wfq.wfq_build(wl.xyz, wl.params, t_mode=wl.t_mode, store=("fp64",) if prec == "fp64" else ("fp64", prec),
                      device=0)
    build_s = time.perf_counter() - t0
    opts = dict(restart=wl.restart, precision=prec, algorithm="msgmres", max_iter=args.max_iter, shift_dim=shift_dim)
    tune = None
    t0 = time.perf_counter()
    if not args.no_tune and wl.t_mode != "otf":   # matrix-free structures have no stored variants to tune
        # the shapes of the narrow products (one column per direction); the one FP64 residual check
        # per solve keeps the built-in shape
        tune = wfq.wfq_tune(h, "fp64", list(range(1, nd + 1)), reps=2)
    tune_s = time.perf_counter() - t0
    # every step writes q and alpha to device buffers (the results stay in HBM, as the inputs do)
    dev = torch.device("cuda:0")
    q_re = torch.zeros(S * wl.n, dtype=torch.float64, device=dev)
    q_im = torch.zeros_like(q_re)
    a_re = torch.zeros(S * 3, dtype=torch.float64, device=dev)
    a_im = torch.zeros_like(a_re)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step(timing):
        return wfq.wfq_solve_dev(h, wl.omegas_eV, wl.dirs, wl.tol, q_re=q_re, q_im=q_im, alpha_re=a_re,
                                 alpha_im=a_im, stream=stream, timing=timing, **opts)

    for k in range(args.warmup):
        step(False)
        print(f"[bench] warm-up {k + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    wfq.wfq_kernel_stats(h, reset=True)
    torch.cuda.synchronize()
    outs = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        outs.append(step(True))
        print(f"[bench] step {k + 1}/{args.steps}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = wfq.wfq_kernel_stats(h)
    value = S * args.steps / elapsed
    last = outs[-1]
    lat = np.array([r["t_done_ms"] for r in last["info"]])
    iters = np.array([r["iters"] for r in last["info"]])
    statuses = sorted(set(r["status"] for r in last["info"]))
    roofline = roofline_of(stats, prec, False, wl.n, wl.name)
    q = (q_re.cpu().numpy() + 1j * q_im.cpu().numpy()).reshape(S, wl.n)
    alpha = (a_re.cpu().numpy() + 1j * a_im.cpu().numpy()).reshape(S, 3)
    # invariants of every result: charge conservation, reciprocity alpha_lk = alpha_kl across directions
    qsum = float(np.max(np.abs(q.sum(axis=1)) / np.linalg.norm(q, axis=1)))
    A = alpha.reshape(len(wl.omegas_eV), nd, 3)
    recip = float(max(abs(A[w, k, l] - A[w, l, k]) / max(abs(A[w, k, k]), abs(A[w, l, l]))
                      for w in range(A.shape[0]) for k in range(nd) for l in range(nd) if l != k)) if nd > 1 else None

    extra = {}
    if not args.no_reference:
        # per-frequency FP64 solves of sampled systems on the same GPU: GMRES(restart) is both the
        # reference of every sampled result and the per-frequency baseline; QMR the second solver
        nref = args.ref_systems or 2
        sel = [int(round(v)) for v in np.linspace(S // 4, 3 * S // 4, nref)]
        errs, aerrs, t_gm, it_gm = [], [], 0.0, []
        for s_ in sel:
            a, k = divmod(s_, nd)
            torch.cuda.synchronize(); t1 = time.perf_counter()
            r1 = wfq.wfq_solve(h, wl.omegas_eV[a:a + 1], wl.dirs[k:k + 1], wl.tol, want_q=True, restart=wl.restart,
                               precision="fp64", algorithm="gmres", max_iter=20000)
            torch.cuda.synchronize(); t_gm += time.perf_counter() - t1
            it_gm.append(r1["info"][0]["iters"])
            qr = r1["q"][0, 0]
            errs.append(float(np.linalg.norm(q[s_] - qr) / np.linalg.norm(qr)))
            ar = r1["alpha"][0, 0]
            aerrs.append(float(np.abs(alpha[s_] - ar).max() / np.abs(ar).max()))
        s_q = sel[len(sel) // 2]
        a, k = divmod(s_q, nd)
        torch.cuda.synchronize(); t1 = time.perf_counter()
        rq = wfq.wfq_solve(h, wl.omegas_eV[a:a + 1], wl.dirs[k:k + 1], wl.tol, want_q=True, algorithm="qmr",
                           restart=100000, precision="fp64", max_iter=20000)
        torch.cuda.synchronize(); t_qmr = time.perf_counter() - t1
        qq = rq["q"][0, 0]
        extra = dict(
            max_rel_err_q_vs_fp64=max(errs), max_rel_err_alpha_vs_fp64=max(aerrs),
            fp64_reference=f"per-frequency FP64 GMRES({wl.restart}) of {len(sel)} sampled systems {sel}",
            fp64_per_frequency_solves_per_s=len(sel) / t_gm, speedup_vs_fp64_per_frequency=value * t_gm / len(sel),
            per_frequency_gmres=dict(solver=f"GMRES({wl.restart})", precision="fp64", systems=sel, iters=it_gm,
                                     s_per_solve=t_gm / len(sel)),
            per_frequency_qmr=dict(solver="J-symmetric QMR", precision="fp64", systems=[s_q],
                                   iters=rq["info"][0]["iters"], s_per_solve=t_qmr,
                                   status=rq["info"][0]["status"], relres=rq["info"][0]["relres"],
                                   rel_err_q_vs_multishift=float(np.linalg.norm(q[s_q] - qq) / np.linalg.norm(qq))))
    cpu = None
    if not args.no_cpu_baseline:
        it = float(np.mean(extra["per_frequency_gmres"]["iters"])) if extra else float(iters.mean())
        cpu = cpu_baseline_rows(wl, it)
    line = dict(
        metric=METRIC, value=value, unit="solves/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=elapsed / args.steps * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=prec, data="synthetic",
        config=dict(workload=wl.name, n_atoms=wl.n, n_systems=S, n_omega=len(wl.omegas_eV), n_dir=nd,
                    precision=prec, algorithm="msgmres", shift_dim=shift_dim, restart=wl.restart, tol=wl.tol,
                    description=wl.description),
        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
        iters_mean=float(iters.mean()), iters_max=int(iters.max()),
        relres_max=max(r["relres"] for r in last["info"]), statuses=statuses,
        max_abs_charge_sum_rel=qsum, max_reciprocity_rel=recip, build_s=build_s, tune_s=tune_s,
        tuned={str(c): v for c, v in zip(tune["ncols"], tune["chosen"])} if tune else None,
        roofline=roofline, cpu_baseline=cpu, kernels=kernel_table(stats), **extra)
    h.close()
    return line


def plateau_peaks(y):
    """Indices of local maxima of a sequence, a run of equal values counting once (its middle), when
    both neighbouring runs are lower."""
    runs, i = [], 0
    while i < len(y):
        j = i
        while j + 1 < len(y) and y[j + 1] == y[i]:
            j += 1
        runs.append((i, j, y[i]))
        i = j + 1
    return [(runs[k][0] + runs[k][1]) // 2 for k in range(1, len(runs) - 1)
            if runs[k][2] > runs[k - 1][2] and runs[k][2] > runs[k + 1][2]]


def ni_study(wfq):
    """The paper's NI study: full GMRES from q0 = 0 with ||r||_2 < 1e-6 a.u. (the multi-shift basis
    gives every frequency the full-GMRES iterate of its own shift), sigma_k per frequency, and how
    often a local maximum of sigma_k has a local maximum of NI within one and two grid points."""
    import wfq_inputs as wi
    from wfq_inputs import geometry as geo
    sharp = dict(wi.workloads.GRAPHENE, fermi_energy_eV=1.51, tau=17000.0)
    disk = wi.workload("disk600_spectrum")
    cases = [("disk600_spectrum", disk.xyz, disk.params, disk.omegas_eV, [0, 1]),
             ("disk600, eps_F 1.51 eV, tau 17000 a.u.", disk.xyz, sharp, np.arange(1, 401) * 0.01, [0, 1]),
             ("(10,10) nanotube, 100 cells, eps_F 1.51 eV, tau 17000 a.u.", geo.nanotube(10, 10, 100), sharp,
              np.arange(1, 201) * 0.01, [0, 2])]
    lines = []
    for name, xyz, par, om, ks in cases:
        h = wfq.wfq_build(xyz, par)
        rec = dict(study="ni_vs_sigma", structure=name, n_atoms=int(len(xyz)), omega_eV=[round(float(w), 4) for w in om],
                   threshold_abs=1e-6, directions={})
        for k in ks:
            d = np.eye(3)[k:k + 1]
            bn = float(np.linalg.norm(wfq.wfq_rhs(h, d)[0]))
            out = wfq.wfq_solve(h, om, d, 1e-6 / bn, want_q=False, algorithm="msgmres", precision="fp64",
                                shift_dim=1024, max_iter=20000)
            ni = [r["iters"] for r in out["info"]]
            sg = [r["sigma"] for r in out["info"]]
            ps, pn = plateau_peaks(sg), plateau_peaks(ni)
            near = lambda tol: (float(np.mean([min((abs(p - q) for q in pn), default=99) <= tol for p in ps]))
                                if ps else None)
            rec["directions"]["xyz"[k]] = dict(
                ni=ni, sigma_bohr2=[float(f"{v:.6g}") for v in sg], status=int(out["status"]),
                sigma_peaks_eV=[rec["omega_eV"][p] for p in ps], ni_peaks_eV=[rec["omega_eV"][p] for p in pn],
                matched_within_1=near(1), matched_within_2=near(2), full_gmres=bool(max(ni) <= 1024),
                chance_within_2=min(1.0, 5 * len(pn) / len(ni)))
        h.close()
        lines.append(rec)
    return lines


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
        print(json.dumps(dict(error="the library runs on one GPU; --gpus must be 1 (multi-GPU sharding is a design, not an implementation)")))
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
    if args.ni_study:
        for rec in ni_study(wfq):
            print(json.dumps(rec))
        return
    wl = wi.workload(args.workload)
    if args.restart > 0:
        wl.restart = args.restart
    if wl.name == "disk600":
        line = bench_latency(args, wl, wfq, torch)
    elif wl.name == "serve_mix":
        line = bench_serve(args, wl, wfq, torch)
    elif (args.algorithm or wl.algorithm) == "msgmres" and wl.n > 50000:
        line = bench_multishift(args, wl, wfq, torch)
    else:
        line = bench_batched(args, wl, wfq, torch)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
