"""Python binding of libwfq (ctypes). Argument marshalling only: every computation runs in the HIP
library. There is no fallback: if libwfq.so is missing or cannot be loaded, every call raises.

The functions carry the names of the C entry points declared in include/wfq.h.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwfq.so")

WFQ_OK, WFQ_EINVAL, WFQ_ENOMEM, WFQ_EDEVICE, WFQ_ESINGULAR, WFQ_ENOCONV = 0, 1, 2, 3, 4, 5
WFQ_EBREAKDOWN, WFQ_ENUMERIC, WFQ_EAGAIN, WFQ_EDISCONNECTED, WFQ_ENOTFOUND = 6, 7, 8, 9, 10
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESINGULAR", 5: "ENOCONV",
                6: "EBREAKDOWN", 7: "ENUMERIC", 8: "EAGAIN", 9: "EDISCONNECTED", 10: "ENOTFOUND"}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
PREC_NAMES = {v: k for k, v in PREC.items()}
ALGO = {"gmres": 0, "qmr": 1, "msgmres": 2}
TMODE = {"auto": 0, "stored": 1, "otf": 2}
STORE = {"fp64": 1, "fp32": 2, "bf16": 4}


class WfqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("n", C.c_int64), ("xyz", C.POINTER(C.c_double)), ("eta", C.POINTER(C.c_double)),
                ("species", C.POINTER(C.c_int32))]


class Species(C.Structure):
    _fields_ = [("eta", C.c_double), ("r0", C.c_double)]


class Params(C.Structure):
    _fields_ = [("eta", C.c_double), ("r0", C.c_double), ("fermi_d", C.c_double), ("fermi_s", C.c_double),
                ("cutoff_eps", C.c_double), ("W", C.c_double), ("tau", C.c_double), ("t_mode", C.c_int32),
                ("store_mask", C.c_uint32), ("device_budget", C.c_uint64), ("device", C.c_int32),
                ("material", C.c_int32), ("fermi_energy", C.c_double), ("valence", C.c_double),
                ("eff_mass", C.c_double), ("lattice_nn", C.c_double), ("n_species", C.c_int32),
                ("species", C.POINTER(Species))]


class SolveOpts(C.Structure):
    _fields_ = [("algorithm", C.c_int32), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("E0", C.c_double), ("max_batch", C.c_int32), ("timing", C.c_int32),
                ("escalate", C.c_int32), ("progress", C.c_int32), ("shift_dim", C.c_int32),
                ("graphs", C.c_int32), ("warm_start", C.c_int32), ("block_jacobi", C.c_int32),
                ("qmr_breakdown", C.c_double), ("ms_relax", C.c_double), ("recycle", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("cycles", C.c_int32), ("precision", C.c_int32),
                ("relres", C.c_double), ("rmse", C.c_double), ("err_est", C.c_double), ("t_done_ms", C.c_double),
                ("sigma", C.c_double)]


class ServeCfg(C.Structure):
    _fields_ = [("device_budget", C.c_uint64), ("max_jobs", C.c_int32), ("max_queue", C.c_int32),
                ("device", C.c_int32), ("opts", SolveOpts), ("tol", C.c_double)]


class Job(C.Structure):
    _fields_ = [("geom", Geometry), ("params", Params), ("omegas_eV", C.POINTER(C.c_double)),
                ("n_omega", C.c_int32), ("dirs", C.POINTER(C.c_double)), ("n_dir", C.c_int32)]


class JobTiming(C.Structure):
    _fields_ = [("t_submit_ms", C.c_double), ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double),
                ("latency_ms", C.c_double), ("status", C.c_int32), ("n_systems", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("jobs_done", C.c_int64), ("systems_done", C.c_int64), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("solves_per_s", C.c_double), ("busy_frac", C.c_double),
                ("max_resident", C.c_int32)]


_DP = C.POINTER(C.c_double)
_I64P = C.POINTER(C.c_int64)
_lib = None

_SIGNATURES = {
    "wfq_build": (C.c_int, [C.POINTER(Geometry), C.POINTER(Params), C.POINTER(C.c_void_p)]),
    "wfq_destroy": (None, [C.c_void_p]),
    "wfq_solve": (C.c_int, [C.c_void_p, _DP, C.c_int32, _DP, C.c_int32, C.c_double, C.POINTER(SolveOpts),
                            _DP, _DP, _DP, _DP, C.POINTER(Result)]),
    "wfq_solve_dev": (C.c_int, [C.c_void_p, _DP, C.c_int32, _DP, C.c_int32, C.c_double, C.POINTER(SolveOpts),
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Result), C.c_void_p]),
    "wfq_info": (C.c_int, [C.c_void_p, _I64P, _I64P, _I64P]),
    "wfq_sample_T": (C.c_int, [C.c_void_p, C.c_int32, _I64P, _I64P, C.c_int64, _DP]),
    "wfq_export_L": (C.c_int, [C.c_void_p, _I64P, _I64P, _DP]),
    "wfq_apply_T": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _DP, _DP]),
    "wfq_apply_T_variant": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _DP, _DP]),
    "wfq_apply_op": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _DP, _DP, _DP, _DP, _DP, _DP]),
    "wfq_apply_op_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "wfq_noalloc_scratch_bytes": (C.c_uint64, []),
    "wfq_rhs": (C.c_int, [C.c_void_p, _DP, C.c_int32, C.c_double, _DP]),
    "wfq_kernel_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_char_p), _I64P, _DP, _DP, _DP,
                                   C.c_int32]),
    "wfq_serve": (C.c_int, [C.POINTER(ServeCfg), C.POINTER(C.c_void_p)]),
    "wfq_submit": (C.c_int, [C.c_void_p, C.POINTER(Job), C.POINTER(C.c_uint64)]),
    "wfq_poll": (C.c_int, [C.c_void_p, C.c_uint64, _DP, _DP, _DP, _DP, C.POINTER(Result), C.POINTER(JobTiming)]),
    "wfq_wait": (C.c_int, [C.c_void_p, C.c_uint64, _DP, _DP, _DP, _DP, C.POINTER(Result), C.POINTER(JobTiming)]),
    "wfq_serve_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "wfq_serve_stop": (None, [C.c_void_p]),
    "wfq_last_error": (C.c_char_p, []),
    "wfq_material_weight": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_double)]),
    "wfq_isotropic_sigma": (C.c_int, [_DP, C.POINTER(Result), C.c_int32, _DP]),
    "wfq_tx_variants": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_char_p), C.POINTER(C.c_int32)]),
    "wfq_tune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32, _DP,
                           C.POINTER(C.c_int32)]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libwfq.so (raises if it is missing: there is no fallback path).

    PyTorch ships its own HIP runtime and loads it under the same SONAME (libamdhip64.so.7) that
    libwfq.so needs. Importing torch first makes libwfq bind to that already-loaded runtime, so the
    process holds one HIP runtime and torch's device buffers and streams are valid inside libwfq.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libwfq.so not found at {path}; build it with python -m paper_2103_00438_amd.build")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def wfq_last_error() -> str:
    return load().wfq_last_error().decode()


def _check(rc: int, allow=(WFQ_OK,)) -> int:
    if rc not in allow:
        raise WfqError(rc, wfq_last_error())
    return rc


def _dp(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Handle:
    """Owner of one device-resident structure (wfq_handle*)."""

    def __init__(self, ptr: int, n: int, status: int):
        self.ptr = C.c_void_p(ptr)
        self.n = n
        self.build_status = status

    def close(self):
        if self.ptr and self.ptr.value:
            load().wfq_destroy(self.ptr)
            self.ptr = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


MATERIAL = {None: 0, "graphene2D": 1, "metal3D": 2}


def make_params(params: dict, t_mode="stored", store=("fp64", "fp32"), budget=0, device=0) -> Params:
    """wfq_params from a parameter dict: eta, r0, fermi_d, fermi_s, cutoff_eps, tau, and either W or the
    material data (material "graphene2D" with fermi_energy_eV, or "metal3D" with valence and
    eff_mass; optional lattice_nn in Angstrom); optional species [(eta, r0), ...]. The Species array
    is kept on the returned object (p._species) for the duration of the call."""
    eta = params.get("eta", 0.0)
    p = Params()
    p.eta = float(eta) if np.isscalar(eta) else 0.0
    p.r0 = float(params["r0"])
    p.fermi_d = float(params["fermi_d"])
    p.fermi_s = float(params["fermi_s"])
    p.cutoff_eps = float(params["cutoff_eps"])
    p.W = float(params.get("W") or 0.0)
    p.tau = float(params["tau"])
    p.t_mode = TMODE[t_mode]
    p.store_mask = sum(STORE[s] for s in store)
    p.device_budget = int(budget)
    p.device = int(device)
    p.material = MATERIAL[params.get("material")]
    p.fermi_energy = float(params.get("fermi_energy_eV") or 0.0)
    p.valence = float(params.get("valence") or 0.0)
    p.eff_mass = float(params.get("eff_mass") or 0.0)
    p.lattice_nn = float(params.get("lattice_nn") or 0.0)
    sp = params.get("species")
    if sp:
        arr = (Species * len(sp))(*[Species(float(e), float(r)) for e, r in sp])
        p._species = arr
        p.n_species = len(sp)
        p.species = C.cast(arr, C.POINTER(Species))
    return p


def wfq_build(xyz, params: dict, t_mode="stored", store=("fp64", "fp32"), budget=0, device=0,
              species=None) -> Handle:
    """Set up a structure (positions in Angstrom, (N, 3)). `params` as in the workload descriptions;
    `species` [N] indices into params["species"] (None: every atom is species 0)."""
    lib = load()
    xyz = _f64(xyz)
    n = xyz.shape[0]
    eta = params.get("eta", 0.0)
    eta_arr = None if np.isscalar(eta) else _f64(eta)
    sp_arr = None if species is None else np.ascontiguousarray(species, dtype=np.int32)
    g = Geometry(n, _dp(xyz), _dp(eta_arr), sp_arr.ctypes.data_as(C.POINTER(C.c_int32)) if sp_arr is not None else None)
    p = make_params(params, t_mode, store, budget, device)
    out = C.c_void_p()
    rc = lib.wfq_build(C.byref(g), C.byref(p), C.byref(out))
    _check(rc, (WFQ_OK, WFQ_EDISCONNECTED))
    return Handle(out.value, n, rc)


def wfq_material_weight(params: dict) -> float:
    """The W wfq_build uses for these parameters (the W override or the material closure); host only."""
    p = make_params(params)
    W = C.c_double()
    _check(load().wfq_material_weight(C.byref(p), C.byref(W)))
    return W.value


def wfq_destroy(h: Handle) -> None:
    h.close()


def make_opts(algorithm="gmres", restart=50, max_iter=100000, precision="fp64", E0=1.0, max_batch=0,
              timing=False, escalate=True, progress=False, shift_dim=0, graphs=False, warm_start=False,
              block_jacobi=False, qmr_breakdown=0.0, ms_relax=0.0, recycle=0) -> SolveOpts:
    return SolveOpts(ALGO[algorithm], int(restart), int(max_iter), PREC[precision], float(E0), int(max_batch),
                     int(bool(timing)), int(bool(escalate)), int(bool(progress)), int(shift_dim),
                     int(bool(graphs)), int(bool(warm_start)), int(bool(block_jacobi)), float(qmr_breakdown),
                     float(ms_relax), int(recycle))


def _results(info):
    return [dict(status=r.status, iters=r.iters, cycles=r.cycles, precision=PREC_NAMES[r.precision],
                 relres=r.relres, rmse=r.rmse, err_est=r.err_est, t_done_ms=r.t_done_ms, sigma=r.sigma) for r in info]


def wfq_solve(h: Handle, omegas_eV, dirs, tol, want_q=True, check=True, **opts) -> dict:
    """Solve every (frequency, direction) system. Returns q [n_omega, n_dir, N] complex,
    alpha [n_omega, n_dir, 3] complex, info (list of dicts) and the status code."""
    lib = load()
    om = _f64(omegas_eV).ravel()
    d = _f64(dirs).reshape(-1, 3)
    no, nd, n = len(om), len(d), h.n
    S = no * nd
    qr = np.zeros((no, nd, n)) if want_q else None
    qi = np.zeros((no, nd, n)) if want_q else None
    ar = np.zeros((no, nd, 3))
    ai = np.zeros((no, nd, 3))
    info = (Result * S)()
    o = make_opts(**opts)
    rc = lib.wfq_solve(h.ptr, _dp(om), no, _dp(d), nd, float(tol), C.byref(o), _dp(qr), _dp(qi), _dp(ar), _dp(ai),
                       info)
    if check:
        _check(rc, (WFQ_OK, WFQ_ENOCONV, WFQ_ENUMERIC, WFQ_EBREAKDOWN))
    out = dict(q=(qr + 1j * qi) if want_q else None, alpha=ar + 1j * ai, info=_results(info), status=rc,
               sigma=np.array([r.sigma for r in info]).reshape(no, nd))
    if nd == 3:
        iso = np.zeros(no)
        if lib.wfq_isotropic_sigma(_dp(d), info, no, _dp(iso)) == WFQ_OK:   # orthonormal directions only
            out["sigma_iso"] = iso
    return out


def wfq_isotropic_sigma(dirs, sigma) -> np.ndarray:
    """Eq. (iso-cross) from sigma [n_omega, 3] of three orthonormal directions dirs [3, 3] (host)."""
    d = _f64(dirs).reshape(3, 3)
    sg = _f64(sigma).reshape(-1, 3)
    info = (Result * sg.size)()
    for i, v in enumerate(sg.ravel()):
        info[i].sigma = float(v)
    out = np.zeros(len(sg))
    _check(load().wfq_isotropic_sigma(_dp(d), info, len(sg), _dp(out)))
    return out


def wfq_solve_dev(h: Handle, omegas_eV, dirs, tol, q_re=None, q_im=None, alpha_re=None, alpha_im=None,
                  stream=None, **opts) -> dict:
    """As wfq_solve, outputs written to caller-provided device buffers (e.g. torch tensors on cuda)."""
    lib = load()
    om = _f64(omegas_eV).ravel()
    d = _f64(dirs).reshape(-1, 3)
    S = len(om) * len(d)
    info = (Result * S)()
    o = make_opts(**opts)

    def ptr(t):
        return None if t is None else C.c_void_p(t.data_ptr())

    st = None if stream is None else C.c_void_p(int(stream))
    rc = lib.wfq_solve_dev(h.ptr, _dp(om), len(om), _dp(d), len(d), float(tol), C.byref(o), ptr(q_re), ptr(q_im),
                           ptr(alpha_re), ptr(alpha_im), info, st)
    _check(rc, (WFQ_OK, WFQ_ENOCONV, WFQ_ENUMERIC, WFQ_EBREAKDOWN))
    return dict(info=_results(info), status=rc)


def wfq_info(h: Handle) -> dict:
    n, nnz, b = C.c_int64(), C.c_int64(), C.c_int64()
    _check(load().wfq_info(h.ptr, C.byref(n), C.byref(nnz), C.byref(b)))
    return dict(n=n.value, nnz=nnz.value, bytes=b.value)


def wfq_sample_T(h: Handle, precision, i, j) -> np.ndarray:
    i = np.ascontiguousarray(i, dtype=np.int64)
    j = np.ascontiguousarray(j, dtype=np.int64)
    out = np.zeros(len(i))
    _check(load().wfq_sample_T(h.ptr, PREC[precision], i.ctypes.data_as(_I64P), j.ctypes.data_as(_I64P), len(i),
                               _dp(out)))
    return out


def wfq_export_L(h: Handle):
    nnz = wfq_info(h)["nnz"]
    r = np.zeros(nnz, dtype=np.int64)
    c = np.zeros(nnz, dtype=np.int64)
    v = np.zeros(nnz)
    _check(load().wfq_export_L(h.ptr, r.ctypes.data_as(_I64P), c.ctypes.data_as(_I64P), _dp(v)))
    return r, c, v


def wfq_apply_T(h: Handle, precision, X) -> np.ndarray:
    X = _f64(X)
    if X.ndim == 1:
        X = X[None, :]
    Y = np.zeros_like(X)
    _check(load().wfq_apply_T(h.ptr, PREC[precision], X.shape[0], _dp(X), _dp(Y)))
    return Y


def wfq_apply_T_variant(h: Handle, precision, variant, X) -> np.ndarray:
    """Y = T X through one named (or indexed) block-product variant of the precision."""
    if isinstance(variant, str):
        names = [v[0] for v in wfq_tx_variants(precision)]
        variant = names.index(variant)
    X = _f64(X)
    if X.ndim == 1:
        X = X[None, :]
    Y = np.zeros_like(X)
    _check(load().wfq_apply_T_variant(h.ptr, PREC[precision], int(variant), X.shape[0], _dp(X), _dp(Y)))
    return Y


def wfq_apply_op(h: Handle, precision, z, X) -> np.ndarray:
    X = np.atleast_2d(np.asarray(X, dtype=np.complex128))
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    xr, xi = _f64(X.real), _f64(X.imag)
    zr, zi = _f64(z.real), _f64(z.imag)
    yr, yi = np.zeros_like(xr), np.zeros_like(xi)
    _check(load().wfq_apply_op(h.ptr, PREC[precision], X.shape[0], _dp(zr), _dp(zi), _dp(xr), _dp(xi), _dp(yr),
                               _dp(yi)))
    return yr + 1j * yi


def wfq_apply_op_noalloc(h: Handle, precision, z_re, z_im, X_re, X_im, Y_re, Y_im, stream=None) -> int:
    """Y = (L T + z_s I) X_s with device buffers (e.g. torch float64 tensors on cuda: z [nsys],
    X and Y [nsys, N] in the caller's atom order); only enqueues work on `stream`."""
    nsys = int(z_re.numel())

    def ptr(t):
        return C.c_void_p(t.data_ptr())

    st = None if stream is None else C.c_void_p(int(stream))
    return _check(load().wfq_apply_op_noalloc(h.ptr, PREC[precision], nsys, ptr(z_re), ptr(z_im), ptr(X_re),
                                              ptr(X_im), ptr(Y_re), ptr(Y_im), st))


def wfq_noalloc_scratch_bytes() -> int:
    return int(load().wfq_noalloc_scratch_bytes())


def wfq_rhs(h: Handle, dirs, E0=1.0) -> np.ndarray:
    d = _f64(dirs).reshape(-1, 3)
    out = np.zeros((len(d), h.n))
    _check(load().wfq_rhs(h.ptr, _dp(d), len(d), float(E0), _dp(out)))
    return out


def wfq_kernel_stats(h: Handle, reset=False) -> dict:
    lib = load()
    nc = C.c_int32()
    _check(lib.wfq_kernel_stats(h.ptr, C.byref(nc), None, None, None, None, None, 0))
    k = nc.value
    names = (C.c_char_p * k)()
    la = np.zeros(k, dtype=np.int64)
    ms, fl, by = np.zeros(k), np.zeros(k), np.zeros(k)
    _check(lib.wfq_kernel_stats(h.ptr, C.byref(nc), names, la.ctypes.data_as(_I64P), _dp(ms), _dp(fl), _dp(by),
                                int(reset)))
    return {names[q].decode(): dict(launches=int(la[q]), ms=float(ms[q]), flops=float(fl[q]), bytes=float(by[q]))
            for q in range(k)}


def wfq_tx_variants(precision) -> list:
    lib = load()
    cnt = C.c_int32()
    _check(lib.wfq_tx_variants(PREC[precision], C.byref(cnt), None, None))
    names = (C.c_char_p * cnt.value)()
    mx = (C.c_int32 * cnt.value)()
    _check(lib.wfq_tx_variants(PREC[precision], C.byref(cnt), names, mx))
    return [(names[k].decode(), mx[k]) for k in range(cnt.value)]


def wfq_tune(h: Handle, precision, ncols, reps=5) -> dict:
    """Time every block-product shape for each column count; the handle keeps the fastest."""
    names = [v[0] for v in wfq_tx_variants(precision)]
    nc = np.ascontiguousarray(ncols, dtype=np.int32)
    ms = np.zeros((len(nc), len(names)))
    chosen = np.zeros(len(nc), dtype=np.int32)
    _check(load().wfq_tune(h.ptr, PREC[precision], nc.ctypes.data_as(C.POINTER(C.c_int32)), len(nc), int(reps),
                           _dp(ms), chosen.ctypes.data_as(C.POINTER(C.c_int32))))
    return dict(variants=names, ncols=nc.tolist(), ms=ms, chosen=[names[c] if c >= 0 else None for c in chosen])


# ------------------------------------------------------------------ serving

class Server:
    def __init__(self, ptr):
        self.ptr = C.c_void_p(ptr)
        self.jobs = {}   # ticket -> (n, S, n_omega, n_dir) for result shapes

    def stop(self):
        if self.ptr and self.ptr.value:
            load().wfq_serve_stop(self.ptr)
            self.ptr = C.c_void_p(None)

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def wfq_serve(tol, device_budget=0, max_jobs=4, max_queue=1024, device=0, **opts) -> Server:
    cfg = ServeCfg(int(device_budget), int(max_jobs), int(max_queue), int(device), make_opts(**opts), float(tol))
    out = C.c_void_p()
    _check(load().wfq_serve(C.byref(cfg), C.byref(out)))
    return Server(out.value)


def wfq_submit(s: Server, xyz, params: dict, omegas_eV, dirs, species=None) -> int:
    """Queue one structure; `species` as in wfq_build. The server copies every array before returning."""
    xyz = _f64(xyz)
    om = _f64(omegas_eV).ravel()
    d = _f64(dirs).reshape(-1, 3)
    eta = params.get("eta", 0.0)
    eta_arr = None if np.isscalar(eta) else _f64(eta)
    sp_arr = None if species is None else np.ascontiguousarray(species, dtype=np.int32)
    pp = make_params(params)   # holds the species table until the call returns
    g = Geometry(xyz.shape[0], _dp(xyz), _dp(eta_arr),
                 sp_arr.ctypes.data_as(C.POINTER(C.c_int32)) if sp_arr is not None else None)
    job = Job(g, pp, _dp(om), len(om), _dp(d), len(d))
    t = C.c_uint64()
    _check(load().wfq_submit(s.ptr, C.byref(job), C.byref(t)))
    s.jobs[t.value] = (xyz.shape[0], len(om), len(d))
    return t.value


def _collect(s: Server, ticket: int, blocking: bool):
    n, no, nd = s.jobs[ticket]
    S = no * nd
    qr, qi = np.zeros((no, nd, n)), np.zeros((no, nd, n))
    ar, ai = np.zeros((no, nd, 3)), np.zeros((no, nd, 3))
    info = (Result * S)()
    tm = JobTiming()
    f = load().wfq_wait if blocking else load().wfq_poll
    rc = f(s.ptr, C.c_uint64(ticket), _dp(qr), _dp(qi), _dp(ar), _dp(ai), info, C.byref(tm))
    if rc == WFQ_EAGAIN:
        return None
    del s.jobs[ticket]
    _check(rc, (WFQ_OK, WFQ_ENOCONV, WFQ_ENUMERIC, WFQ_EBREAKDOWN))
    timing = dict(t_submit_ms=tm.t_submit_ms, t_admit_ms=tm.t_admit_ms, t_done_ms=tm.t_done_ms,
                  latency_ms=tm.latency_ms, status=tm.status, n_systems=tm.n_systems)
    return dict(q=qr + 1j * qi, alpha=ar + 1j * ai, info=_results(info), timing=timing, status=rc)


def wfq_poll(s: Server, ticket: int):
    return _collect(s, ticket, False)


def wfq_wait(s: Server, ticket: int):
    return _collect(s, ticket, True)


def wfq_serve_stats(s: Server) -> dict:
    st = Stats()
    _check(load().wfq_serve_stats(s.ptr, C.byref(st)))
    return dict(jobs_done=st.jobs_done, systems_done=st.systems_done, p50_ms=st.p50_ms, p99_ms=st.p99_ms,
                solves_per_s=st.solves_per_s, busy_frac=st.busy_frac, max_resident=st.max_resident)


def wfq_serve_stop(s: Server) -> None:
    s.stop()
