"""Parity at the benchmark sizes (needs an MI355X).

At full size the oracle cannot solve, so the checks are (i) outputs the oracle computes one by one
(sampled rows of T X, sampled rows of the FP64 residual of the GPU solution), (ii) properties that
hold at any size (charge conservation, reciprocity), and (iii) dense-LU parity on seeded sub-windows
cut from the same structures.
"""

import numpy as np
import pytest

from oracle import wfq_oracle as O
import wfq_inputs as wi
from wfq_inputs import geometry as geo
from helpers import UNIT, round_to

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


def sampled_rows(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def test_cnt20k_benchmark_configuration(lib):
    # the benchmark's launch configuration: 192 systems, FP32 T inside FP64 refinement, tuned shapes
    wl = wi.workload("cnt20k")
    h = lib.wfq_build(wl.xyz, wl.params)
    lib.wfq_tune(h, "fp32", [64, 128, 192, 256, 320, 384], reps=1)
    out = lib.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, restart=wl.restart, precision="fp32")
    h.close()
    assert out["status"] == 0
    assert max(r["relres"] for r in out["info"]) <= wl.tol
    # properties at any size
    Q = out["q"]
    for a in (0, 31, 63):
        for k in range(3):
            assert abs(Q[a, k].sum()) <= 1e-8 * np.linalg.norm(Q[a, k])
        A = out["alpha"][a].T
        assert abs(A[0, 1] - A[1, 0]) <= 1e-5 * abs(A[0, 0])
    # oracle FP64 residual on sampled rows: |r_i| <= ||r||_2 <= tol ||b||
    P = O.Problem(wl.xyz, wl.params, dense_T=False)
    rows = sampled_rows(wl.n, 48, 7)
    for a, k in ((0, 0), (32, 2), (63, 1)):
        b = P.rhs(wl.dirs[k])
        r = P.residual_rows(wl.omegas_eV[a], wl.dirs[k], Q[a, k], rows)
        assert np.max(np.abs(r)) <= wl.tol * np.linalg.norm(b)


def test_sheet1m_products_sampled_rows(lib):
    wl = wi.workload("sheet1m")
    h = lib.wfq_build(wl.xyz, wl.params, t_mode="otf")
    X = np.random.default_rng(11).standard_normal((2, wl.n))
    Y32 = lib.wfq_apply_T(h, "fp32", X)
    Y64 = lib.wfq_apply_T(h, "fp64", X)
    h.close()
    xyz = O.angstrom_to_bohr(wl.xyz)
    eta = np.full(wl.n, wl.params["eta"])
    rows = sampled_rows(wl.n, 24, 3)
    Trows = O.coulomb_rows(xyz, eta, rows)
    ref = X @ Trows.T                                 # [2][rows]
    bound = np.abs(X) @ np.abs(Trows).T
    assert np.all(np.abs(Y64[:, rows] - ref) <= 256 * UNIT["fp64"] * bound)
    Xq = round_to("fp32", X)
    ref32 = Xq @ Trows.T
    # element error of the FP32 erf (3.2e-7) + geometry and tile accumulation in FP32 (Kahan across tiles)
    assert np.all(np.abs(Y32[:, rows] - ref32) <= (3.2e-7 + 2 * 64 * UNIT["fp32"] + 16 * UNIT["fp32"]) * bound)


def test_sheet1m_subwindow_solve(lib):
    wl = wi.workload("sheet1m")
    sub = wi.sub_window(wl.xyz, 2000, seed=55)
    P = O.Problem(sub, wl.params)
    h = lib.wfq_build(sub, wl.params, t_mode="otf")
    om = wl.omegas_eV[[0, 7]]
    out = lib.wfq_solve(h, om, wl.dirs, 1e-9, restart=wl.restart, precision="fp32")
    h.close()
    assert out["status"] == 0
    for a in range(2):
        for k in range(2):
            ref = P.solve_lu(om[a], wl.dirs[k])
            assert np.linalg.norm(out["q"][a, k] - ref) / np.linalg.norm(ref) <= 1e-6


def test_fcc_sphere_long_neighbour_lists_interleaved_spmm(lib):
    # a 9 500-atom sphere: above the size where the SpMM reads interleaved planes, with ~320
    # neighbours per row (8-row blocks); checked by the oracle's FP64 residual on sampled rows
    wl = wi.workloads.FCC_METAL
    xyz = geo.jitter(geo.fcc_sphere(34.0), 0.02, 34)
    assert len(xyz) > 8192
    h = lib.wfq_build(xyz, wl)
    om = np.array([2.0, 3.5])
    dirs = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    tol = 1e-8
    out = lib.wfq_solve(h, om, dirs, tol, restart=100, precision="fp32")
    h.close()
    assert out["status"] == 0
    assert max(r["relres"] for r in out["info"]) <= tol
    P = O.Problem(xyz, wl, dense_T=False)
    rows = sampled_rows(len(xyz), 48, 9)
    for a in range(2):
        for k in range(2):
            b = P.rhs(dirs[k])
            r = P.residual_rows(om[a], dirs[k], out["q"][a, k], rows)
            assert np.max(np.abs(r)) <= tol * np.linalg.norm(b), (a, k)


@pytest.mark.parametrize("algorithm", ["gmres", "qmr"])
def test_fcc_subsphere_bf16(lib, algorithm):
    # a 2000-atom sphere cut from the same lattice and jitter recipe as the 120k-atom workload
    wl = wi.workloads.FCC_METAL
    xyz = geo.jitter(geo.fcc_sphere(20.2), 0.02, 33)
    P = O.Problem(xyz, wl)
    h = lib.wfq_build(xyz, wl, store=("fp64", "fp32", "bf16"))
    om = np.array([1.5, 3.0, 4.5])
    dirs = np.eye(3)
    out = lib.wfq_solve(h, om, dirs, 1e-9, restart=100, precision="bf16", algorithm=algorithm)
    h.close()
    assert out["status"] == 0
    for a in range(3):
        for k in range(3):
            ref = P.solve_lu(om[a], dirs[k])
            assert np.linalg.norm(out["q"][a, k] - ref) / np.linalg.norm(ref) <= 1e-6


def test_fcc120k_bf16_product_sampled_rows(lib):
    wl = wi.workload("fcc120k")
    h = lib.wfq_build(wl.xyz, wl.params, store=("fp64", "bf16"))
    X = np.random.default_rng(5).standard_normal((3, wl.n))
    Y16 = lib.wfq_apply_T(h, "bf16", X)
    Y64 = lib.wfq_apply_T(h, "fp64", X)
    h.close()
    xyz = O.angstrom_to_bohr(wl.xyz)
    eta = np.full(wl.n, wl.params["eta"])
    rows = sampled_rows(wl.n, 32, 9)
    Trows = O.coulomb_rows(xyz, eta, rows)
    bound = np.abs(X) @ np.abs(Trows).T
    assert np.all(np.abs(Y64[:, rows] - X @ Trows.T) <= 2 * wl.n * UNIT["fp64"] * bound)
    Tq = round_to("bf16", Trows)
    Xq = round_to("bf16", X)
    assert np.all(np.abs(Y16[:, rows] - Xq @ Tq.T) <= 2 * wl.n * UNIT["fp32"] * (np.abs(Xq) @ np.abs(Tq).T))


def _check_full_solution(wl, out, om, dirs, tol, rows_seed, bnorm=None):
    """The oracle's FP64 residual on 48 sampled rows of every system (each row from pairwise elements
    by the C++ oracle), charge conservation within what the residual allows and reciprocity. The
    scale ||b_k|| is the oracle's when it can build the whole L (all pairs), else `bnorm` (the
    library's right-hand sides, themselves checked against the oracle's in the step tests)."""
    from oracle.cpp_oracle import CppProblem
    P = CppProblem(wl.xyz, wl.params, dense_T=False, build_L=bnorm is None)
    rows = sampled_rows(wl.n, 48, rows_seed)
    for a in range(len(om)):
        for k in range(len(dirs)):
            q = out["q"][a, k]
            bn = np.linalg.norm(P.rhs(dirs[k])) if bnorm is None else bnorm[k]
            r = P.residual_rows(om[a], dirs[k], q, rows)
            # |r_i| <= ||r||_2 <= tol ||b|| (the library's own FP64 check), recomputed here row by row
            assert np.max(np.abs(r)) <= tol * bn, (a, k)
            # 1^T (L T + z I) q = z sum q = 1^T (b - r) = -1^T r, so |sum q| <= sqrt(N) tol ||b|| / |z|
            assert abs(q.sum()) <= 2 * np.sqrt(wl.n) * tol * bn / abs(P.z(om[a])), (a, k)
        A = out["alpha"][a]   # [dir][component]
        if len(dirs) > 1:
            assert abs(A[0, 1] - A[1, 0]) <= 1e-6 * max(abs(A[0, 0]), abs(A[1, 1])), a


def test_fcc120k_multishift_full_solution(lib):
    # the benchmark's solver on the full 119 879-atom sphere: 2 frequencies x 2 field directions by
    # multi-shift GMRES in FP64 with the recomputed narrow products, checked row by row by the oracle
    wl = wi.workload("fcc120k")
    om = wl.omegas_eV[[20, 100]]
    dirs = wl.dirs[:2]
    h = lib.wfq_build(wl.xyz, wl.params, store=("fp64",))
    out = lib.wfq_solve(h, om, dirs, wl.tol, restart=wl.restart, precision="fp64", algorithm="msgmres",
                        shift_dim=wl.extra["shift_dim"])
    h.close()
    assert out["status"] == 0
    assert max(r["relres"] for r in out["info"]) <= wl.tol
    _check_full_solution(wl, out, om, dirs, wl.tol, 13)


@pytest.mark.parametrize("nd", [1, 4])
def test_multishift_symmetric_products_one_and_four_directions(lib, nd):
    # multi-shift FP64 on a 70 249-atom FCC sphere (symmetric narrow products, last block partial) with
    # one field direction and with four (x, y, z and the body diagonal: 4-column products and SpMM
    # gathers); every result checked row by row by the oracle, with charge conservation and reciprocity
    from types import SimpleNamespace
    par = dict(wi.workloads.FCC_METAL)
    xyz = geo.jitter(geo.fcc_sphere(66.0), 0.02, 11)
    wl = SimpleNamespace(xyz=xyz, params=par, n=len(xyz))
    dirs = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 1.0, 1.0]])[:nd]
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    om = np.array([2.2, 3.6])
    tol = 1e-7
    h = lib.wfq_build(xyz, par, t_mode="otf")
    out = lib.wfq_solve(h, om, dirs, tol, restart=100, precision="fp64", algorithm="msgmres", shift_dim=1500)
    bnorm = np.linalg.norm(lib.wfq_rhs(h, dirs), axis=1)
    h.close()
    assert out["status"] == 0, out["info"]
    assert max(r["relres"] for r in out["info"]) <= tol
    assert all(r["cycles"] == 0 for r in out["info"]), [r["cycles"] for r in out["info"]]
    _check_full_solution(wl, out, om, dirs, tol, 17 + nd, bnorm=bnorm)


def test_sheet1m_multishift_full_solution(lib):
    # the full 10^6-atom sheet, matrix-free: 1 frequency x 2 in-plane directions by multi-shift GMRES
    # in FP64 (every T element recomputed in every product), checked row by row by the oracle
    wl = wi.workload("sheet1m")
    om = wl.omegas_eV[[3]]
    h = lib.wfq_build(wl.xyz, wl.params, t_mode="otf")
    out = lib.wfq_solve(h, om, wl.dirs, wl.tol, restart=wl.restart, precision="fp64", algorithm="msgmres",
                        shift_dim=1500)
    bnorm = np.linalg.norm(lib.wfq_rhs(h, wl.dirs), axis=1)
    h.close()
    assert out["status"] == 0
    assert max(r["relres"] for r in out["info"]) <= wl.tol
    _check_full_solution(wl, out, om, wl.dirs, wl.tol, 17, bnorm=bnorm)
