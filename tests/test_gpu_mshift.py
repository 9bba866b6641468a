"""Multi-shift GMRES (one real Krylov basis of L T per field direction for all frequencies) against
the CPU oracle (needs an MI355X).

References: the oracle's dense LU solution of every (frequency, direction) system, and the oracle's
own multi-shift GMRES for the number of shared-basis steps each frequency needs. The GPU result must
have FP64 relative residual <= tol and match LU to 1e-6 relative error in every precision of T (the
shared-basis phase hands its iterates to batched GMRES with FP64 refinement).
"""

import numpy as np
import pytest

from oracle import wfq_oracle as O
from helpers import GRAPHENE, ragged_tube
import wfq_inputs as wi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def tube_case():
    xyz = ragged_tube()
    P = O.Problem(xyz, GRAPHENE)
    om = np.array([0.05, 0.2, 0.31, 0.55, 0.77, 1.0])
    dirs = np.eye(3)
    ref = {(a, k): P.solve_lu(om[a], dirs[k]) for a in range(len(om)) for k in range(3)}
    return xyz, P, om, dirs, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_multishift_matches_lu(lib, tube_case, prec):
    xyz, P, om, dirs, ref = tube_case
    h = lib.wfq_build(xyz, GRAPHENE, store=("fp64", "fp32", "bf16"))
    tol = 1e-9
    out = lib.wfq_solve(h, om, dirs, tol, algorithm="msgmres", restart=30, precision=prec, shift_dim=400)
    h.close()
    assert out["status"] == 0, out["info"]
    for a in range(len(om)):
        for k in range(3):
            info = out["info"][a * 3 + k]
            assert info["status"] == 0 and info["relres"] <= tol, (a, k, info)
            q = out["q"][a, k]
            assert rel(q, ref[(a, k)]) <= 1e-6, (prec, a, k, rel(q, ref[(a, k)]))
            # charge conservation: 1^T L = 0 and 1^T b = 0 give z sum(q) = -sum(r) exactly, so
            # |sum q| <= sqrt(N) ||r|| / |z| (plus rounding)
            bn = np.linalg.norm(P.rhs(dirs[k]))
            bound = np.sqrt(P.n) * info["relres"] * bn / abs(P.z(om[a])) + 1e-9 * np.linalg.norm(q)
            assert abs(q.sum()) <= bound, (a, k, abs(q.sum()), bound)
    for a in range(len(om)):
        A = out["alpha"][a].T
        assert abs(A[0, 1] - A[1, 0]) <= 1e-6 * abs(A[0, 0])      # reciprocity
        assert A[0, 0].imag > 0 and A[2, 2].imag > 0


def test_closing_residual_is_that_of_the_returned_charges(lib, tube_case):
    # FP64 solves form T q of the shared-basis iterates from the kept products T v_j: the reported
    # relative residual must be the oracle's ||b - (L T + z I) q|| / ||b|| of the returned q
    xyz, P, om, dirs, ref = tube_case
    h = lib.wfq_build(xyz, GRAPHENE)
    tol = 1e-9
    out = lib.wfq_solve(h, om, dirs, tol, algorithm="msgmres", restart=30, precision="fp64", shift_dim=400)
    h.close()
    assert out["status"] == 0, out["info"]
    for a in range(len(om)):
        for k in range(3):
            info = out["info"][a * 3 + k]
            q = out["q"][a, k]
            r = P.residual(om[a], dirs[k], q)
            assert info["iters"] > 0 and info["cycles"] == 0, (a, k, info)
            assert abs(r - info["relres"]) <= 1e-3 * r + 1e-14, (a, k, r, info["relres"])


def test_multishift_steps_match_oracle(lib, tube_case):
    # FP64 T: the shared basis needs as many steps per frequency as the oracle's multi-shift GMRES
    # (same Krylov space, same stop rule ||r|| <= tol ||b||), and no refinement cycle afterwards
    xyz, P, om, dirs, ref = tube_case
    tol = 1e-8
    h = lib.wfq_build(xyz, GRAPHENE)
    out = lib.wfq_solve(h, om, dirs, tol, algorithm="msgmres", restart=30, precision="fp64", shift_dim=600)
    h.close()
    for k in range(3):
        X, oi = P.solve_multishift(om, dirs[k], tol, maxdim=600)
        for a in range(len(om)):
            info = out["info"][a * 3 + k]
            assert abs(info["iters"] - int(oi["iters"][a])) <= 2, (a, k, info["iters"], oi["iters"][a])
            assert info["cycles"] <= 1
            assert rel(out["q"][a, k], X[a]) <= 1e-6


def test_multishift_small_basis_falls_back(lib, tube_case):
    # a shared basis far too small for the tolerance: every system continues in batched GMRES from
    # the shared-basis iterate and still converges to the LU solution
    xyz, P, om, dirs, ref = tube_case
    tol = 1e-9
    h = lib.wfq_build(xyz, GRAPHENE)
    out = lib.wfq_solve(h, om[:3], dirs[:2], tol, algorithm="msgmres", restart=20, precision="fp64", shift_dim=8)
    h.close()
    assert out["status"] == 0
    for a in range(3):
        for k in range(2):
            info = out["info"][a * 2 + k]
            assert info["relres"] <= tol and info["iters"] > 8 and info["cycles"] >= 1
            assert rel(out["q"][a, k], ref[(a, k)]) <= 1e-6


def test_multishift_equals_batched_gmres(lib):
    # the disk workload, all three directions, several frequencies: the multi-shift result and the
    # batched GMRES result are the same solutions (both within tol of the exact one)
    wl = wi.workload("disk600")
    om = np.linspace(0.1, 1.2, 9)
    dirs = np.eye(3)
    h = lib.wfq_build(wl.xyz, wl.params)
    a = lib.wfq_solve(h, om, dirs, 1e-10, algorithm="msgmres", restart=50, precision="fp64")
    b = lib.wfq_solve(h, om, dirs, 1e-10, algorithm="gmres", restart=50, precision="fp64")
    h.close()
    assert a["status"] == 0 and b["status"] == 0
    for i in range(len(om)):
        for k in range(3):
            assert rel(a["q"][i, k], b["q"][i, k]) <= 1e-7
    # one shared basis per direction: far fewer T products than one basis per system
    assert max(r["iters"] for r in a["info"]) <= max(r["iters"] for r in b["info"]) + 2


def test_multishift_options_rejected(lib):
    wl = wi.workload("disk600")
    h = lib.wfq_build(wl.xyz, wl.params)
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_solve(h, [0.3], [[1, 0, 0]], 1e-8, algorithm="msgmres", shift_dim=5000)
    assert e.value.code == lib.WFQ_EINVAL
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_solve(h, [0.3], [[1, 0, 0]], 1e-8, algorithm="msgmres", restart=300)
    assert e.value.code == lib.WFQ_EINVAL
    h.close()
