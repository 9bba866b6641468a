"""J-symmetric QMR-from-BCG on the GPU against the oracle (needs an MI355X)."""

import numpy as np
import pytest

from oracle import wfq_oracle as O
from helpers import GRAPHENE, ragged_tube

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


@pytest.fixture(scope="module")
def case():
    xyz = ragged_tube()
    P = O.Problem(xyz, GRAPHENE)
    om = np.array([0.05, 0.31, 0.77, 1.0])
    dirs = np.eye(3)
    ref = {(a, k): P.solve_lu(om[a], dirs[k]) for a in range(len(om)) for k in range(3)}
    return xyz, P, om, dirs, ref


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_qmr_matches_lu(lib, case, prec):
    xyz, P, om, dirs, ref = case
    h = lib.wfq_build(xyz, GRAPHENE, store=("fp64", "fp32", "bf16"))
    tol = 1e-8
    out = lib.wfq_solve(h, om, dirs, tol, algorithm="qmr", restart=60, precision=prec)
    assert out["status"] == 0, out["info"]
    for a in range(len(om)):
        for k in range(3):
            info = out["info"][a * 3 + k]
            assert info["relres"] <= tol
            assert rel(out["q"][a, k], ref[(a, k)]) <= 1e-6
    h.close()


def test_qmr_iteration_count_matches_oracle(lib, case):
    # FP64 throughout and no refinement point before convergence: the GPU runs the oracle's recurrences
    xyz, P, om, dirs, ref = case
    h = lib.wfq_build(xyz, GRAPHENE)
    tol = 1e-8
    for a, k in ((1, 0), (3, 2)):
        out = lib.wfq_solve(h, om[a:a + 1], dirs[k:k + 1], tol, algorithm="qmr", restart=5000, precision="fp64")
        _, info = P.solve_qmr(om[a], dirs[k], 0.5 * tol)
        assert abs(out["info"][0]["iters"] - info["iters"]) <= 2, (out["info"][0]["iters"], info["iters"])
    h.close()


def test_qmr_needs_more_iterations_than_gmres(lib, case):
    # QMR quasi-minimises the residual, full GMRES minimises it: NI(QMR) >= NI(GMRES) without restarts
    xyz, P, om, dirs, ref = case
    h = lib.wfq_build(xyz, GRAPHENE)
    g = lib.wfq_solve(h, om[2:3], dirs[:1], 1e-8, algorithm="gmres", restart=250, precision="fp64")
    q = lib.wfq_solve(h, om[2:3], dirs[:1], 1e-8, algorithm="qmr", restart=5000, precision="fp64")
    assert q["info"][0]["iters"] >= g["info"][0]["iters"]
    h.close()


def test_qmr_breakdown_falls_back_to_gmres(lib, case):
    # QMR runs without look-ahead: when the bilinear form of a step is (near) zero the system leaves
    # QMR and continues in GMRES from its QMR iterate. A threshold that every step meets forces that
    # path on every system; the results must still be the LU solutions.
    xyz, P, om, dirs, ref = case
    h = lib.wfq_build(xyz, GRAPHENE)
    tol = 1e-8
    out = lib.wfq_solve(h, om, dirs, tol, algorithm="qmr", restart=60, precision="fp64", qmr_breakdown=1e30)
    assert out["status"] == 0, out["info"]
    for a in range(len(om)):
        for k in range(3):
            info = out["info"][a * 3 + k]
            assert info["status"] == 0 and info["relres"] <= tol
            assert info["iters"] > 0
            assert rel(out["q"][a, k], ref[(a, k)]) <= 1e-6
    # the same systems with the default threshold take the QMR route and agree
    plain = lib.wfq_solve(h, om, dirs, tol, algorithm="qmr", restart=60, precision="fp64")
    assert rel(plain["q"], out["q"]) <= 2e-6
    h.close()


def test_qmr_breakdown_threshold_is_checked(lib, case):
    xyz = case[0]
    h = lib.wfq_build(xyz, GRAPHENE)
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_solve(h, [0.3], np.eye(3)[:1], 1e-8, algorithm="qmr", qmr_breakdown=-1.0)
    assert e.value.code == lib.WFQ_EINVAL
    h.close()
