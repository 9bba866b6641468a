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
