"""Warm starts across neighbouring frequencies against the CPU oracle (needs an MI355X).

With warm_start, every second frequency (and the highest) of each direction is solved from q0 = 0 and
each other system starts from the straight-line interpolation in z of its two solved neighbours.
References: the oracle's dense LU solution of every system (the result), and the oracle's own warm
sweep (the number of GMRES steps the interpolated start saves).
"""

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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def tube():
    xyz = ragged_tube()
    return xyz, O.Problem(xyz, GRAPHENE)


def test_warm_sweep_matches_lu_and_oracle_steps(lib, tube):
    xyz, P = tube
    # frequencies given out of order: the pairing follows sorted frequency, per direction
    om = np.array([0.6, 0.2, 1.0, 0.4, 0.3, 0.8, 0.5, 0.9, 0.7])
    dirs = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    tol = 1e-10
    h = lib.wfq_build(xyz, GRAPHENE)
    # GMRES(100): no restart within these step counts, so the GPU and the oracle build the same Krylov
    # space from the same start; the GPU's inner target is half the outer tolerance (a step or two more)
    warm = lib.wfq_solve(h, om, dirs, tol, restart=100, precision="fp64", warm_start=True)
    cold = lib.wfq_solve(h, om, dirs, tol, restart=100, precision="fp64")
    h.close()
    assert warm["status"] == 0 and cold["status"] == 0
    for k in range(2):
        Qo, it_o, first = P.solve_warm_sweep(om, dirs[k], restart=100, tol=tol)
        assert first.tolist() == [True, True, True, True, False, True, False, False, False]
        for a in range(len(om)):
            info = warm["info"][a * 2 + k]
            assert info["status"] == 0 and info["relres"] <= tol
            ref = P.solve_lu(om[a], dirs[k])
            assert rel(warm["q"][a, k], ref) <= 1e-6, (a, k)
            if first[a]:
                # solved from zero: the same solve as without warm starts
                # (the narrower block product may round differently: one step either way)
                assert abs(info["iters"] - cold["info"][a * 2 + k]["iters"]) <= 1
            else:
                # same start (up to the neighbours' 1e-10 residuals), same Krylov space: the oracle's
                # step count, and fewer steps than from zero. The start's residual is close to the
                # tolerance, so the step that crosses it moves by one with the rounding order of the
                # products (the oracle alone: 31 or 32 steps for one system), and the GPU stops on half
                # the tolerance (one or two more)
                assert -1 <= info["iters"] - int(it_o[a]) <= 4, (a, k, info["iters"], it_o[a])
                assert info["iters"] < cold["info"][a * 2 + k]["iters"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_warm_sweep_mixed_precision(lib, tube, prec):
    xyz, P = tube
    om = np.linspace(0.1, 1.2, 12)
    d = np.array([[0.0, 1.0, 0.0]])
    tol = 1e-9
    h = lib.wfq_build(xyz, GRAPHENE, store=("fp64", "fp32", "bf16"))
    warm = lib.wfq_solve(h, om, d, tol, restart=20, precision=prec, warm_start=True)
    cold = lib.wfq_solve(h, om, d, tol, restart=20, precision=prec)
    h.close()
    assert warm["status"] == 0
    for a in range(len(om)):
        assert warm["info"][a]["relres"] <= tol
        assert rel(warm["q"][a, 0], P.solve_lu(om[a], d[0])) <= 1e-6
    assert sum(r["iters"] for r in warm["info"]) < sum(r["iters"] for r in cold["info"])


def test_warm_start_small_batches_and_rejects(lib, tube):
    # batches smaller than the sweep: each batch plans its own pairs; two frequencies: no warm pass
    xyz, P = tube
    om = np.linspace(0.2, 0.9, 7)
    d = np.array([[1.0, 0.0, 0.0]])
    h = lib.wfq_build(xyz, GRAPHENE)
    out = lib.wfq_solve(h, om, d, 1e-10, restart=20, precision="fp64", warm_start=True, max_batch=3)
    assert out["status"] == 0
    for a in range(len(om)):
        assert rel(out["q"][a, 0], P.solve_lu(om[a], d[0])) <= 1e-6
    two = lib.wfq_solve(h, om[:2], d, 1e-10, restart=20, precision="fp64", warm_start=True)
    ref = lib.wfq_solve(h, om[:2], d, 1e-10, restart=20, precision="fp64")
    assert [r["iters"] for r in two["info"]] == [r["iters"] for r in ref["info"]]
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_solve(h, om, d, 1e-10, algorithm="qmr", warm_start=True)
    assert e.value.code == lib.WFQ_EINVAL
    h.close()
