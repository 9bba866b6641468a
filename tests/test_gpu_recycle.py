"""Subspace recycling across a frequency sweep on the GPU, against the oracle (needs an MI355X).

Every second frequency (and the highest) is solved from zero; each other one by GMRES augmented
with the span of its nearest solved neighbours' solutions (GCRO). The results must be the LU
solutions, the iteration counts those of the oracle's recycled sweep, and fewer than with
interpolated warm starts.
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


@pytest.fixture(scope="module")
def sweep():
    xyz = ragged_tube(periods=30)
    P = O.Problem(xyz, GRAPHENE)
    om = np.linspace(0.05, 1.2, 12)
    d = np.array([0.0, 0.0, 1.0])
    ref = np.array([P.solve_lu(w, d) for w in om])
    return xyz, P, om, d, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_recycled_sweep_matches_lu(lib, sweep, prec):
    xyz, P, om, d, ref = sweep
    h = lib.wfq_build(xyz, GRAPHENE)
    out = lib.wfq_solve(h, om, d[None], 1e-8, algorithm="gmres", restart=30, precision=prec, recycle=4)
    h.close()
    assert out["status"] == 0, out["info"]
    for a in range(len(om)):
        assert out["info"][a]["relres"] <= 1e-8
        assert np.linalg.norm(out["q"][a, 0] - ref[a]) <= 1e-6 * np.linalg.norm(ref[a])


def test_recycled_sweep_iterations_match_the_oracle(lib, sweep):
    xyz, P, om, d, ref = sweep
    h = lib.wfq_build(xyz, GRAPHENE)
    out = lib.wfq_solve(h, om, d[None], 1e-8, algorithm="gmres", restart=30, precision="fp64", recycle=4)
    h.close()
    _, it_ref, first = P.solve_recycled_sweep(om, d, 30, 0.5e-8, 4)
    it = np.array([r["iters"] for r in out["info"]])
    # the library's inner stop is at half the tolerance, the oracle's explicit check at 0.5e-8 here
    assert np.all(np.abs(it - it_ref) <= np.maximum(3, 0.15 * it_ref)), (it.tolist(), it_ref.tolist())


def test_recycling_saves_iterations_against_warm_starts(lib, sweep):
    xyz, P, om, d, ref = sweep
    h = lib.wfq_build(xyz, GRAPHENE)
    rec = lib.wfq_solve(h, om, d[None], 1e-8, algorithm="gmres", restart=30, recycle=4, want_q=False)
    warm = lib.wfq_solve(h, om, d[None], 1e-8, algorithm="gmres", restart=30, warm_start=True, want_q=False)
    zero = lib.wfq_solve(h, om, d[None], 1e-8, algorithm="gmres", restart=30, want_q=False)
    h.close()
    n_rec = sum(r["iters"] for r in rec["info"])
    n_warm = sum(r["iters"] for r in warm["info"])
    n_zero = sum(r["iters"] for r in zero["info"])
    print(f"iterations over the sweep: q0 = 0 {n_zero}, warm starts {n_warm}, recycling {n_rec}")
    assert n_rec < n_warm < n_zero


def test_recycling_options(lib, sweep):
    xyz, P, om, d, ref = sweep
    h = lib.wfq_build(xyz, GRAPHENE)
    for bad in (dict(recycle=9), dict(recycle=-1), dict(recycle=2, algorithm="qmr"),
                dict(recycle=2, algorithm="msgmres"), dict(recycle=2, block_jacobi=True)):
        opts = dict(dict(algorithm="gmres", restart=30), **bad)
        with pytest.raises(lib.WfqError) as e:
            lib.wfq_solve(h, om[:3], d[None], 1e-8, **opts)
        assert e.value.code == lib.WFQ_EINVAL, bad
    # fewer than three frequencies: plain GMRES from zero, the same counts as without the option
    a = lib.wfq_solve(h, om[:2], d[None], 1e-8, algorithm="gmres", restart=30, recycle=4)
    b = lib.wfq_solve(h, om[:2], d[None], 1e-8, algorithm="gmres", restart=30)
    assert [r["iters"] for r in a["info"]] == [r["iters"] for r in b["info"]]
    h.close()
