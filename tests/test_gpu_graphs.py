"""Inner-iteration chunks replayed as HIP graphs (needs an MI355X).

A chunk of steps runs eagerly the first time its launch sequence is seen, is captured the second
time and replayed after that. Captured and replayed chunks launch the same kernels with the same
arguments as the eager ones, so every solve must be bitwise identical to the same solve with graphs
switched off: q, alpha, iteration and cycle counts, and the FP64 relative residual. Each test
repeats the solve several times on one handle (eager, capture, replays) with other eager work and
host synchronisations in between, and checks every repetition; the solutions themselves are checked
against the CPU oracle's dense LU solution.
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


def same(a, b):
    assert a["status"] == b["status"]
    assert np.array_equal(a["q"], b["q"])
    assert np.array_equal(a["alpha"], b["alpha"])
    for ra, rb in zip(a["info"], b["info"]):
        for k in ("status", "iters", "cycles", "precision", "relres"):
            assert ra[k] == rb[k], (k, ra, rb)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_gmres_replays_match_eager(lib):
    # the disk workload, one system, FP64 GMRES(20): several restart cycles, so the chunk keys of
    # the first cycle repeat inside one solve as well as across solves
    wl = wi.workload("disk600")
    h = lib.wfq_build(wl.xyz, wl.params)
    om, d = [0.3], [[1.0, 0.0, 0.0]]
    ref = lib.wfq_solve(h, om, d, 1e-10, restart=20, precision="fp64", graphs=False)
    assert ref["status"] == 0 and ref["info"][0]["cycles"] >= 2
    P = O.Problem(wl.xyz, wl.params)
    assert rel(ref["q"][0, 0], P.solve_lu(0.3, np.array(d[0]))) <= 1e-6
    for rep in range(4):
        out = lib.wfq_solve(h, om, d, 1e-10, restart=20, precision="fp64", graphs=True)
        same(out, ref)
        # eager work on the handle's stream between the replays
        x = np.random.default_rng(rep).standard_normal((2, h.n))
        lib.wfq_apply_T(h, "fp64", x)
    h.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batched_mixed_groups_replay(lib, prec):
    # 5 frequencies x 2 directions on a ragged tube in reduced precision with escalation: precision
    # groups and list sizes change between chunks, each change is its own graph
    xyz = ragged_tube()
    h = lib.wfq_build(xyz, GRAPHENE, store=("fp64", "fp32", "bf16"))
    om = [0.05, 0.2, 0.4, 0.8, 1.3]
    dirs = [[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]
    ref = lib.wfq_solve(h, om, dirs, 1e-9, restart=16, precision=prec, graphs=False)
    assert ref["status"] == 0
    outs = [lib.wfq_solve(h, om, dirs, 1e-9, restart=16, precision=prec, graphs=True) for _ in range(3)]
    for out in outs:
        same(out, ref)
    P = O.Problem(xyz, GRAPHENE)
    for a in (0, 3):
        assert rel(ref["q"][a, 1], P.solve_lu(om[a], np.array(dirs[1]))) <= 1e-6
    h.close()


def test_multishift_replays_match_eager(lib):
    # 40 frequencies x 3 directions through the shared-basis phase and the batched GMRES after it
    wl = wi.workload("disk600")
    h = lib.wfq_build(wl.xyz, wl.params)
    om = np.linspace(0.05, 1.5, 40)
    dirs = np.eye(3)
    ref = lib.wfq_solve(h, om, dirs, 1e-10, algorithm="msgmres", restart=50, precision="fp64", graphs=False)
    assert ref["status"] == 0
    for _ in range(3):
        same(lib.wfq_solve(h, om, dirs, 1e-10, algorithm="msgmres", restart=50, precision="fp64", graphs=True), ref)
    P = O.Problem(wl.xyz, wl.params)
    for a in (0, 17, 39):
        assert rel(ref["q"][a, 1], P.solve_lu(om[a], dirs[1])) <= 1e-6
    h.close()


def test_shape_change_and_tuning_invalidate(lib):
    # alternating shapes replace the handle's work space (and its graphs); tuning the block product
    # changes the launch sequence, so graphs captured before it must not be replayed after it
    wl = wi.workload("disk600")
    h = lib.wfq_build(wl.xyz, wl.params)
    om, d = [0.2, 0.5, 0.9], [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]
    ref_a = lib.wfq_solve(h, om, d, 1e-10, restart=30, precision="fp64", graphs=False)
    ref_b = lib.wfq_solve(h, om[:1], d[:1], 1e-10, restart=30, precision="fp64", graphs=False)
    for _ in range(2):
        same(lib.wfq_solve(h, om, d, 1e-10, restart=30, precision="fp64", graphs=True), ref_a)
        same(lib.wfq_solve(h, om, d, 1e-10, restart=30, precision="fp64", graphs=True), ref_a)
        same(lib.wfq_solve(h, om[:1], d[:1], 1e-10, restart=30, precision="fp64", graphs=True), ref_b)
    lib.wfq_solve(h, om, d, 1e-10, restart=30, precision="fp64", graphs=True)
    lib.wfq_solve(h, om, d, 1e-10, restart=30, precision="fp64", graphs=True)   # captured
    lib.wfq_tune(h, "fp64", [2, 4, 6, 12], reps=2)
    ref_t = lib.wfq_solve(h, om, d, 1e-10, restart=30, precision="fp64", graphs=False)
    for _ in range(3):
        same(lib.wfq_solve(h, om, d, 1e-10, restart=30, precision="fp64", graphs=True), ref_t)
    for i in range(len(om)):
        for k in range(len(d)):
            assert rel(ref_t["q"][i, k], ref_a["q"][i, k]) <= 1e-9
    h.close()
