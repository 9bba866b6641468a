"""Failure and warning paths of the library on the GPU, each checked against the oracle where it has
a result (needs an MI355X): device budgets that cannot hold the structure or one system's Krylov work
space (WFQ_ENOMEM), a structure whose Kbar graph has two components (WFQ_EDISCONNECTED: each
component conserves its own charge), and frequencies at or below zero (WFQ_ESINGULAR)."""

import numpy as np
import pytest

from oracle import wfq_oracle as O
from wfq_inputs import geometry as geo
from helpers import GRAPHENE

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_budget_below_structure_is_enomem(lib):
    xyz = geo.jitter(geo.graphene_disk(14.0), 0.01, 41)
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_build(xyz, GRAPHENE, budget=1 << 16)
    assert e.value.code == lib.WFQ_ENOMEM


def test_budget_below_one_system_is_enomem(lib):
    # a budget that holds the structure (T in FP64 and FP32, L) but not one system's GMRES(200) basis
    xyz = geo.jitter(geo.graphene_disk(20.0), 0.01, 42)
    h0 = lib.wfq_build(xyz, GRAPHENE)
    need = lib.wfq_info(h0)["bytes"]
    h0.close()
    h = lib.wfq_build(xyz, GRAPHENE, budget=need + (1 << 20))
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_solve(h, [0.3], np.eye(3)[:1], 1e-8, restart=200, precision="fp64")
    assert e.value.code == lib.WFQ_ENOMEM
    # with room for the work space the same handle solves
    h.close()
    h = lib.wfq_build(xyz, GRAPHENE, budget=need + (256 << 20))
    out = lib.wfq_solve(h, [0.3], np.eye(3)[:1], 1e-8, restart=200, precision="fp64")
    assert out["status"] == 0
    h.close()


def test_disconnected_structure_conserves_charge_per_component(lib):
    # two disks 30 Angstrom apart: no Kbar coupling between them (cutoff 5.2 Angstrom), T couples them
    a = geo.graphene_disk(9.0)
    b = geo.graphene_disk(7.0) + np.array([40.0, 0.0, 0.0])
    xyz = geo.jitter(np.vstack([a, b]), 0.01, 43)
    na = len(a)
    h = lib.wfq_build(xyz, GRAPHENE)
    assert h.build_status == lib.WFQ_EDISCONNECTED
    P = O.Problem(xyz, GRAPHENE)
    om = np.array([0.2, 0.9])
    dirs = np.eye(3)[:2]
    out = lib.wfq_solve(h, om, dirs, 1e-9, restart=60, precision="fp64")
    assert out["status"] == 0
    for i in range(len(om)):
        for k in range(len(dirs)):
            q = out["q"][i, k]
            ref = P.solve_lu(om[i], dirs[k])
            assert rel(q, ref) <= 1e-6
            for part in (q[:na], q[na:]):
                assert abs(part.sum()) <= 1e-9 * np.linalg.norm(q)
    h.close()


def test_nonpositive_frequency_is_singular(lib):
    xyz = geo.jitter(geo.graphene_disk(10.0), 0.01, 44)
    h = lib.wfq_build(xyz, GRAPHENE)
    for om in ([0.0], [0.3, -0.1]):
        with pytest.raises(lib.WfqError) as e:
            lib.wfq_solve(h, om, np.eye(3)[:1], 1e-8)
        assert e.value.code == lib.WFQ_ESINGULAR
    h.close()
