"""Structures of two species and the material closure of W on the GPU, against the oracle (needs an
MI355X).

Each atom carries the hardness and r0 of its species; a pair of atoms of different species uses the
mean of their r0 in the Fermi damping and the cutoff. W comes from the material data (the Drude
sum-rule closure), computed by the library on the host and by the oracle from its own lattice sum.
"""

import numpy as np
import pytest

from oracle import wfq_oracle as O
from helpers import GRAPHENE, ragged_tube
import wfq_inputs as wi
from wfq_inputs import geometry as geo

pytestmark = pytest.mark.gpu

FCC = wi.workloads.FCC_METAL


def two_species(par, n, frac, seed):
    """par with a species table (species 0 = par's own eta and r0, species 1 harder and 4 % wider)
    and a seeded per-atom species array with about `frac` atoms of species 1."""
    sp = [(par["eta"], par["r0"]), (1.25 * par["eta"], 1.04 * par["r0"])]
    idx = (np.random.default_rng(seed).random(n) < frac).astype(np.int32)
    return dict(par, species=sp), idx


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


@pytest.fixture(scope="module")
def tube():
    xyz = ragged_tube()
    par, idx = two_species(GRAPHENE, len(xyz), 0.3, 5)
    return xyz, par, idx, O.Problem(xyz, par, species=idx)


@pytest.fixture(scope="module")
def sphere():
    xyz = geo.jitter(geo.fcc_sphere(11.0), 0.01, 8)
    par, idx = two_species(FCC, len(xyz), 0.5, 9)
    return xyz, par, idx, O.Problem(xyz, par, species=idx)


@pytest.mark.parametrize("which", ["tube", "sphere"])
def test_two_species_model_matrices(lib, request, which):
    xyz, par, idx, P = request.getfixturevalue(which)
    assert 0 < idx.sum() < len(idx)
    h = lib.wfq_build(xyz, par, species=idx)
    # T: per-species hardness on the diagonal and in the Gaussian widths of every pair
    rng = np.random.default_rng(3)
    i = np.concatenate([np.arange(P.n), rng.integers(0, P.n, 4000)])
    j = np.concatenate([np.arange(P.n), rng.integers(0, P.n, 4000)])
    t = lib.wfq_sample_T(h, "fp64", i, j)
    assert np.max(np.abs(t - P.T[i, j]) / np.abs(P.T[i, j])) < 1e-14
    # L: the same sparsity and values, pair r0 the mean of the two species' values
    r, c, v = lib.wfq_export_L(h)
    L = P.L.tocoo()
    mine = {(a, b): x for a, b, x in zip(r, c, v)}
    ref = {(a, b): x for a, b, x in zip(L.row, L.col, L.data)}
    # pairs that sit within rounding of their cutoff may fall on either side: their value is ~eps/r
    tiny = 1e-12 * np.max(np.abs(L.data))
    for k in set(mine) ^ set(ref):
        assert abs(mine.get(k, 0.0) - ref.get(k, 0.0)) <= tiny, k
    for k in set(mine) & set(ref):
        assert abs(mine[k] - ref[k]) <= 1e-13 * abs(ref[k]) + tiny, k
    h.close()


@pytest.mark.parametrize("which", ["tube", "sphere"])
def test_two_species_solutions_match_lu(lib, request, which):
    xyz, par, idx, P = request.getfixturevalue(which)
    h = lib.wfq_build(xyz, par, species=idx)
    om = np.array([0.2, 0.6, 1.0]) if which == "tube" else np.array([2.0, 4.0, 5.2])
    dirs = np.eye(3)
    out = lib.wfq_solve(h, om, dirs, 1e-9, algorithm="gmres", restart=80, precision="fp64")
    assert out["status"] == 0, out["info"]
    for a in range(len(om)):
        for k in range(3):
            q = P.solve_lu(om[a], dirs[k])
            assert rel(out["q"][a, k], q) <= 1e-7, (a, k)
            ref_alpha = O.polarisability(P.xyz, q[:, None])[:, 0]
            assert np.linalg.norm(out["alpha"][a, k] - ref_alpha) <= 1e-7 * np.linalg.norm(ref_alpha)
    h.close()


def test_two_species_through_the_server(lib, tube):
    # the server copies the species table and the per-atom indices before wfq_submit returns
    xyz, par, idx, P = tube
    s = lib.wfq_serve(1e-9, max_jobs=2, algorithm="gmres", restart=80)
    try:
        t = lib.wfq_submit(s, xyz, par, [0.6], np.eye(3)[:2], species=idx.copy())
        res = lib.wfq_wait(s, t)
    finally:
        lib.wfq_serve_stop(s)
    assert res["status"] == 0
    for k in range(2):
        assert rel(res["q"][0, k], P.solve_lu(0.6, np.eye(3)[k])) <= 1e-7


def test_bad_species_input_is_rejected(lib, tube):
    xyz, par, idx, _ = tube
    bad = idx.copy()
    bad[7] = 2                                   # only species 0 and 1 exist
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_build(xyz, par, species=bad)
    assert e.value.code == lib.WFQ_EINVAL
    with pytest.raises(lib.WfqError) as e:     # a species array without a table
        lib.wfq_build(xyz, GRAPHENE, species=idx)
    assert e.value.code == lib.WFQ_EINVAL


def test_material_weight_enters_the_operator(lib):
    # W only enters through z(omega) = -(omega^2 + i omega / tau) / W: a build given the closure's value
    # as an explicit override gives the same operator as the one that computes it from eps_F
    xyz = ragged_tube(periods=10)
    W = O.material_weight(GRAPHENE)
    h1 = lib.wfq_build(xyz, GRAPHENE)
    h2 = lib.wfq_build(xyz, dict(GRAPHENE, W=W))
    o1 = lib.wfq_solve(h1, [0.5], np.eye(3)[:1], 1e-10, algorithm="gmres", restart=80)
    o2 = lib.wfq_solve(h2, [0.5], np.eye(3)[:1], 1e-10, algorithm="gmres", restart=80)
    assert rel(o1["q"], o2["q"]) <= 1e-9
    h1.close()
    h2.close()
