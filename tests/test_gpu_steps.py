"""Step-by-step parity of the HIP path against the CPU oracle (needs an MI355X).

Each stage of the hot path is called through the C interface and compared element by element
with the oracle on the same seeded structure: the damped Coulomb matrix in each storage precision,
the Drude Laplacian, the right-hand sides, the block product T X in each precision and every tile
variant, and the full operator (L T + z I) X.
"""

import numpy as np
import pytest

from oracle import wfq_oracle as O
from helpers import GRAPHENE, UNIT, ragged_tube, round_to
import wfq_inputs as wi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


@pytest.fixture(scope="module")
def tube():
    xyz = ragged_tube()                      # 1200 atoms: 4 full 256-tiles and a ragged tail
    return xyz, O.Problem(xyz, GRAPHENE)


@pytest.fixture(scope="module")
def handle(lib, tube):
    xyz, _ = tube
    h = lib.wfq_build(xyz, GRAPHENE, store=("fp64", "fp32", "bf16"))
    yield h
    h.close()


def test_T_elements_all_precisions(lib, handle, tube):
    _, P = tube
    n = P.n
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i, j = i.ravel(), j.ravel()
    ref = P.T[i, j]
    t64 = lib.wfq_sample_T(handle, "fp64", i, j)
    assert np.max(np.abs(t64 - ref) / np.abs(ref)) < 4e-16 * 8      # a few ulps (erf implementations)
    for prec in ("fp32", "bf16"):
        tp = lib.wfq_sample_T(handle, prec, i, j)
        # stored copy = FP64 value rounded to nearest; allow the FP64 ulps to flip a tie
        assert np.max(np.abs(tp - ref) / np.abs(ref)) <= UNIT[prec] * (1 + 1e-6)
        exact = tp == round_to(prec, ref)
        assert exact.mean() > 0.9999


def test_laplacian_structure_and_values(lib, handle, tube):
    _, P = tube
    r, c, v = lib.wfq_export_L(handle)
    L = P.L.tocoo()
    got = {(a, b): x for a, b, x in zip(r, c, v)}
    want = {(a, b): x for a, b, x in zip(L.row, L.col, L.data)}
    assert set(got) == set(want)                                     # same sparsity pattern, exactly
    keys = list(want)
    g = np.array([got[k] for k in keys])
    w = np.array([want[k] for k in keys])
    assert np.allclose(g, w, rtol=1e-13, atol=1e-16)
    rows = np.zeros(P.n)
    np.add.at(rows, r, v)
    assert np.max(np.abs(rows)) < 1e-14 * np.max(np.abs(v))


def test_rhs(lib, handle, tube):
    _, P = tube
    dirs = np.eye(3)
    b = lib.wfq_rhs(handle, dirs, E0=1.0)
    for k in range(3):
        ref = P.rhs(dirs[k])
        # b is a short sum of large terms (positions times L): bound the rounding by |L| |r . k|
        scale = np.abs(P.L) @ np.abs(P.xyz @ dirs[k])
        assert np.all(np.abs(b[k] - ref) <= 64 * UNIT["fp64"] * scale)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("ncol", [1, 2, 5, 8, 9, 24, 32, 33, 64, 65, 130])
def test_block_product(lib, handle, tube, prec, ncol):
    _, P = tube
    rng = np.random.default_rng(100 + ncol)
    X = rng.standard_normal((ncol, P.n))
    Y = lib.wfq_apply_T(handle, prec, X)
    Tq = round_to(prec, P.T)
    Xq = round_to(prec, X)
    ref = Xq @ Tq                     # T symmetric: row c of Y is T x_c
    bound = np.abs(Xq) @ np.abs(Tq)
    # accumulation error of an n-term sum in the accumulator precision (FP64 or FP32)
    u_acc = UNIT["fp64"] if prec == "fp64" else UNIT["fp32"]
    assert np.all(np.abs(Y - ref) <= 2 * P.n * u_acc * bound + 1e-300)


def test_block_product_larger_than_staging_chunk(lib, handle, tube):
    # 3500 columns: X and Y are 35.8 MB each, more than the 32 MiB pinned staging chunk through which
    # host arrays are copied, so both copy directions take more than one chunk
    _, P = tube
    rng = np.random.default_rng(77)
    X = rng.standard_normal((3500, P.n))
    Y = lib.wfq_apply_T(handle, "fp64", X)
    ref = X @ P.T
    bound = np.abs(X) @ np.abs(P.T)
    # element by element within the accumulation bound: a chunk copied to a wrong offset (or not at
    # all) would put whole rows of Y far outside it
    assert np.all(np.abs(Y - ref) <= 2 * P.n * UNIT["fp64"] * bound + 1e-300)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_every_block_product_variant(lib, handle, tube, prec):
    # each shape the autotuner may choose, at ragged widths (partial column tiles, split k parts)
    _, P = tube
    Tq = round_to(prec, P.T)
    u_acc = UNIT["fp64"] if prec == "fp64" else UNIT["fp32"]
    rng = np.random.default_rng(31)
    for name, max_ncol in lib.wfq_tx_variants(prec):
        widths = [max_ncol, max_ncol - 1] if max_ncol < 64 else [3, 97, 200]
        for ncol in widths:
            if ncol < 1:
                continue
            X = rng.standard_normal((ncol, P.n))
            Y = lib.wfq_apply_T_variant(handle, prec, name, X)
            Xq = round_to(prec, X)
            ref = Xq @ Tq
            bound = np.abs(Xq) @ np.abs(Tq)
            assert np.all(np.abs(Y - ref) <= 2 * P.n * u_acc * bound + 1e-300), (name, ncol)


def test_variant_entry_point_rejects(lib, handle):
    X = np.ones((5, handle.n))
    with pytest.raises(lib.WfqError):
        lib.wfq_apply_T_variant(handle, "fp32", "skinny4", X)       # 5 columns > 4
    with pytest.raises(lib.WfqError):
        lib.wfq_apply_T_variant(handle, "fp32", 10 ** 6, X)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_operator_apply(lib, handle, tube, prec):
    _, P = tube
    rng = np.random.default_rng(7)
    S = 5
    X = rng.standard_normal((S, P.n)) + 1j * rng.standard_normal((S, P.n))
    z = np.array([P.z(om) for om in (0.05, 0.2, 0.4, 0.7, 1.0)])
    Y = lib.wfq_apply_op(handle, prec, z, X)
    L = P.L
    for s in range(S):
        if prec == "fp64":
            ref = L @ (P.T @ X[s]) + z[s] * X[s]
            scale = np.abs(L) @ (np.abs(P.T) @ np.abs(X[s])) + np.abs(z[s] * X[s])
            assert np.all(np.abs(Y[s] - ref) <= 1e-12 * scale)
        else:
            Tq = round_to(prec, P.T)
            xr, xi = round_to(prec, X[s].real), round_to(prec, X[s].imag)
            ty = Tq @ xr + 1j * (Tq @ xi)
            ref = L @ ty + z[s] * X[s]
            scale = np.abs(L) @ (np.abs(Tq) @ (np.abs(xr) + np.abs(xi))) + np.abs(z[s] * X[s])
            assert np.all(np.abs(Y[s] - ref) <= 2 * P.n * UNIT["fp32"] * scale)


def test_small_structure_dimer(lib):
    # N = 2: one 256-tile of padding around two atoms
    xyz = np.array([[0.0, 0.0, 0.0], [1.7, 0.0, 0.0]])
    P = O.Problem(xyz, GRAPHENE)
    h = lib.wfq_build(xyz, GRAPHENE)
    t = lib.wfq_sample_T(h, "fp64", [0, 0, 1, 1], [0, 1, 0, 1])
    assert np.allclose(t, P.T.ravel(), rtol=1e-15)
    Y = lib.wfq_apply_T(h, "fp64", np.array([[1.0, -2.0]]))
    assert np.allclose(Y[0], P.T @ np.array([1.0, -2.0]), rtol=1e-14)
    h.close()
