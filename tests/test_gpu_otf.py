"""Matrix-free (on-the-fly) T products and solves against the oracle (needs an MI355X)."""

import numpy as np
import pytest

from oracle import wfq_oracle as O
from helpers import GRAPHENE, UNIT, ragged_tube, round_to

pytestmark = pytest.mark.gpu

# FP32 elements use a rational/exponential erf with absolute error <= 1.5e-7 (relative <= 3e-7
# for the arguments >= 1/2 where it is used) and the Maclaurin series below 1/2.
ERF_REL = 3.2e-7


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


@pytest.fixture(scope="module")
def tube():
    xyz = ragged_tube()
    return xyz, O.Problem(xyz, GRAPHENE)


@pytest.mark.parametrize("ncol", [1, 2, 31, 32, 33, 64])
def test_otf_products(lib, tube, ncol):
    xyz, P = tube
    h = lib.wfq_build(xyz, GRAPHENE, t_mode="otf")
    X = np.random.default_rng(ncol).standard_normal((ncol, P.n))
    bound = np.abs(X) @ np.abs(P.T)
    Y64 = lib.wfq_apply_T(h, "fp64", X)
    assert np.all(np.abs(Y64 - X @ P.T) <= 64 * UNIT["fp64"] * bound + 1e-300)
    Y32 = lib.wfq_apply_T(h, "fp32", X)
    Xq = round_to("fp32", X)
    ref = Xq @ P.T
    # element error (erf approximation + FP32 geometry) + accumulation inside 64-source tiles (FP32)
    tol = (ERF_REL + 16 * UNIT["fp32"] + 2 * 64 * UNIT["fp32"]) * (np.abs(Xq) @ np.abs(P.T))
    assert np.all(np.abs(Y32 - ref) <= tol)
    h.close()


def test_otf_element_accuracy_across_branch(lib):
    # a dimer scanned through r / sqrt(d_i^2 + d_j^2) = 0.05 .. 6: T_12 from the product with e_2
    eta = 0.6
    d = np.sqrt(2 / np.pi) / eta
    sig = np.sqrt(2) * d
    worst = 0.0
    for x in np.concatenate([np.linspace(0.05, 0.95, 19), np.linspace(1.0, 6.0, 11)]):
        r_bohr = x * sig
        xyz = np.array([[0.0, 0.0, 0.0], [r_bohr * O.BOHR_A, 0.0, 0.0]])
        P = O.Problem(xyz, dict(GRAPHENE, eta=eta))
        h = lib.wfq_build(xyz, dict(GRAPHENE, eta=eta), t_mode="otf")
        y = lib.wfq_apply_T(h, "fp32", np.array([[0.0, 1.0]]))[0]
        h.close()
        worst = max(worst, abs(y[0] - P.T[0, 1]) / P.T[0, 1])
    assert worst <= ERF_REL + 8 * UNIT["fp32"]


def test_otf_matches_stored_fp64(lib, tube):
    xyz, P = tube
    hs = lib.wfq_build(xyz, GRAPHENE)
    ho = lib.wfq_build(xyz, GRAPHENE, t_mode="otf")
    X = np.random.default_rng(3).standard_normal((8, P.n))
    a = lib.wfq_apply_T(hs, "fp64", X)
    b = lib.wfq_apply_T(ho, "fp64", X)
    assert np.all(np.abs(a - b) <= 64 * UNIT["fp64"] * (np.abs(X) @ np.abs(P.T)))
    hs.close()
    ho.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_otf_solve_matches_lu(lib, tube, prec):
    xyz, P = tube
    h = lib.wfq_build(xyz, GRAPHENE, t_mode="otf")
    om = np.array([0.15, 0.6])
    dirs = np.eye(3)[:2]
    out = lib.wfq_solve(h, om, dirs, 1e-8, restart=60, precision=prec)
    assert out["status"] == 0
    for a in range(2):
        for k in range(2):
            ref = P.solve_lu(om[a], dirs[k])
            q = out["q"][a, k]
            assert np.linalg.norm(q - ref) / np.linalg.norm(ref) <= 1e-6
            assert out["info"][a * 2 + k]["relres"] <= 1e-8
    with pytest.raises(lib.WfqError):
        lib.wfq_solve(h, om, dirs, 1e-8, precision="bf16")
    h.close()


@pytest.mark.parametrize("ncol", [1, 2, 3, 4])
def test_narrow_recomputed_product_on_a_metal_sphere(lib, ncol):
    # The narrow FP64 product that recomputes T's elements (far-field 1/r for every pair plus the
    # sparse near-field correction) on a 1 433-atom FCC sphere, where every atom has hundreds of
    # neighbours inside the near-field radius: against the oracle's dense T, through the registered
    # variants of a stored handle and through a matrix-free handle.
    import wfq_inputs as wi
    from wfq_inputs import geometry as geo
    xyz = geo.jitter(geo.fcc_sphere(18.0), 0.02, 3)
    par = wi.workloads.FCC_METAL
    P = O.Problem(xyz, par)
    X = np.random.default_rng(ncol).standard_normal((ncol, P.n))
    ref = X @ P.T.T
    bound = np.abs(X) @ np.abs(P.T).T
    names = [v[0] for v in lib.wfq_tx_variants("fp64")]
    h = lib.wfq_build(xyz, par, store=("fp64",))
    for var in ("otfn2", "otfn4"):
        k = names.index(var)
        if ncol > dict(lib.wfq_tx_variants("fp64"))[var]:
            continue
        Y = lib.wfq_apply_T_variant(h, "fp64", k, X)
        assert np.all(np.abs(Y - ref) <= 1e-13 * bound), var
    h.close()
    hf = lib.wfq_build(xyz, par, t_mode="otf")
    Y = lib.wfq_apply_T(hf, "fp64", X)
    assert np.all(np.abs(Y - ref) <= 1e-13 * bound)
    hf.close()


def test_matrix_free_fp64_product_in_chunks(lib):
    # matrix-free FP64 products of up to 12 columns run as narrow products of 4 columns each
    xyz = ragged_tube()
    P = O.Problem(xyz, GRAPHENE)
    X = np.random.default_rng(8).standard_normal((11, P.n))
    hf = lib.wfq_build(xyz, GRAPHENE, t_mode="otf")
    Y = lib.wfq_apply_T(hf, "fp64", X)
    hf.close()
    assert np.all(np.abs(Y - X @ P.T.T) <= 1e-13 * (np.abs(X) @ np.abs(P.T).T))


@pytest.mark.parametrize("ncol", [1, 2, 3, 4])
def test_symmetric_narrow_product_on_a_large_sphere(lib, ncol):
    # From 65 536 atoms on, the narrow product evaluates each pair of atoms once for both rows (blocks
    # of 1 024 atoms, the source-side sums rotated across the lanes, block contributions added in
    # order). A 72k-atom FCC sphere whose last block is partial, against the C++ oracle's pairwise
    # rows: every 997th row and the last five.
    import wfq_inputs as wi
    from wfq_inputs import geometry as geo
    from oracle.cpp_oracle import CppProblem
    par = wi.workloads.FCC_METAL
    xyz = geo.jitter(geo.fcc_sphere(66.0), 0.02, 11)
    n = len(xyz)
    assert n >= 65536 and n % 1024 != 0
    X = np.random.default_rng(40 + ncol).standard_normal((ncol, n))
    hf = lib.wfq_build(xyz, par, t_mode="otf")
    Y = lib.wfq_apply_T(hf, "fp64", X)
    hf.close()
    P = CppProblem(xyz, par, dense_T=False, build_L=False)
    rows = np.r_[np.arange(0, n, 997), np.arange(n - 5, n)]
    ref = P.apply_T_rows(rows, X.T)
    bound = P.apply_T_rows(rows, np.abs(X).T)
    assert np.all(np.abs(Y[:, rows].T - ref) <= 1e-13 * bound)


@pytest.mark.parametrize("case", ["tube", "sphere"])
def test_narrow_fp64_product_moved_away_from_the_origin(lib, case):
    # T depends on distances only. Both narrow FP64 kernels (one-sided on the 1 200-atom tube,
    # symmetric on a 72k-atom sphere) take coordinates relative to an origin inside the work-group and
    # form r^2 by expansion where the blocks' bounding spheres keep its rounding small, so the product
    # of the structure moved by about 1 200 A equals the oracle's (and the unmoved product) to rounding.
    shift = np.array([700.0, -400.0, 900.0])
    if case == "tube":
        xyz, par = ragged_tube(), GRAPHENE
    else:
        import wfq_inputs as wi
        from wfq_inputs import geometry as geo
        par = wi.workloads.FCC_METAL
        xyz = geo.jitter(geo.fcc_sphere(66.0), 0.02, 11)
    n = len(xyz)
    X = np.random.default_rng(77).standard_normal((3, n))
    Y = []
    for p in (xyz, xyz + shift):
        h = lib.wfq_build(p, par, t_mode="otf")
        Y.append(lib.wfq_apply_T(h, "fp64", X))
        h.close()
    if case == "tube":
        P = O.Problem(xyz, par)
        rows = np.arange(n)
        ref, bound = (X @ P.T).T, (np.abs(X) @ np.abs(P.T)).T
    else:
        from oracle.cpp_oracle import CppProblem
        P = CppProblem(xyz, par, dense_T=False, build_L=False)
        rows = np.r_[np.arange(0, n, 1499), np.arange(n - 3, n)]
        ref, bound = P.apply_T_rows(rows, X.T), P.apply_T_rows(rows, np.abs(X).T)
    for y in Y:
        assert np.all(np.abs(y[:, rows].T - ref) <= 1e-13 * bound)
    assert np.all(np.abs(Y[1][:, rows] - Y[0][:, rows]).T <= 2e-13 * bound)
