"""Block-Jacobi right preconditioning of the batched GMRES against the CPU oracle (needs an MI355X).

The library's blocks are runs of 64 atoms in its internal order, which wfq_export_L reveals (its
triplets come row by row in that order); the oracle's `solve_block_jacobi` is given the same index
sets. References: the oracle's dense LU solution of every system (the result) and the oracle's own
block-Jacobi GMRES (the number of steps, which depends on the preconditioner actually applied).
"""

import numpy as np
import pytest

from oracle import wfq_oracle as O
import wfq_inputs as wi
from helpers import GRAPHENE, ragged_tube

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def internal_blocks(lib, h):
    rows, _, _ = lib.wfq_export_L(h)
    _, first = np.unique(rows, return_index=True)
    order = rows[np.sort(first)]
    assert sorted(order.tolist()) == list(range(h.n))
    return [order[k:k + 64] for k in range(0, h.n, 64)]


@pytest.fixture(scope="module")
def tube():
    xyz = ragged_tube()   # 1200 atoms: 18 full blocks, a block of 48 atoms and one of padding only
    return xyz, O.Problem(xyz, GRAPHENE)


@pytest.fixture(scope="module")
def disk():
    wl = wi.workload("disk600")   # 612 atoms
    return wl, O.Problem(wl.xyz, wl.params)


@pytest.mark.parametrize("which", ["tube", "disk"])
def test_block_jacobi_matches_lu_and_oracle_steps(lib, tube, disk, which):
    if which == "tube":
        xyz, P = tube
        params, dirs, om = GRAPHENE, np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]]), np.array([0.3, 1.0, 1.5])
    else:
        wl, P = disk
        xyz, params = wl.xyz, wl.params
        dirs, om = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]), np.array([0.3, 1.0, 1.5])
    tol = 1e-10
    h = lib.wfq_build(xyz, params)
    blocks = internal_blocks(lib, h)
    # GMRES(150): no restart within these step counts, so both sides build the same Krylov space
    pre = lib.wfq_solve(h, om, dirs, tol, restart=150, precision="fp64", block_jacobi=True)
    plain = lib.wfq_solve(h, om, dirs, tol, restart=150, precision="fp64")
    h.close()
    assert pre["status"] == 0 and plain["status"] == 0
    for a in range(len(om)):
        for k in range(len(dirs)):
            info = pre["info"][a * len(dirs) + k]
            assert info["status"] == 0 and info["relres"] <= tol
            ref = P.solve_lu(om[a], dirs[k])
            assert rel(pre["q"][a, k], ref) <= 1e-6, (a, k)
            _, oi = P.solve_block_jacobi(om[a], dirs[k], blocks, restart=150, tol=tol)
            # the GPU's inner target is half the outer tolerance: a step or two more
            assert -1 <= info["iters"] - oi["iters"] <= 3, (a, k, info["iters"], oi["iters"])
    if which == "disk":
        # the disk above its lowest resonances: far fewer steps than without the preconditioner
        for a in (1, 2):
            for k in range(len(dirs)):
                s = a * len(dirs) + k
                assert pre["info"][s]["iters"] < 0.7 * plain["info"][s]["iters"], (a, k)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_block_jacobi_mixed_precision_restarts_batches(lib, disk, prec):
    # narrow block products inside FP64 refinement, GMRES(10) (the iterate update through M^-1 at
    # every cycle end), and batches of 5 systems (the blocks inverted again for every batch)
    wl, P = disk
    om = np.linspace(0.2, 1.4, 7)
    d = np.array([[0.6, 0.8, 0.0]])
    tol = 1e-9
    h = lib.wfq_build(wl.xyz, wl.params, store=("fp64", "fp32", "bf16"))
    out = lib.wfq_solve(h, om, d, tol, restart=10, precision=prec, block_jacobi=True, max_batch=5)
    h.close()
    assert out["status"] == 0
    for a in range(len(om)):
        assert out["info"][a]["relres"] <= tol
        assert rel(out["q"][a, 0], P.solve_lu(om[a], d[0])) <= 1e-6, a


def test_block_jacobi_device_outputs_and_rejects(lib, tube):
    import torch
    xyz, P = tube
    om = np.array([0.5, 1.2])
    d = np.array([[0.0, 0.0, 1.0]])
    h = lib.wfq_build(xyz, GRAPHENE)
    host = lib.wfq_solve(h, om, d, 1e-10, restart=50, block_jacobi=True)
    n, S = h.n, len(om) * len(d)
    qr = torch.zeros(S * n, dtype=torch.float64, device="cuda:0")
    qi = torch.zeros(S * n, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.Stream("cuda:0")
    # the same kernels on the same inputs: bitwise the same charges, also when the inner steps are
    # captured as HIP graphs (the second solve of the shape replays what the first captured)
    for graphs in (False, True, True):
        qr.zero_()
        qi.zero_()
        dev = lib.wfq_solve_dev(h, om, d, 1e-10, q_re=qr, q_im=qi, stream=stream.cuda_stream, restart=50,
                                block_jacobi=True, graphs=graphs)
        torch.cuda.synchronize()
        assert dev["status"] == 0
        qd = (qr.cpu().numpy() + 1j * qi.cpu().numpy()).reshape(host["q"].shape)
        assert np.array_equal(qd, host["q"]), graphs
    for a in range(len(om)):
        assert rel(host["q"][a, 0], P.solve_lu(om[a], d[0])) <= 1e-6
    for bad in (dict(algorithm="qmr"), dict(algorithm="msgmres"), dict(warm_start=True)):
        with pytest.raises(lib.WfqError) as e:
            lib.wfq_solve(h, om, d, 1e-10, block_jacobi=True, **bad)
        assert e.value.code == lib.WFQ_EINVAL, bad
    h.close()
    hm = lib.wfq_build(xyz, GRAPHENE, t_mode="otf", store=())
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_solve(hm, om, d, 1e-10, block_jacobi=True)
    assert e.value.code == lib.WFQ_EINVAL
    hm.close()
