"""The allocation-free operator entry point wfq_apply_op_noalloc (device buffers, static scratch)
against the existing entry point wfq_apply_op on the same inputs, and both against the oracle's
operator with the same element-wise bound as the operator test (needs an MI355X). Two calls in a row
share the scratch; the second has a smaller input, so anything the first left behind would show."""

import numpy as np
import pytest

from oracle import wfq_oracle as O
from helpers import GRAPHENE, UNIT, ragged_tube, round_to
from wfq_inputs import geometry as geo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


def run_noalloc(lib, torch, h, prec, z, X):
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    zr, zi, xr, xi = t(z.real), t(z.imag), t(X.real), t(X.imag)
    yr = torch.full_like(xr, float("nan"))
    yi = torch.full_like(xi, float("nan"))
    stream = torch.cuda.Stream(dev)
    torch.cuda.synchronize()
    lib.wfq_apply_op_noalloc(h, prec, zr, zi, xr, xi, yr, yi, stream=stream.cuda_stream)
    stream.synchronize()
    return yr.cpu().numpy() + 1j * yi.cpu().numpy()


def oracle_bound_ok(P, prec, z, X, Y):
    L = P.L
    for s in range(X.shape[0]):
        if prec == "fp64":
            ref = L @ (P.T @ X[s]) + z[s] * X[s]
            scale = np.abs(L) @ (np.abs(P.T) @ np.abs(X[s])) + np.abs(z[s] * X[s])
            if not np.all(np.abs(Y[s] - ref) <= 1e-12 * scale):
                return False
        else:
            Tq = round_to(prec, P.T)
            xr, xi = round_to(prec, X[s].real), round_to(prec, X[s].imag)
            ref = L @ (Tq @ xr + 1j * (Tq @ xi)) + z[s] * X[s]
            scale = np.abs(L) @ (np.abs(Tq) @ (np.abs(xr) + np.abs(xi))) + np.abs(z[s] * X[s])
            if not np.all(np.abs(Y[s] - ref) <= 2 * P.n * UNIT["fp32"] * scale):
                return False
    return True


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_noalloc_matches_apply_op_on_two_calls(lib, prec):
    import torch
    cases = [(ragged_tube(), 7, 11), (geo.jitter(geo.graphene_disk(9.0), 0.01, 12), 2, 13)]   # second is smaller
    for xyz, nsys, seed in cases:
        P = O.Problem(xyz, GRAPHENE)
        h = lib.wfq_build(xyz, GRAPHENE, store=("fp64", "fp32", "bf16"))
        rng = np.random.default_rng(seed)
        X = rng.standard_normal((nsys, P.n)) + 1j * rng.standard_normal((nsys, P.n))
        z = np.array([P.z(om) for om in np.linspace(0.05, 1.0, nsys)])
        y_ref = lib.wfq_apply_op(h, prec, z, X)
        y = run_noalloc(lib, torch, h, prec, z, X)
        assert np.all(np.isfinite(y))
        # the same kernels; only the split of the block product's k range may differ
        tol = {"fp64": 1e-13, "fp32": 1e-5, "bf16": 1e-5}[prec]
        assert np.linalg.norm(y - y_ref) <= tol * np.linalg.norm(y_ref)
        assert oracle_bound_ok(P, prec, z, X, y)
        h.close()


def test_noalloc_rejects_what_does_not_fit(lib):
    import torch
    xyz = ragged_tube()
    h = lib.wfq_build(xyz, GRAPHENE)
    n = len(xyz)
    cap = lib.wfq_noalloc_scratch_bytes()
    assert cap == 256 << 20
    nsys = cap // (16 * 1280) + 1          # the systems' vectors alone exceed the scratch
    dev = torch.device("cuda:0")
    z = torch.zeros(nsys, dtype=torch.float64, device=dev)
    X = torch.zeros((nsys, n), dtype=torch.float64, device=dev)
    Y = torch.zeros_like(X)
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_apply_op_noalloc(h, "fp64", z, z, X, X, Y, Y)
    assert e.value.code == lib.WFQ_ENOMEM
    with pytest.raises(lib.WfqError) as e:
        lib.wfq_apply_op_noalloc(h, "bf16", z[:1], z[:1], X[:1], X[:1], Y[:1], Y[:1])   # no BF16 copy built
    assert e.value.code == lib.WFQ_EINVAL
    h.close()
