"""The error bound err_est against measured errors (needs an MI355X).

err_est bounds |q - q*|_T / |q*|_T in the Coulomb norm |v|_T = sqrt(v^H T v). Checked against the
LU solution of the oracle at loose and tight tolerances, for every algorithm and with FP32 inner
products, off and on a plasmon resonance, on the 600-atom disk and a ragged tube; the 2-norm error
must then lie within sqrt(kappa_2(T)) err_est.
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


def resonance(P, lo, hi, n=40):
    """Frequency (eV) of the largest Im alpha_xx on a grid, by LU solves of the oracle."""
    om = np.linspace(lo, hi, n)
    im = [np.imag(O.polarisability(P.xyz, P.solve_lu(w, [1, 0, 0])[:, None])[0, 0]) for w in om]
    return float(om[int(np.argmax(im))])


@pytest.fixture(scope="module")
def cases():
    disk = wi.workload("disk600")
    tube = ragged_tube(periods=30)
    out = {}
    for name, xyz, par, grid in (("disk600", disk.xyz, disk.params, (0.1, 1.5)),
                                 ("tube", tube, GRAPHENE, (0.05, 1.2))):
        P = O.Problem(xyz, par)
        om = np.array(sorted({0.05, 0.4, 1.0, resonance(P, *grid)}))
        dirs = np.eye(3)[:2]
        ref = {(a, k): P.solve_lu(om[a], dirs[k]) for a in range(len(om)) for k in range(len(dirs))}
        ev = np.linalg.eigvalsh(P.T)
        out[name] = (xyz, par, P, om, dirs, ref, np.sqrt(ev[-1] / ev[0]))
    return out


def tnorm(P, v):
    return np.sqrt(np.real(np.vdot(v, P.T @ v)))


@pytest.mark.parametrize("name", ["disk600", "tube"])
@pytest.mark.parametrize("algorithm,prec", [("gmres", "fp64"), ("gmres", "fp32"), ("msgmres", "fp64"),
                                            ("qmr", "fp64")])
@pytest.mark.parametrize("tol", [1e-4, 1e-8])
def test_error_bound_holds(lib, cases, name, algorithm, prec, tol):
    xyz, par, P, om, dirs, ref, sqrt_kt = cases[name]
    h = lib.wfq_build(xyz, par)
    out = lib.wfq_solve(h, om, dirs, tol, algorithm=algorithm, restart=40, precision=prec)
    h.close()
    assert out["status"] == 0, out["info"]
    ratios = []
    for a in range(len(om)):
        for k in range(len(dirs)):
            info = out["info"][a * len(dirs) + k]
            q, qs = out["q"][a, k], ref[(a, k)]
            err_t = tnorm(P, q - qs) / tnorm(P, qs)
            err_2 = np.linalg.norm(q - qs) / np.linalg.norm(qs)
            est = info["err_est"]
            assert 0 < est < 1
            assert err_t <= est, (om[a], k, err_t, est, info["relres"])
            assert err_2 <= sqrt_kt * est, (om[a], k, err_2, est)
            ratios.append(err_t / est)
    # the bound is not vacuous: within three orders of magnitude of the error for some system
    assert max(ratios) >= 1e-3, ratios
    print(f"{name} {algorithm} {prec} tol {tol:g}: error / bound in [{min(ratios):.2g}, {max(ratios):.2g}]")


def test_error_bound_of_an_exact_start(lib, cases):
    # b = 0 (a field along z on a flat disk has no in-plane potential difference): q = 0 is exact
    xyz, par, P, om, dirs, ref, _ = cases["disk600"]
    flat = xyz.copy()
    flat[:, 2] = 0.0
    h = lib.wfq_build(flat, par)
    out = lib.wfq_solve(h, om[:1], np.array([[0.0, 0.0, 1.0]]), 1e-8, algorithm="gmres", restart=40)
    h.close()
    assert out["info"][0]["relres"] == 0.0 and out["info"][0]["err_est"] == 0.0
