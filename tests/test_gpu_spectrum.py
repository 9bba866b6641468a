"""Spectrum scans (the cross-section over a 200-point frequency grid) against the oracle's LU-free
modal closed form (needs an MI355X).

The multi-shift solve of the disk over 0.01..2.00 eV must reproduce sigma_k(omega) of Eq. (long-cross)
computed from the eigendecomposition of T^(1/2) L T^(1/2) at every frequency, keep sigma >= 0
(passivity) and place the resonance peaks where the closed form has them.
"""

import numpy as np
import pytest

from oracle import wfq_oracle as O
import wfq_inputs as wi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


def modal_sigma(P, om, k):
    lam, U, th, tih = O.modal_decomposition(P.L, P.T)
    R = P.xyz[:, k:k + 1]
    a = U.T @ (tih @ R)
    out = []
    for w in om:
        q = tih @ (U @ ((lam / (lam + P.z(w)))[:, None] * a))
        out.append(O.cross_section(O.ev_to_hartree(w), R[:, 0] @ q[:, 0]))
    return np.array(out)


def peaks(s):
    return [i for i in range(1, len(s) - 1) if s[i] > s[i - 1] and s[i] > s[i + 1] and s[i] > 0.05 * s.max()]


def test_disk_spectrum_matches_modal_form(lib):
    wl = wi.workload("disk600_spectrum")
    P = O.Problem(wl.xyz, wl.params)
    h = lib.wfq_build(wl.xyz, wl.params)
    out = lib.wfq_solve(h, wl.omegas_eV, wl.dirs, wl.tol, want_q=False, algorithm="msgmres",
                        restart=wl.restart, precision="fp64")
    h.close()
    assert out["status"] == 0
    assert max(r["relres"] for r in out["info"]) <= wl.tol
    for k in range(2):                                   # the two in-plane directions
        sig_gpu = np.array([O.cross_section(O.ev_to_hartree(w), out["alpha"][a, k, k])
                            for a, w in enumerate(wl.omegas_eV)])
        sig_ref = modal_sigma(P, wl.omegas_eV, k)
        assert np.all(sig_gpu >= 0)
        assert np.max(np.abs(sig_gpu - sig_ref)) <= 1e-6 * sig_ref.max()
        assert peaks(sig_gpu) == peaks(sig_ref)
