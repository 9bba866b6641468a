"""The oracle's pins, run against both oracle implementations: the Python one (numpy/scipy) and
the plain C++ one (oracle/wfq_oracle.cpp, OpenMP, its own LU, GMRES and QMR). Every check compares
an implementation with something the paper or the mathematics fixes (closed forms, limits,
invariants, independent algorithms), never one implementation with the other; the last test adds a
cross-check of the two on a larger structure. Also here: the pins of the cross sections (the
Thomas-Reiche-Kuhn sum rule) and of the material closure (the Froehlich frequency of a Drude sphere).
"""

import math

import numpy as np
import pytest

from oracle import wfq_oracle as O
from oracle.cpp_oracle import CppProblem
import wfq_inputs as wi
from wfq_inputs import geometry as geo

G = wi.workloads.GRAPHENE
FCC = wi.workloads.FCC_METAL
WG = O.material_weight(G)     # W of the graphene parameters (sum-rule closure)
WF = O.material_weight(FCC)


@pytest.fixture(params=["python", "cpp"])
def make(request):
    def f(xyz, params=G, dense_T=True, species=None):
        if request.param == "python":
            return O.Problem(xyz, params, dense_T=dense_T, species=species)
        return CppProblem(xyz, params, dense_T=dense_T, species=species)
    f.kind = request.param
    return f


def t_matrix(P):
    """The whole T of an implementation (from its stored matrix or its element function)."""
    if isinstance(P, O.Problem):
        return P.T
    i, j = np.meshgrid(np.arange(P.n), np.arange(P.n), indexing="ij")
    return P.sample_T(i.ravel(), j.ravel()).reshape(P.n, P.n)


def alpha(P, Q):
    return O.polarisability(P.xyz, Q) if isinstance(P, O.Problem) else P.polarisability(Q)


def disk(seed=7, radius=9.0):
    return geo.jitter(geo.graphene_disk(radius), 0.02, seed)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ----------------------------------------------------------------- elements

def test_t_limits_symmetry_and_cholesky(make):
    # far field: erf -> 1, T_ij = 1/r; contact: T_ii = eta; SPD (Cholesky succeeds)
    xyz = np.array([[0.0, 0.0, 0.0], [40.0, 0.0, 0.0], [0.3, 0.0, 0.0], [1.42, 0.0, 0.0]])
    P = make(xyz)
    T = t_matrix(P)
    r = 40.0 / O.BOHR_A
    assert T[0, 1] == pytest.approx(1.0 / r, rel=1e-14)
    assert T[0, 0] == pytest.approx(G["eta"], rel=1e-15)
    # short distance: erf(x)/r -> 2/sqrt(pi) / w (1 - x^2/3 + x^4/10) / ... with x = r / w
    d = math.sqrt(2 / math.pi) / G["eta"]
    w = math.sqrt(2) * d
    rs = 0.3 / O.BOHR_A
    x = rs / w
    # Maclaurin series of erf: sum_k (-1)^k x^(2k+1) / (k! (2k+1))
    series = 2 / math.sqrt(math.pi) / w * sum((-1) ** k * x ** (2 * k) / (math.factorial(k) * (2 * k + 1)) for k in range(10))
    assert T[0, 2] == pytest.approx(series, rel=1e-9)
    Tb = t_matrix(make(disk(radius=7.0)))
    assert np.array_equal(Tb, Tb.T)
    np.linalg.cholesky(Tb)


def test_fermi_midpoint_through_l(make):
    # a dimer at r = s r0: 1 - f = 1/2 exactly, so L_12 = -1/(2 r) and L_11 = 1/(2 r)
    r_A = G["fermi_s"] * G["r0"]
    P = make(np.array([[0.0, 0.0, 0.0], [r_A, 0.0, 0.0]]))
    L = P.L.toarray()
    r = r_A / O.BOHR_A
    assert L[0, 1] == pytest.approx(-0.5 / r, rel=1e-14)
    assert L[0, 0] == pytest.approx(0.5 / r, rel=1e-14)


def test_laplacian_structure_and_neighbour_count(make):
    P = make(disk(radius=12.0))
    L = P.L.toarray()
    assert np.array_equal(L, L.T)
    assert np.max(np.abs(L.sum(axis=1))) < 1e-14 * np.max(np.abs(L))
    off = L - np.diag(np.diag(L))
    assert np.all(off <= 0)
    ev = np.linalg.eigvalsh(L)
    assert ev.min() > -1e-12 * ev.max() and np.sum(np.abs(ev) < 1e-10 * ev.max()) == 1
    # the ideal honeycomb has 36 neighbours inside r_c = 5.16 Angstrom: the central atom of an ideal disk
    Pi = make(geo.graphene_disk(12.0))
    c = np.argmin(np.sum(geo.graphene_disk(12.0) ** 2, axis=1))
    assert Pi.L[c].nnz == 37


def test_two_species_dimer_closed_form(make):
    # atoms of two species: T_ii = eta_i, T_01 = erf(r / sqrt(d_0^2 + d_1^2)) / r with d_i = sqrt(2/pi) / eta_i,
    # Kbar_01 from the pair r0 (r0_0 + r0_1) / 2. The dimer's charges are c (1, -1), so
    # alpha_xx = Kbar r^2 / (Kbar (eta_0 + eta_1 - 2 T_01) + z).
    eta0, eta1, r0a, r0b = 0.45, 0.8, 1.42, 1.63
    par = dict(G, species=[(eta0, r0a), (eta1, r0b)])
    r_A = 1.7
    P = make(np.array([[0.0, 0.0, 0.0], [r_A, 0.0, 0.0]]), par, species=[0, 1])
    r = r_A / O.BOHR_A
    r0 = 0.5 * (r0a + r0b) / O.BOHR_A
    k = (1.0 - 1.0 / (1.0 + math.exp(-12.0 * (r / (1.1 * r0) - 1.0)))) / r
    d0, d1 = math.sqrt(2 / math.pi) / eta0, math.sqrt(2 / math.pi) / eta1
    t = math.erf(r / math.sqrt(d0 * d0 + d1 * d1)) / r
    T = t_matrix(P)
    assert T[0, 0] == eta0 and T[1, 1] == eta1
    assert T[0, 1] == pytest.approx(t, rel=1e-15) and T[1, 0] == T[0, 1]
    assert P.L.toarray()[0, 1] == pytest.approx(-k, rel=1e-14)
    for om in (0.1, 0.7, 3.0):
        oh = om / 27.211386245988
        z = -(oh * oh + 1j * oh / 170.0) / WG
        q = P.solve_lu(om, [1, 0, 0])
        a = alpha(P, q[:, None])
        assert a[0, 0] == pytest.approx(k * r * r / (k * (eta0 + eta1 - 2 * t) + z), rel=1e-13)


def test_pair_cutoff_follows_the_pair_r0(make):
    # r_c = s r0 (1 + ln(1/eps - 1) / d) is 5.16 Angstrom for r0 = 1.42 and 5.48 for the mixed pair of
    # r0 = 1.42 and 1.60: a dimer at 5.3 Angstrom is coupled only when one atom is of the wider species
    eps = G["cutoff_eps"]
    par = dict(G, species=[(G["eta"], 1.42), (G["eta"], 1.60)])
    rc = [O.cutoff_radius(r0, 12.0, 1.1, eps) for r0 in (1.42, 1.51)]
    assert rc[0] < 5.3 < rc[1]
    xyz = np.array([[0.0, 0.0, 0.0], [5.3, 0.0, 0.0]])
    assert not np.any(make(xyz, par, species=[0, 0]).L.toarray())
    L = make(xyz, par, species=[0, 1]).L.toarray()
    r = 5.3 / O.BOHR_A
    k = (1.0 - 1.0 / (1.0 + math.exp(-12.0 * (r / (1.1 * 1.51 / O.BOHR_A) - 1.0)))) / r
    assert L[0, 1] == pytest.approx(-k, rel=1e-13) and 0 < k * r < eps * 1e3


def test_one_species_table_equals_the_scalar_parameters(make):
    xyz = disk(radius=8.0)
    a = make(xyz)
    b = make(xyz, dict(G, species=[(G["eta"], G["r0"]), (2 * G["eta"], 2 * G["r0"])]),
             species=np.zeros(len(xyz), dtype=np.int32))
    assert np.array_equal(a.L.toarray(), b.L.toarray())
    assert np.array_equal(t_matrix(a), t_matrix(b))


# ----------------------------------------------------------------- solutions

def test_dimer_closed_form(make):
    r_A = 1.7
    P = make(np.array([[0.0, 0.0, 0.0], [r_A, 0.0, 0.0]]))
    r = r_A / O.BOHR_A
    k = (1.0 - 1.0 / (1.0 + math.exp(-12.0 * (r / (1.1 * G["r0"] / O.BOHR_A) - 1.0)))) / r
    d = math.sqrt(2 / math.pi) / G["eta"]
    t = math.erf(r / math.sqrt(2 * d * d)) / r
    for om in (0.1, 0.7, 3.0):
        oh = om / 27.211386245988
        z = -(oh * oh + 1j * oh / 170.0) / WG
        q = P.solve_lu(om, [1, 0, 0])
        a = alpha(P, q[:, None])
        assert a[0, 0] == pytest.approx(k * r * r / (k * (2 * G["eta"] - 2 * t) + z), rel=1e-13)
        assert abs(q[0] + q[1]) < 1e-14 * abs(q[0])


def test_lu_matches_modal_form_static_and_high_frequency_limits(make):
    P = make(disk(radius=10.0))
    L, T, R = P.L, t_matrix(P), P.xyz
    for om in (0.2, 0.9):
        Qm = O.solve_modal(L, T, P.z(om), R)
        for k in range(3):
            assert rel(P.solve_lu(om, np.eye(3)[k]), Qm[:, k]) <= 1e-10
    a0 = O.static_polarisability(T, R)
    a = alpha(P, np.column_stack([P.solve_lu(1e-6, e) for e in np.eye(3)]))
    assert np.allclose(a[:2, :2], a0[:2, :2], rtol=1e-6, atol=1e-8 * np.max(np.abs(a0)))
    Ld = L.toarray()
    om = 400.0
    z = P.z(om)
    a = alpha(P, np.column_stack([P.solve_lu(om, e) for e in np.eye(3)]))
    a1 = R.T @ Ld @ R / z
    a2 = a1 - R.T @ Ld @ T @ Ld @ R / z ** 2
    assert np.abs(a - a2)[:2, :2].max() < 1e-2 * np.abs(a - a1)[:2, :2].max()


def test_conservation_reciprocity_passivity_covariance(make):
    xyz = disk(radius=10.0)
    P = make(xyz)
    for om in (0.15, 1.4):
        Q = np.column_stack([P.solve_lu(om, e) for e in np.eye(3)])
        assert np.max(np.abs(Q.sum(axis=0))) < 1e-12 * np.max(np.linalg.norm(Q, axis=0))
        a = alpha(P, Q)
        assert abs(a[0, 1] - a[1, 0]) <= 1e-10 * abs(a[0, 0])
        assert a[0, 0].imag > 0 and a[1, 1].imag > 0
    om = 0.4
    a = alpha(P, np.column_stack([P.solve_lu(om, e) for e in np.eye(3)]))
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Pr = make(xyz @ Rz.T + np.array([3.0, -7.0, 11.0]))
    ar = alpha(Pr, np.column_stack([Pr.solve_lu(om, e) for e in np.eye(3)]))
    # rotation covariance; the translation leaves alpha unchanged because sum q = 0
    assert np.allclose(ar, Rz @ a @ Rz.T, rtol=1e-9, atol=1e-9 * np.abs(a).max())


# ----------------------------------------------------------------- iterative solvers

def test_gmres_full_space_and_restarted(make):
    P = make(disk(radius=8.0))
    for om in (0.3, 1.1):
        q = P.solve_lu(om, [1, 0, 0])
        x, info = P.solve_gmres(om, [1, 0, 0], restart=P.n, tol=1e-13)
        assert info["cycles"] == 1
        assert rel(x, q) <= 1e-9
    P = make(disk(radius=10.0))
    q = P.solve_lu(0.8, [0, 1, 0])
    x, info = P.solve_gmres(0.8, [0, 1, 0], restart=10, tol=1e-10)
    assert info["cycles"] > 1 and info["relres"] <= 1e-10
    assert rel(x, q) <= 1e-7
    assert P.residual(0.8, [0, 1, 0], x) == pytest.approx(info["relres"], rel=1e-6)


def test_qmr_matches_lu(make):
    P = make(disk(radius=10.0))
    for om, d in ((0.3, [1, 0, 0]), (1.2, [0, 1, 0])):
        q = P.solve_lu(om, d)
        x, info = P.solve_qmr(om, d, tol=1e-11)
        assert not info["breakdown"]
        assert P.residual(om, d, x) <= 1e-10
        assert rel(x, q) <= 1e-8


def test_residual_rows_and_matrix_free_products(make):
    xyz = disk(radius=10.0)
    P = make(xyz)
    q = P.solve_lu(0.5, [1, 0, 0]) * (1 + 1e-6)
    r_full = P.rhs([1, 0, 0]) - P.apply(P.z(0.5))(q)
    rows = np.array([0, 3, 17, P.n - 1])
    assert np.allclose(P.residual_rows(0.5, [1, 0, 0], q, rows), r_full[rows], rtol=1e-10, atol=1e-14)
    Pf = make(xyz, dense_T=False)
    x = np.random.default_rng(2).standard_normal((P.n, 2)) @ np.array([1.0, 1j])
    assert np.allclose(Pf.apply_T(x), t_matrix(P) @ x, rtol=1e-13, atol=0)
    if hasattr(Pf, "apply_T_rows"):   # the C++ oracle's sampled rows of the matrix-free product
        X = np.random.default_rng(4).standard_normal((P.n, 3))
        assert np.allclose(Pf.apply_T_rows(rows, X), (t_matrix(P) @ X)[rows], rtol=1e-13, atol=0)


def test_complex_t_product_applies_the_real_matrix_to_each_part(make):
    # T is real: T x for complex x is T Re x + i T Im x, computed without a complex copy of T
    P = make(disk(radius=8.0))
    rng = np.random.default_rng(3)
    x = rng.standard_normal(P.n) + 1j * rng.standard_normal(P.n)
    T = t_matrix(P)
    y = P.apply_T(x)
    assert np.allclose(y.real, T @ x.real, rtol=1e-13, atol=0) and np.allclose(y.imag, T @ x.imag, rtol=1e-13, atol=0)


# ----------------------------------------------------------------- observables

def lorentz_dimer(P, r_A, om_eV):
    """alpha_xx of the dimer at r_A (closed form of test_dimer_closed_form) as an array over om_eV."""
    r = r_A / O.BOHR_A
    k = (1.0 - 1.0 / (1.0 + math.exp(-12.0 * (r / (1.1 * G["r0"] / O.BOHR_A) - 1.0)))) / r
    d = math.sqrt(2 / math.pi) / G["eta"]
    t = math.erf(r / math.sqrt(2 * d * d)) / r
    oh = np.asarray(om_eV) / 27.211386245988
    z = -(oh * oh + 1j * oh / G["tau"]) / WG
    return k * r * r / (k * (2 * G["eta"] - 2 * t) + z), k * r * r


def test_cross_section_obeys_the_trk_sum_rule():
    # The dimer is a Lorentz oscillator alpha = F / (w0^2 - w^2 - i w / tau) with F = W Kbar r^2. For any
    # such response the integral of sigma = (4 pi w / c) Im alpha over w in (0, inf) is 2 pi^2 F / c
    # (Thomas-Reiche-Kuhn), whatever w0 and tau. A wrong prefactor, omega in eV instead of Hartree or
    # the real part in place of the imaginary one all change the integral.
    om_eV = np.linspace(1e-4, 400.0, 4_000_001)
    a, krr = lorentz_dimer(None, 1.7, om_eV)
    sig = O.cross_section(O.ev_to_hartree(om_eV), a)
    integral = np.trapezoid(sig, O.ev_to_hartree(om_eV))
    tail = 2 * math.pi * WG * krr / (O.C_AU * O.ev_to_hartree(400.0) * G["tau"])   # (4 pi / c) F gamma / w_max
    assert integral + tail == pytest.approx(2 * math.pi ** 2 * WG * krr / O.C_AU, rel=2e-4)
    assert np.all(sig > 0)


def test_isotropic_cross_section_sum_rule_and_rotation_invariance():
    # sigma = (1/3) sum_k sigma_k (Eq. iso-cross): it is invariant under rotations of the structure
    # (the trace of alpha), and its TRK integral is (2 pi^2 / c) W tr(R^T L R) / 3 (the f-sum of every
    # direction, from the high-frequency term R^T L R / z of the response).
    xyz = geo.jitter(geo.nanotube(3, 3, 3), 0.02, 5)
    P = O.Problem(xyz, G)
    lam, U, th, tih = O.modal_decomposition(P.L, P.T)
    A = U.T @ (tih @ P.xyz)
    om_eV = np.concatenate([np.linspace(1e-4, 40.0, 400_001), np.linspace(40.0, 4000.0, 100_001)[1:]])
    oh = O.ev_to_hartree(om_eV)
    z = -(oh * oh + 1j * oh / G["tau"]) / WG
    # alpha(omega) from the modal form, all three diagonal entries at every frequency
    frac = lam[None, :] / (lam[None, :] + z[:, None])
    diag = np.stack([frac @ (A[:, k] ** 2) for k in range(3)])
    alpha_w = np.zeros((3, 3, len(om_eV)), dtype=complex)
    for k in range(3):
        alpha_w[k, k] = diag[k]
    sig = O.isotropic_cross_section(oh, alpha_w)
    Ld = P.L.toarray()
    trk = 2 * math.pi ** 2 * WG * np.trace(P.xyz.T @ Ld @ P.xyz) / 3 / O.C_AU
    assert np.trapezoid(sig, oh) == pytest.approx(trk, rel=2e-3)
    th_ = 0.9
    Rx = np.array([[1, 0, 0], [0, math.cos(th_), -math.sin(th_)], [0, math.sin(th_), math.cos(th_)]])
    a = O.polarisability(P.xyz, np.column_stack([P.solve_lu(1.3, e) for e in np.eye(3)]))
    Pr = O.Problem(xyz @ Rx.T, G)
    ar = O.polarisability(Pr.xyz, np.column_stack([Pr.solve_lu(1.3, e) for e in np.eye(3)]))
    w = O.ev_to_hartree(1.3)
    assert O.isotropic_cross_section(w, ar) == pytest.approx(O.isotropic_cross_section(w, a), rel=1e-9)
    assert O.isotropic_cross_section(w, a) == pytest.approx(np.mean([O.cross_section(w, a[k, k]) for k in range(3)]), rel=1e-14)
    # the individual sigma_k do change under the rotation (about x: y and z mix)
    assert abs(O.cross_section(w, ar[1, 1]) - O.cross_section(w, a[1, 1])) > 1e-3 * abs(O.cross_section(w, a[1, 1]))


def test_metal_closure_gives_the_froehlich_frequency():
    # With W from the sum-rule closure (n_e = 4 / a^3, m* = 1), the brightest dipole mode of an ideal
    # FCC sphere approaches the classical surface plasmon of a Drude sphere, w_p / sqrt(3) with
    # w_p^2 = 4 pi n_e / m* (5.18 eV), from below as the sphere grows.
    a = geo.A_FCC / O.BOHR_A
    w_frohlich = math.sqrt(4 * math.pi * 4 / a ** 3 / 3) * O.HARTREE_EV
    prev = 0.0
    for R in (12.0, 16.0):
        P = O.Problem(geo.fcc_sphere(R), FCC)
        lam, U, th, tih = O.modal_decomposition(P.L, P.T)
        wgt = lam * (U.T @ (tih @ P.xyz[:, 0])) ** 2
        om = np.sqrt(np.maximum(lam, 0) * WF) * O.HARTREE_EV
        peak = om[np.argmax(wgt)]
        assert prev < peak < w_frohlich
        prev = peak
    assert prev == pytest.approx(w_frohlich, rel=0.05)


# ----------------------------------------------------------------- the two implementations

def test_cpp_and_python_oracles_agree_on_a_tube():
    xyz = geo.jitter(geo.nanotube(5, 5, 30), 0.01, 9)
    P, Q = O.Problem(xyz, G), CppProblem(xyz, G)
    assert abs(P.L - Q.L).max() <= 1e-15 * abs(P.L).max()
    for om, d in ((0.2, [0, 0, 1]), (0.9, [1, 0, 0])):
        qp = P.solve_lu(om, d)
        qc = Q.solve_lu(om, d)
        assert rel(qc, qp) <= 1e-10
        x, info = Q.solve_gmres(om, d, 40, 1e-10)
        assert info["relres"] <= 1e-10 and rel(x, qp) <= 1e-8


def test_cpp_qmr_takes_the_steps_of_the_pinned_recurrence():
    # The Python QMR is pinned step by step (its smoothing of CG is MINRES, test_oracle.py); the C++
    # QMR runs the same recurrences in its own code, so it must stop at the same step with the same
    # smoothed residual (a wrong smoothing weight or a conjugated bilinear form changes both).
    xyz = geo.jitter(geo.graphene_disk(10.0), 0.02, 7)
    P, Q = O.Problem(xyz, G), CppProblem(xyz, G)
    for om, d in ((0.3, [1, 0, 0]), (1.2, [0, 1, 0])):
        xp, ip = P.solve_qmr(om, d, tol=1e-9)
        xc, ic = Q.solve_qmr(om, d, tol=1e-9)
        assert ic["iters"] == ip["iters"]
        assert ic["relres"] == pytest.approx(ip["relres"], rel=5e-2)   # rounding differs between the two
        assert rel(xc, xp) <= 1e-10
