// Plain CPU FP64 oracle of the omegaFQ linear-response problem, C++17 + OpenMP.
//
// TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's CPU-baseline leg
// load it (through oracle/cpp_oracle.py); the device library never does. It shares no code with the
// device library and is written from the definitions of Lafiosca, Giovannini, Benzi and Cappelli,
// "Fully Atomistic Modeling of Realistic Plasmonic Materials: Assessing the Performance of Iterative
// Solvers" (arXiv 2103.00438), with the same readings of the paper as the Python oracle
// (oracle/wfq_oracle.py):
//   * Eq. (wfq-original): the "+ i omega" term is the diagonal shift i omega delta_ij;
//   * width-from-hardness equation: d_i = sqrt(2/pi) / eta_i;
//   * Eq. (k-tot-matrix) with a constant effective area folded into W = 2 n0 A, so that
//     Kbar_ij = (1 - f(r_ij)) / r_ij and z(omega) = -(omega^2 + i omega / tau) / W (Eq. z-def);
//   * Kbar truncated where 1 - f < eps_c, i.e. beyond r_c = s r0 (1 + ln(1/eps_c - 1) / d);
//   * a pair of atoms of two species uses r0_ij = (r0_i + r0_j) / 2 in f and in r_c;
//   * the sign-flipped system (L T + z I) q = b, L = P - Kbar (Eq. a-matrix-product and the
//     definition of P), b = E0 L (r . k) (Eqs. potential, r-vector-def), T = D (Eq. d-matrix).
// Everything is double / std::complex<double> in Hartree atomic units; positions come in Angstrom
// and frequencies in eV.
//
// What is here: T elements and products (stored dense or recomputed per row), L by an all-pairs
// neighbour search, the right-hand side, the operator, dense complex LU with partial pivoting,
// restarted GMRES(m) with modified Gram-Schmidt and Givens rotations (Saad & Schultz), J-symmetric
// QMR from BCG without look-ahead (J = T, QMR smoothing of Zhou & Walker), the FP64 residual (whole
// or row by row from pairwise elements) and the polarisability alpha_lk = sum_i r_il q_i / E0.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

constexpr double kBohrA = 0.529177210903;      // Angstrom per bohr (CODATA 2018)
constexpr double kHartreeEV = 27.211386245988;  // eV per Hartree (CODATA 2018)
constexpr double kPi = 3.14159265358979323846;

struct Problem {
    int64_t n = 0;
    std::vector<double> pos;   // [n][3], bohr
    std::vector<double> eta;   // hardness
    std::vector<double> wid;   // Gaussian width d_i
    std::vector<double> r0;    // per-atom r0 (bohr); a pair takes the mean of its two atoms' values
    double fd = 0, fs = 0, cfac = 0, W = 0, tau = 0;
    bool have_L = false;
    std::vector<int64_t> rp;   // CSR of L = P - Kbar (diagonal entry first in each row)
    std::vector<int64_t> ci;
    std::vector<double> lv;
    std::vector<double> T;     // dense row-major n x n, or empty (rows recomputed)

    double dist(int64_t i, int64_t j) const {
        const double dx = pos[3 * i] - pos[3 * j], dy = pos[3 * i + 1] - pos[3 * j + 1],
                     dz = pos[3 * i + 2] - pos[3 * j + 2];
        return std::sqrt(dx * dx + dy * dy + dz * dz);
    }
    // Eq. (d-matrix): erf(r_ij / sqrt(d_i^2 + d_j^2)) / r_ij, eta_i on the diagonal
    double t_elem(int64_t i, int64_t j) const {
        if (i == j) return eta[i];
        const double r = dist(i, j);
        return std::erf(r / std::sqrt(wid[i] * wid[i] + wid[j] * wid[j])) / r;
    }
    // Eq. (fermi) and Eq. (k-tot-factor) with unit area: (1 - f(r)) / r, zero beyond r_c of the pair
    double kbar(int64_t i, int64_t j) const {
        const double r = dist(i, j), r0ij = 0.5 * (r0[i] + r0[j]);
        if (!(r < fs * r0ij * cfac) || r == 0.0) return 0.0;
        const double f = 1.0 / (1.0 + std::exp(-fd * (r / (fs * r0ij) - 1.0)));
        return (1.0 - f) / r;
    }
    // one row of L: the diagonal P_ii = sum_k Kbar_ik first, then -Kbar_ij for the neighbours j
    void l_row(int64_t i, std::vector<int64_t>& cols, std::vector<double>& vals) const {
        cols.clear();
        vals.clear();
        cols.push_back(i);
        vals.push_back(0.0);
        double diag = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double k = kbar(i, j);
            if (k != 0.0) {
                cols.push_back(j);
                vals.push_back(-k);
                diag += k;
            }
        }
        vals[0] = diag;
    }
    // y = T x for one real vector (or two at once), stored or recomputed rows
    void apply_T2(const double* xa, const double* xb, double* ya, double* yb) const {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double sa = 0.0, sb = 0.0;
            if (!T.empty()) {
                const double* row = T.data() + i * n;
                for (int64_t j = 0; j < n; ++j) {
                    sa += row[j] * xa[j];
                    if (xb) sb += row[j] * xb[j];
                }
            } else {
                for (int64_t j = 0; j < n; ++j) {
                    const double t = t_elem(i, j);
                    sa += t * xa[j];
                    if (xb) sb += t * xb[j];
                }
            }
            ya[i] = sa;
            if (yb) yb[i] = sb;
        }
    }
    void apply_L(const std::vector<double>& x, std::vector<double>& y) const {
        y.assign(n, 0.0);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += lv[p] * x[ci[p]];
            y[i] = s;
        }
    }
    // y = (L T + z I) x for complex x: T acts on the real and imaginary parts separately
    void apply_op(cplx z, const std::vector<cplx>& x, std::vector<cplx>& y) const {
        std::vector<double> xr(n), xi(n), tr(n), ti(n), lr, li;
        for (int64_t i = 0; i < n; ++i) {
            xr[i] = x[i].real();
            xi[i] = x[i].imag();
        }
        apply_T2(xr.data(), xi.data(), tr.data(), ti.data());
        apply_L(tr, lr);
        apply_L(ti, li);
        y.resize(n);
        for (int64_t i = 0; i < n; ++i) y[i] = cplx(lr[i], li[i]) + z * x[i];
    }
    // the operator with T in place of L T (the J of the J-symmetric QMR): y = T x, complex x
    void apply_Tc(const std::vector<cplx>& x, std::vector<cplx>& y) const {
        std::vector<double> xr(n), xi(n), tr(n), ti(n);
        for (int64_t i = 0; i < n; ++i) {
            xr[i] = x[i].real();
            xi[i] = x[i].imag();
        }
        apply_T2(xr.data(), xi.data(), tr.data(), ti.data());
        y.resize(n);
        for (int64_t i = 0; i < n; ++i) y[i] = cplx(tr[i], ti[i]);
    }
    void apply_Lc(const std::vector<cplx>& x, std::vector<cplx>& y) const {
        y.assign(n, cplx(0.0, 0.0));
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            cplx s(0.0, 0.0);
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += lv[p] * x[ci[p]];
            y[i] = s;
        }
    }
    cplx shift(double omega_eV) const {
        const double om = omega_eV / kHartreeEV;
        return cplx(-om * om / W, -om / tau / W);
    }
    void rhs(const double* dir, double E0, std::vector<cplx>& b) const {
        std::vector<double> k(n), lk;
        for (int64_t i = 0; i < n; ++i) k[i] = pos[3 * i] * dir[0] + pos[3 * i + 1] * dir[1] + pos[3 * i + 2] * dir[2];
        apply_L(k, lk);
        b.resize(n);
        for (int64_t i = 0; i < n; ++i) b[i] = E0 * lk[i];
    }
};

double norm2(const std::vector<cplx>& v) {
    double s = 0.0;
    for (const cplx& a : v) s += std::norm(a);
    return std::sqrt(s);
}

// <a, b> = sum conj(a_i) b_i
cplx dotc(const std::vector<cplx>& a, const std::vector<cplx>& b) {
    cplx s(0.0, 0.0);
    for (size_t i = 0; i < a.size(); ++i) s += std::conj(a[i]) * b[i];
    return s;
}

// a^T b without conjugation (the bilinear form of the J-symmetric method)
cplx dotu(const std::vector<cplx>& a, const std::vector<cplx>& b) {
    cplx s(0.0, 0.0);
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

// complex Givens rotation [c s; -conj(s) c] [a; b] = [rho; 0], c real
void givens(cplx a, cplx b, double& c, cplx& s) {
    if (b == cplx(0.0, 0.0)) {
        c = 1.0;
        s = 0.0;
        return;
    }
    if (a == cplx(0.0, 0.0)) {
        c = 0.0;
        s = std::conj(b) / std::abs(b);
        return;
    }
    const double nu = std::hypot(std::abs(a), std::abs(b));
    c = std::abs(a) / nu;
    s = (a / std::abs(a)) * std::conj(b) / nu;
}

}  // namespace

extern "C" {

// Builds one structure. xyz_A [n][3] Angstrom, eta [n] Hartree, r0_A [n] Angstrom; mode bit 0: store
// T densely (n^2 doubles), bit 1: build L (all-pairs search, O(n^2)); without bit 1 only the
// row-by-row functions that compute L rows themselves may be used. Returns NULL on bad input.
void* orc_create(int64_t n, const double* xyz_A, const double* eta, const double* r0_A, double fermi_d,
                 double fermi_s, double cutoff_eps, double W, double tau, int mode) {
    if (n < 1 || !xyz_A || !eta || !r0_A || !(fermi_d > 0) || !(fermi_s > 0) || !(cutoff_eps > 0) ||
        !(cutoff_eps < 0.5) || !(W > 0) || !(tau > 0))
        return nullptr;
    for (int64_t i = 0; i < n; ++i)
        if (!(r0_A[i] > 0) || !(eta[i] > 0)) return nullptr;
    Problem* P = new (std::nothrow) Problem();
    if (!P) return nullptr;
    try {
        P->n = n;
        P->pos.resize(3 * n);
        for (int64_t i = 0; i < 3 * n; ++i) P->pos[i] = xyz_A[i] / kBohrA;
        P->eta.assign(eta, eta + n);
        P->wid.resize(n);
        for (int64_t i = 0; i < n; ++i) P->wid[i] = std::sqrt(2.0 / kPi) / eta[i];
        P->r0.resize(n);
        for (int64_t i = 0; i < n; ++i) P->r0[i] = r0_A[i] / kBohrA;
        P->fd = fermi_d;
        P->fs = fermi_s;
        P->cfac = 1.0 + std::log(1.0 / cutoff_eps - 1.0) / fermi_d;
        P->W = W;
        P->tau = tau;
        if (mode & 2) {
            std::vector<std::vector<int64_t>> cols(n);
            std::vector<std::vector<double>> vals(n);
#pragma omp parallel
            {
                std::vector<int64_t> c;
                std::vector<double> v;
#pragma omp for schedule(dynamic, 64)
                for (int64_t i = 0; i < n; ++i) {
                    P->l_row(i, c, v);
                    cols[i] = c;
                    vals[i] = v;
                }
            }
            P->rp.assign(n + 1, 0);
            for (int64_t i = 0; i < n; ++i) P->rp[i + 1] = P->rp[i] + (int64_t)cols[i].size();
            P->ci.resize(P->rp[n]);
            P->lv.resize(P->rp[n]);
            for (int64_t i = 0; i < n; ++i) {
                std::copy(cols[i].begin(), cols[i].end(), P->ci.begin() + P->rp[i]);
                std::copy(vals[i].begin(), vals[i].end(), P->lv.begin() + P->rp[i]);
            }
            P->have_L = true;
        }
        if (mode & 1) {
            P->T.resize((size_t)n * n);
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t i = 0; i < n; ++i)
                for (int64_t j = 0; j < n; ++j) P->T[(size_t)i * n + j] = P->t_elem(i, j);
        }
    } catch (...) {
        delete P;
        return nullptr;
    }
    return P;
}

void orc_destroy(void* h) { delete static_cast<Problem*>(h); }

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int64_t orc_nnz(void* h) {
    const Problem* P = static_cast<const Problem*>(h);
    return P->have_L ? P->rp[P->n] : -1;
}

// L as triplets (CSR order), nnz entries each
int orc_export_L(void* h, int64_t* rows, int64_t* cols, double* vals) {
    const Problem* P = static_cast<const Problem*>(h);
    if (!P->have_L) return 1;
    for (int64_t i = 0; i < P->n; ++i)
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) {
            rows[p] = i;
            cols[p] = P->ci[p];
            vals[p] = P->lv[p];
        }
    return 0;
}

void orc_sample_T(void* h, int64_t count, const int64_t* i, const int64_t* j, double* out) {
    const Problem* P = static_cast<const Problem*>(h);
    for (int64_t k = 0; k < count; ++k) out[k] = P->t_elem(i[k], j[k]);
}

// Y[c] = T X[c] for ncol real vectors [ncol][n]
void orc_apply_T(void* h, int ncol, const double* X, double* Y) {
    const Problem* P = static_cast<const Problem*>(h);
    for (int c = 0; c < ncol; ++c) P->apply_T2(X + (size_t)c * P->n, nullptr, Y + (size_t)c * P->n, nullptr);
}

// y[k] = (T x)[rows[k]] for ncol real vectors X [ncol][n] -> Y [ncol][count], from pairwise elements
// (a bounded sample of the matrix-free product, used to time it on structures too large to store T)
void orc_apply_T_rows(void* h, int64_t count, const int64_t* rows, int ncol, const double* X, double* Y) {
    const Problem* P = static_cast<const Problem*>(h);
    const int64_t n = P->n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < count; ++k) {
        std::vector<double> acc(ncol, 0.0);
        for (int64_t j = 0; j < n; ++j) {
            const double t = P->t_elem(rows[k], j);
            for (int c = 0; c < ncol; ++c) acc[c] += t * X[(size_t)c * n + j];
        }
        for (int c = 0; c < ncol; ++c) Y[(size_t)c * count + k] = acc[c];
    }
}

// y = (L T + z I) x, planar complex
int orc_apply(void* h, double z_re, double z_im, const double* xr, const double* xi, double* yr, double* yi) {
    const Problem* P = static_cast<const Problem*>(h);
    if (!P->have_L) return 1;
    std::vector<cplx> x(P->n), y;
    for (int64_t i = 0; i < P->n; ++i) x[i] = cplx(xr[i], xi[i]);
    P->apply_op(cplx(z_re, z_im), x, y);
    for (int64_t i = 0; i < P->n; ++i) {
        yr[i] = y[i].real();
        yi[i] = y[i].imag();
    }
    return 0;
}

void orc_shift(void* h, double omega_eV, double* z_re, double* z_im) {
    const cplx z = static_cast<const Problem*>(h)->shift(omega_eV);
    *z_re = z.real();
    *z_im = z.imag();
}

int orc_rhs(void* h, const double* dir, double E0, double* b) {
    const Problem* P = static_cast<const Problem*>(h);
    if (!P->have_L) return 1;
    std::vector<cplx> bb;
    P->rhs(dir, E0, bb);
    for (int64_t i = 0; i < P->n; ++i) b[i] = bb[i].real();
    return 0;
}

// q = (L T + z I)^-1 b by dense complex LU with partial pivoting (needs the stored T)
int orc_solve_lu(void* h, double omega_eV, const double* dir, double E0, double* qr, double* qi) {
    const Problem* P = static_cast<const Problem*>(h);
    if (!P->have_L || P->T.empty()) return 1;
    const int64_t n = P->n;
    const cplx z = P->shift(omega_eV);
    std::vector<cplx> M((size_t)n * n);
    // row i of L T is the combination of the rows of T selected by row i of L
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        cplx* mi = M.data() + (size_t)i * n;
        for (int64_t j = 0; j < n; ++j) mi[j] = 0.0;
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) {
            const double l = P->lv[p];
            const double* tk = P->T.data() + (size_t)P->ci[p] * n;
            for (int64_t j = 0; j < n; ++j) mi[j] += l * tk[j];
        }
        mi[i] += z;
    }
    std::vector<cplx> b;
    P->rhs(dir, E0, b);
    // forward elimination with row pivoting, applied to b as it goes
    for (int64_t k = 0; k < n; ++k) {
        int64_t piv = k;
        double best = std::abs(M[(size_t)k * n + k]);
        for (int64_t i = k + 1; i < n; ++i) {
            const double a = std::abs(M[(size_t)i * n + k]);
            if (a > best) {
                best = a;
                piv = i;
            }
        }
        if (best == 0.0) return 2;   // singular
        if (piv != k) {
            std::swap_ranges(M.begin() + (size_t)k * n, M.begin() + (size_t)(k + 1) * n, M.begin() + (size_t)piv * n);
            std::swap(b[k], b[piv]);
        }
        const cplx inv = 1.0 / M[(size_t)k * n + k];
        const cplx* mk = M.data() + (size_t)k * n;
#pragma omp parallel for schedule(static)
        for (int64_t i = k + 1; i < n; ++i) {
            cplx* mi = M.data() + (size_t)i * n;
            const cplx f = mi[k] * inv;
            if (f == cplx(0.0, 0.0)) continue;
            mi[k] = 0.0;
            for (int64_t j = k + 1; j < n; ++j) mi[j] -= f * mk[j];
            b[i] -= f * b[k];
        }
    }
    // back substitution
    for (int64_t i = n - 1; i >= 0; --i) {
        cplx s = b[i];
        const cplx* mi = M.data() + (size_t)i * n;
        for (int64_t j = i + 1; j < n; ++j) s -= mi[j] * b[j];
        b[i] = s / mi[i];
    }
    for (int64_t i = 0; i < n; ++i) {
        qr[i] = b[i].real();
        qi[i] = b[i].imag();
    }
    return 0;
}

// ||b - (L T + z I) q|| / ||b||
double orc_residual(void* h, double omega_eV, const double* dir, double E0, const double* qr, const double* qi) {
    const Problem* P = static_cast<const Problem*>(h);
    if (!P->have_L) return -1.0;
    std::vector<cplx> b, q(P->n), aq;
    P->rhs(dir, E0, b);
    for (int64_t i = 0; i < P->n; ++i) q[i] = cplx(qr[i], qi[i]);
    P->apply_op(P->shift(omega_eV), q, aq);
    double rr = 0.0, bb = 0.0;
    for (int64_t i = 0; i < P->n; ++i) {
        rr += std::norm(b[i] - aq[i]);
        bb += std::norm(b[i]);
    }
    return std::sqrt(rr / bb);
}

// Rows `rows` of b - (L T + z I) q, each from scratch: the row of L by checking every atom, the
// needed entries of T q from pairwise elements. Needs neither the stored T nor the whole L, so it
// serves structures too large for either.
void orc_residual_rows(void* h, double omega_eV, const double* dir, double E0, const double* qr, const double* qi,
                       int64_t count, const int64_t* rows, double* out_re, double* out_im) {
    const Problem* P = static_cast<const Problem*>(h);
    const int64_t n = P->n;
    const cplx z = P->shift(omega_eV);
    for (int64_t k = 0; k < count; ++k) {
        const int64_t i = rows[k];
        std::vector<int64_t> cols;
        std::vector<double> vals;
        P->l_row(i, cols, vals);
        const int64_t m = (int64_t)cols.size();
        std::vector<cplx> tq(m);
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < m; ++a) {
            double sr = 0.0, si = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                const double t = P->t_elem(cols[a], j);
                sr += t * qr[j];
                si += t * qi[j];
            }
            tq[a] = cplx(sr, si);
        }
        cplx lt(0.0, 0.0);
        double bi = 0.0;
        for (int64_t a = 0; a < m; ++a) {
            const int64_t j = cols[a];
            lt += vals[a] * tq[a];
            bi += vals[a] * (P->pos[3 * j] * dir[0] + P->pos[3 * j + 1] * dir[1] + P->pos[3 * j + 2] * dir[2]);
        }
        const cplx r = E0 * bi - (lt + z * cplx(qr[i], qi[i]));
        out_re[k] = r.real();
        out_im[k] = r.imag();
    }
}

// Restarted GMRES(m) from x0 (NULL: zero). Stops when the explicit relative residual, evaluated at
// every restart, is <= tol, or after maxiter products; the Givens estimate ends a cycle early.
// info[0] = products, info[1] = cycles; *relres = final explicit relative residual.
int orc_gmres(void* h, double omega_eV, const double* dir, double E0, int restart, double tol, int maxiter,
              const double* x0r, const double* x0i, double* qr, double* qi, int* info, double* relres) {
    const Problem* P = static_cast<const Problem*>(h);
    if (!P->have_L || restart < 1) return 1;
    const int64_t n = P->n;
    const cplx z = P->shift(omega_eV);
    std::vector<cplx> b, x(n, cplx(0.0, 0.0)), r, w;
    P->rhs(dir, E0, b);
    if (x0r)
        for (int64_t i = 0; i < n; ++i) x[i] = cplx(x0r[i], x0i ? x0i[i] : 0.0);
    const double bnorm = norm2(b);
    int iters = 0, cycles = 0;
    double rel = 0.0;
    const int m = restart;
    while (true) {
        P->apply_op(z, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        const double beta = norm2(r);
        rel = bnorm > 0.0 ? beta / bnorm : 0.0;
        if (rel <= tol || iters >= maxiter || bnorm == 0.0) break;
        ++cycles;
        std::vector<std::vector<cplx>> V(m + 1);
        std::vector<cplx> H((size_t)(m + 1) * m, cplx(0.0, 0.0));   // H[i * m + j]
        std::vector<double> cs(m, 0.0);
        std::vector<cplx> sn(m, cplx(0.0, 0.0)), g(m + 1, cplx(0.0, 0.0));
        g[0] = beta;
        V[0].resize(n);
        for (int64_t i = 0; i < n; ++i) V[0][i] = r[i] / beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            P->apply_op(z, V[j], w);
            ++iters;
            for (int i = 0; i <= j; ++i) {   // modified Gram-Schmidt
                const cplx hij = dotc(V[i], w);
                H[(size_t)i * m + j] = hij;
                for (int64_t t = 0; t < n; ++t) w[t] -= hij * V[i][t];
            }
            const double hn = norm2(w);
            H[(size_t)(j + 1) * m + j] = hn;
            V[j + 1].assign(n, cplx(0.0, 0.0));
            if (hn > 0.0)
                for (int64_t t = 0; t < n; ++t) V[j + 1][t] = w[t] / hn;
            for (int i = 0; i < j; ++i) {   // earlier rotations on the new column
                const cplx a = H[(size_t)i * m + j], c2 = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
                H[(size_t)(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * c2;
            }
            givens(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j], cs[j], sn[j]);
            H[(size_t)j * m + j] = cs[j] * H[(size_t)j * m + j] + sn[j] * H[(size_t)(j + 1) * m + j];
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -std::conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            if (std::abs(g[j + 1]) / bnorm <= tol || hn == 0.0 || iters >= maxiter) break;
        }
        std::vector<cplx> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cplx s = g[i];
            for (int j = i + 1; j < k; ++j) s -= H[(size_t)i * m + j] * y[j];
            y[i] = s / H[(size_t)i * m + i];
        }
        for (int j = 0; j < k; ++j)
            for (int64_t t = 0; t < n; ++t) x[t] += y[j] * V[j][t];
    }
    for (int64_t i = 0; i < n; ++i) {
        qr[i] = x[i].real();
        qi[i] = x[i].imag();
    }
    info[0] = iters;
    info[1] = cycles;
    *relres = rel;
    return 0;
}

// J-symmetric QMR from BCG (J = T) without look-ahead, from x0 = 0. One product with T per step
// (T p by the recurrence T p = T r + beta T p_old); QMR iterates by residual smoothing.
// info[0] = steps, info[1] = 1 on breakdown; *relres = smoothed (QMR) residual estimate / ||b||.
int orc_qmr(void* h, double omega_eV, const double* dir, double E0, double tol, int maxiter, double breakdown,
            double* qr, double* qi, int* info, double* relres) {
    const Problem* P = static_cast<const Problem*>(h);
    if (!P->have_L) return 1;
    const int64_t n = P->n;
    const cplx z = P->shift(omega_eV);
    std::vector<cplx> b, x(n, cplx(0.0, 0.0)), r, tr, p, tp, xq, s, q, lq;
    P->rhs(dir, E0, b);
    const double bnorm = norm2(b);
    info[0] = 0;
    info[1] = 0;
    if (bnorm == 0.0) {
        std::fill(qr, qr + n, 0.0);
        std::fill(qi, qi + n, 0.0);
        *relres = 0.0;
        return 0;
    }
    r = b;   // x0 = 0
    P->apply_Tc(r, tr);
    cplx rho = dotu(r, tr);
    p = r;
    tp = tr;
    xq = x;
    s = r;
    double tau2 = 0.0;
    for (const cplx& a : r) tau2 += std::norm(a);
    double hist = norm2(s) / bnorm;
    int iters = 0;
    while (iters < maxiter && hist > tol) {
        P->apply_Lc(tp, lq);
        q.resize(n);
        for (int64_t i = 0; i < n; ++i) q[i] = lq[i] + z * p[i];   // M p = L (T p) + z p
        const cplx sigma = dotu(tp, q);
        if (std::abs(sigma) <= breakdown * norm2(tp) * norm2(q) || std::abs(rho) <= breakdown * norm2(r) * norm2(tr)) {
            info[1] = 1;
            break;
        }
        const cplx alpha = rho / sigma;
        double nr2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            nr2 += std::norm(r[i]);
        }
        ++iters;
        if (nr2 == 0.0) {
            xq = x;
            s = r;
            hist = 0.0;
            break;
        }
        const double tau2n = 1.0 / (1.0 / tau2 + 1.0 / nr2);
        const double eta = tau2n / nr2;
        for (int64_t i = 0; i < n; ++i) {
            xq[i] += eta * (x[i] - xq[i]);
            s[i] += eta * (r[i] - s[i]);
        }
        tau2 = tau2n;
        hist = norm2(s) / bnorm;
        P->apply_Tc(r, tr);
        const cplx rho_n = dotu(r, tr);
        const cplx beta = rho_n / rho;
        rho = rho_n;
        for (int64_t i = 0; i < n; ++i) {
            p[i] = r[i] + beta * p[i];
            tp[i] = tr[i] + beta * tp[i];
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        qr[i] = xq[i].real();
        qi[i] = xq[i].imag();
    }
    info[0] = iters;
    *relres = hist;
    return 0;
}

// alpha_l = sum_i r_il q_i / E0 for l = x, y, z (complex, planar out)
void orc_polarisability(void* h, const double* qr, const double* qi, double E0, double* a_re, double* a_im) {
    const Problem* P = static_cast<const Problem*>(h);
    for (int l = 0; l < 3; ++l) {
        double sr = 0.0, si = 0.0;
        for (int64_t i = 0; i < P->n; ++i) {
            sr += P->pos[3 * i + l] * qr[i];
            si += P->pos[3 * i + l] * qi[i];
        }
        a_re[l] = sr / E0;
        a_im[l] = si / E0;
    }
}

}  // extern "C"
