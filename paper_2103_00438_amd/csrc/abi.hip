// C interface of libwfq: argument checking, error reporting and handle ownership. The numerical
// work lives in build.hip (structure set-up), gemm.hip / otf.hip (T products), krylov.hip and
// solver.hip (batched Krylov solves) and serve.hip (request loop).
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "krylov.h"
#include "solver.h"

namespace wfq {

namespace {
thread_local std::string g_last_error;
}

void set_error(int code, const std::string& msg) {
    (void)code;
    g_last_error = msg;
}

}  // namespace wfq

using namespace wfq;

struct wfq_handle {
    Structure S;
    hipStream_t stream = nullptr;
    KernelStat stats[KC_COUNT];
};

namespace {

void* scratch_ptr(int device);   // the allocation-free entry point's scratch on `device` (defined below)

const char* kClassNames[KC_COUNT] = {"tx_gemm_f64", "tx_gemm_f32", "tx_gemm_bf16", "tx_skinny", "tx_otf_f32", "tx_otf_f64",
                                     "spmm_shift",  "cgs_dot",     "cgs_update",   "givens",    "pack",
                                     "x_update",    "fp64_residual", "qmr",        "block_jacobi", "other",
                                     "tx_skinny_f32", "tx_skinny_bf16", "tx_otf_narrow", "recycle"};

template <typename F>
int guarded(F&& f) {
    try {
        wfq::g_last_error.clear();
        return f();
    } catch (const Error& e) {
        set_error(e.code, e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error(WFQ_ENOMEM, "host allocation failed");
        return WFQ_ENOMEM;
    } catch (const std::exception& e) {
        set_error(WFQ_EDEVICE, e.what());
        return WFQ_EDEVICE;
    }
}

int fail(int code, const std::string& msg) { throw Error{code, msg}; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

void check_device(int device) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) fail(WFQ_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) fail(WFQ_EINVAL, "device ordinal out of range");
    hipDeviceProp_t prop;
    WFQ_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        fail(WFQ_EDEVICE, std::string("libwfq is built for gfx950, found ") + prop.gcnArchName);
    WFQ_HIP(hipSetDevice(device));
}

void check_opts(const wfq_solve_opts* o) {
    if (!o) fail(WFQ_EINVAL, "opts is NULL");
    if (o->algorithm != WFQ_GMRES && o->algorithm != WFQ_QMR && o->algorithm != WFQ_MSGMRES)
        fail(WFQ_EINVAL, "unknown algorithm");
    if (o->restart < 1) fail(WFQ_EINVAL, "restart must be >= 1");
    if (o->algorithm != WFQ_QMR && o->restart > 256) fail(WFQ_EINVAL, "GMRES restart must be in [1, 256]");
    if (o->shift_dim < 0 || o->shift_dim > 4096) fail(WFQ_EINVAL, "shift_dim must be in [0, 4096]");
    if (o->max_iter < 1) fail(WFQ_EINVAL, "max_iter must be >= 1");
    if (o->precision != WFQ_PREC_FP64 && o->precision != WFQ_PREC_FP32 && o->precision != WFQ_PREC_BF16)
        fail(WFQ_EINVAL, "unknown precision");
    if (!std::isfinite(o->E0) || o->E0 < 0.0) fail(WFQ_EINVAL, "E0 must be finite and >= 0");
    if (o->max_batch < 0) fail(WFQ_EINVAL, "max_batch must be >= 0");
    if (!(o->qmr_breakdown >= 0.0)) fail(WFQ_EINVAL, "qmr_breakdown must be >= 0");
    if (!std::isfinite(o->ms_relax)) fail(WFQ_EINVAL, "ms_relax must be finite");
    if (o->warm_start && o->algorithm != WFQ_GMRES) fail(WFQ_EINVAL, "warm starts are a GMRES option");
    if (o->recycle < 0 || o->recycle > 8) fail(WFQ_EINVAL, "recycle must be in [0, 8]");
    if (o->recycle && o->algorithm != WFQ_GMRES) fail(WFQ_EINVAL, "subspace recycling is a GMRES option");
    if (o->recycle && o->block_jacobi) fail(WFQ_EINVAL, "subspace recycling does not combine with block-Jacobi");
    if (o->block_jacobi && o->algorithm != WFQ_GMRES)
        fail(WFQ_EINVAL, "block-Jacobi preconditioning is a GMRES option");
    if (o->block_jacobi && o->warm_start) fail(WFQ_EINVAL, "block_jacobi and warm_start cannot be combined");
}

// ---- material closure: W = 2 Omega D / S (see wfq.h), on an ideal lattice generated here

constexpr double kBohrAng = 0.529177210903;     // Angstrom per bohr
constexpr double kHartreeEv = 27.211386245988;  // eV per Hartree

// S = sum_j (1 - f(r_0j)) x_0j^2 / r_0j over the neighbours of one site of the ideal lattice with
// nearest-neighbour distance nn (bohr) inside r_c = s nn cfac; 2D honeycomb or 3D FCC. Both lattices
// have a point group that makes the second moment isotropic, so the x component stands for any
// direction (in the plane for the sheet).
double closure_sum(int material, double nn, double fs, double fd, double cfac) {
    const double rc = fs * nn * cfac;
    double S = 0.0;
    auto add = [&](double x, double y, double z) {
        const double r = std::sqrt(x * x + y * y + z * z);
        if (r > 0.0 && r < rc) {
            const double f = 1.0 / (1.0 + std::exp(-fd * (r / (fs * nn) - 1.0)));   // Eq. (fermi)
            S += (1.0 - f) * x * x / r;
        }
    };
    if (material == WFQ_MATERIAL_GRAPHENE2D) {
        // honeycomb: lattice vectors nn (3/2, +-sqrt(3)/2), basis (0, 0) and (nn, 0)
        const double h = std::sqrt(3.0) / 2.0;
        const int K = (int)std::ceil(rc / nn) + 2;
        for (int i = -K; i <= K; ++i)
            for (int j = -K; j <= K; ++j) {
                const double x = nn * 1.5 * (i + j), y = nn * h * (i - j);
                add(x, y, 0.0);
                add(x + nn, y, 0.0);
            }
    } else {
        // FCC: cube edge a = sqrt(2) nn, points (i, j, k) a / 2 with i + j + k even
        const double half = std::sqrt(2.0) * nn / 2.0;
        const int K = (int)std::ceil(rc / half) + 1;
        for (int i = -K; i <= K; ++i)
            for (int j = -K; j <= K; ++j)
                for (int k = -K; k <= K; ++k)
                    if (((i + j + k) & 1) == 0) add(i * half, j * half, k * half);
    }
    return S;
}

// W: the override, or the closure for the material (p already checked)
double material_weight(const wfq_params* p, double r0_species0) {
    if (p->W > 0.0) return p->W;
    if (p->material != WFQ_MATERIAL_GRAPHENE2D && p->material != WFQ_MATERIAL_METAL3D)
        fail(WFQ_EINVAL, "need W > 0 or a material (WFQ_MATERIAL_GRAPHENE2D / WFQ_MATERIAL_METAL3D)");
    const double nn = (p->lattice_nn > 0.0 ? p->lattice_nn : r0_species0) / kBohrAng;
    const double cfac = 1.0 + std::log(1.0 / p->cutoff_eps - 1.0) / p->fermi_d;
    const double S = closure_sum(p->material, nn, p->fermi_s, p->fermi_d, cfac);
    if (!(S > 0.0)) fail(WFQ_EINVAL, "the material closure found no neighbour inside the cutoff");
    double omega, D;
    if (p->material == WFQ_MATERIAL_GRAPHENE2D) {
        if (!finite_pos(p->fermi_energy)) fail(WFQ_EINVAL, "graphene2D needs fermi_energy > 0 (eV)");
        omega = 3.0 * std::sqrt(3.0) / 4.0 * nn * nn;   // area per atom
        D = p->fermi_energy / kHartreeEv / M_PI;         // Drude weight of the sheet, eps_F / pi
    } else {
        if (!finite_pos(p->valence)) fail(WFQ_EINVAL, "metal3D needs valence > 0");
        const double m = p->eff_mass > 0.0 ? p->eff_mass : 1.0;
        const double a = std::sqrt(2.0) * nn;
        omega = a * a * a / 4.0;                         // volume per atom
        D = p->valence / omega / m;                      // n_e / m*
    }
    return 2.0 * omega * D / S;
}

// per-atom hardness and r0 (caller order) from the geometry, the species table and the defaults
void resolve_atoms(const wfq_geometry* g, const wfq_params* p, std::vector<double>& eta, std::vector<double>& r0) {
    const int64_t n = g->n;
    eta.assign(n, p->eta);
    r0.assign(n, p->r0);
    if (p->n_species > 0) {
        if (!p->species) fail(WFQ_EINVAL, "n_species > 0 needs the species table");
        for (int k = 0; k < p->n_species; ++k)
            if (!finite_pos(p->species[k].eta) || !finite_pos(p->species[k].r0))
                fail(WFQ_EINVAL, "every species needs eta > 0 and r0 > 0");
        for (int64_t i = 0; i < n; ++i) {
            const int k = g->species ? g->species[i] : 0;
            if (k < 0 || k >= p->n_species) fail(WFQ_EINVAL, "species index out of range");
            eta[i] = p->species[k].eta;
            r0[i] = p->species[k].r0;
        }
    } else if (g->species) {
        fail(WFQ_EINVAL, "a species array needs n_species > 0 and the species table");
    }
    if (g->eta)
        for (int64_t i = 0; i < n; ++i) eta[i] = g->eta[i];
    for (int64_t i = 0; i < n; ++i) {
        if (!finite_pos(eta[i])) fail(WFQ_EINVAL, "eta must be finite and > 0");
        if (!finite_pos(r0[i])) fail(WFQ_EINVAL, "r0 must be finite and > 0");
    }
}

void check_solve_args(const wfq_handle* h, const double* omegas, int n_omega, const double* dirs, int n_dir,
                      double tol, const wfq_solve_opts* o) {
    if (!h) fail(WFQ_EINVAL, "handle is NULL");
    if (n_omega < 1 || n_dir < 1) fail(WFQ_EINVAL, "need n_omega >= 1 and n_dir >= 1");
    if (!omegas || !dirs) fail(WFQ_EINVAL, "omegas and dirs must not be NULL");
    if (!(tol > 0.0) || !(tol < 1.0)) fail(WFQ_EINVAL, "tol must be in (0, 1)");
    check_opts(o);
    for (int d = 0; d < n_dir; ++d) {
        double nn = 0;
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(dirs[3 * d + a])) fail(WFQ_EINVAL, "field direction is not finite");
            nn += dirs[3 * d + a] * dirs[3 * d + a];
        }
        if (std::fabs(nn - 1.0) > 1e-9) fail(WFQ_EINVAL, "field directions must be unit vectors");
    }
    for (int k = 0; k < n_omega; ++k) {
        if (!std::isfinite(omegas[k])) fail(WFQ_EINVAL, "frequency is not finite");
        if (omegas[k] <= 0.0)
            fail(WFQ_ESINGULAR, "omega <= 0: z(omega) = 0 and L T is singular (rows of L sum to zero)");
    }
}

}  // namespace

extern "C" {

const char* wfq_last_error(void) { return wfq::g_last_error.c_str(); }

int wfq_material_weight(const wfq_params* p, double* W) {
    return guarded([&]() -> int {
        if (!p || !W) fail(WFQ_EINVAL, "params and W must not be NULL");
        if (!finite_pos(p->fermi_d) || !finite_pos(p->fermi_s) || !(p->cutoff_eps > 0.0 && p->cutoff_eps < 0.5))
            fail(WFQ_EINVAL, "fermi_d, fermi_s > 0 and cutoff_eps in (0, 0.5) are needed");
        const double r0 = p->n_species > 0 && p->species ? p->species[0].r0 : p->r0;
        if (!finite_pos(r0) && !(p->lattice_nn > 0.0)) fail(WFQ_EINVAL, "need r0 > 0 or lattice_nn > 0");
        *W = material_weight(p, r0);
        return WFQ_OK;
    });
}

int wfq_isotropic_sigma(const double* dirs, const wfq_result* info, int32_t n_omega, double* sigma_iso) {
    return guarded([&]() -> int {
        if (!dirs || !info || !sigma_iso || n_omega < 1) fail(WFQ_EINVAL, "bad arguments");
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double d = 0.0;
                for (int l = 0; l < 3; ++l) d += dirs[3 * a + l] * dirs[3 * b + l];
                if (!(std::fabs(d - (a == b ? 1.0 : 0.0)) <= 1e-9))
                    fail(WFQ_EINVAL, "the three field directions must be orthonormal");
            }
        for (int w = 0; w < n_omega; ++w)
            sigma_iso[w] = (info[3 * w].sigma + info[3 * w + 1].sigma + info[3 * w + 2].sigma) / 3.0;
        return WFQ_OK;
    });
}

int wfq_build(const wfq_geometry* g, const wfq_params* p, wfq_handle** out) {
    if (out) *out = nullptr;
    return guarded([&]() -> int {
        if (!g || !p || !out) fail(WFQ_EINVAL, "geometry, params and out must not be NULL");
        if (g->n < 2) fail(WFQ_EINVAL, "need at least 2 atoms");
        if (g->n > (int64_t)1 << 30) fail(WFQ_EINVAL, "too many atoms");
        if (!g->xyz) fail(WFQ_EINVAL, "xyz is NULL");
        for (int64_t i = 0; i < 3 * g->n; ++i)
            if (!std::isfinite(g->xyz[i])) fail(WFQ_EINVAL, "positions must be finite");
        if (!finite_pos(p->fermi_d) || !finite_pos(p->fermi_s))
            fail(WFQ_EINVAL, "fermi_d and fermi_s must be finite and > 0");
        if (!(p->cutoff_eps > 0.0 && p->cutoff_eps < 0.5)) fail(WFQ_EINVAL, "cutoff_eps must be in (0, 0.5)");
        if (!finite_pos(p->tau)) fail(WFQ_EINVAL, "tau must be finite and > 0");
        if (!(p->W >= 0.0) || !std::isfinite(p->W)) fail(WFQ_EINVAL, "W must be finite and >= 0");
        std::vector<double> eta_atom, r0_atom;
        resolve_atoms(g, p, eta_atom, r0_atom);
        const double W = material_weight(p, p->n_species > 0 ? p->species[0].r0 : p->r0);
        if (p->t_mode < WFQ_TMODE_AUTO || p->t_mode > WFQ_TMODE_OTF) fail(WFQ_EINVAL, "unknown t_mode");
        if (p->store_mask & ~7u) fail(WFQ_EINVAL, "unknown store_mask bits");
        check_device(p->device);
        auto* h = new wfq_handle();
        h->S.device = p->device;
        for (int k = 0; k < KC_COUNT; ++k) h->stats[k].name = kClassNames[k];
        try {
            WFQ_HIP(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
            size_t free_b = 0, total_b = 0;
            WFQ_HIP(hipMemGetInfo(&free_b, &total_b));
            h->S.budget = p->device_budget ? p->device_budget : (uint64_t)(0.9 * (double)free_b);
            build_structure(h->S, g, p, eta_atom.data(), r0_atom.data(), W, h->stream);
            (void)scratch_ptr(p->device);   // set-up of wfq_apply_op_noalloc's scratch on this device
        } catch (...) {
            free_structure(h->S);
            if (h->stream) (void)hipStreamDestroy(h->stream);
            delete h;
            throw;
        }
        *out = h;
        if (!h->S.connected) {
            set_error(WFQ_EDISCONNECTED, "the Kbar graph is not connected; each component conserves its own charge");
            return WFQ_EDISCONNECTED;
        }
        return WFQ_OK;
    });
}

void wfq_destroy(wfq_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->S.device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_structure(h->S);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

static int solve_impl(wfq_handle* h, const double* omegas_eV, int32_t n_omega, const double* dirs, int32_t n_dir,
                      double tol, const wfq_solve_opts* o, const SolveOutputs& out, hipStream_t st) {
    return guarded([&]() -> int {
        check_solve_args(h, omegas_eV, n_omega, dirs, n_dir, tol, o);
        WFQ_HIP(hipSetDevice(h->S.device));
        if (h->S.t_mode != WFQ_TMODE_STORED && o->precision == WFQ_PREC_BF16)
            fail(WFQ_EINVAL, "matrix-free T runs in FP32 or FP64");
        int rc = solve_all(h->S, omegas_eV, n_omega, dirs, n_dir, tol, *o, out, st, o->timing ? h->stats : nullptr);
        if (rc != WFQ_OK) set_error(rc, "some systems did not converge cleanly (see info[].status)");
        return rc;
    });
}

int wfq_solve(wfq_handle* h, const double* omegas_eV, int32_t n_omega, const double* dirs, int32_t n_dir, double tol,
              const wfq_solve_opts* o, double* q_re, double* q_im, double* alpha_re, double* alpha_im,
              wfq_result* info) {
    SolveOutputs out;
    out.q_re = q_re;
    out.q_im = q_im;
    out.alpha_re = alpha_re;
    out.alpha_im = alpha_im;
    out.info = info;
    out.on_device = false;
    return solve_impl(h, omegas_eV, n_omega, dirs, n_dir, tol, o, out, h ? h->stream : nullptr);
}

int wfq_solve_dev(wfq_handle* h, const double* omegas_eV, int32_t n_omega, const double* dirs, int32_t n_dir,
                  double tol, const wfq_solve_opts* o, double* q_re_dev, double* q_im_dev, double* alpha_re_dev,
                  double* alpha_im_dev, wfq_result* info, void* stream) {
    SolveOutputs out;
    out.q_re = q_re_dev;
    out.q_im = q_im_dev;
    out.alpha_re = alpha_re_dev;
    out.alpha_im = alpha_im_dev;
    out.info = info;
    out.on_device = true;
    return solve_impl(h, omegas_eV, n_omega, dirs, n_dir, tol, o, out, static_cast<hipStream_t>(stream));
}

int wfq_info(const wfq_handle* h, int64_t* n, int64_t* nnz_L, int64_t* bytes_device) {
    return guarded([&]() -> int {
        if (!h) fail(WFQ_EINVAL, "handle is NULL");
        if (n) *n = h->S.n;
        if (nnz_L) *nnz_L = h->S.nnz;
        if (bytes_device) *bytes_device = (int64_t)h->S.bytes;
        return WFQ_OK;
    });
}

namespace {
__global__ void sample_kernel(int prec, const double* T64, const float* T32, const uint16_t* T16, int64_t npad,
                              const int64_t* ii, const int64_t* jj, int64_t count, double* out) {
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    int64_t o = ii[k] * npad + jj[k];
    out[k] = prec == WFQ_PREC_FP64 ? T64[o]
             : prec == WFQ_PREC_FP32 ? (double)T32[o]
                                     : (double)__uint_as_float((uint32_t)T16[o] << 16);
}
}  // namespace

int wfq_sample_T(const wfq_handle* h, int32_t precision, const int64_t* i, const int64_t* j, int64_t count,
                 double* out) {
    return guarded([&]() -> int {
        if (!h || !i || !j || !out || count < 0) fail(WFQ_EINVAL, "bad arguments");
        const Structure& S = h->S;
        if (S.t_mode != WFQ_TMODE_STORED) fail(WFQ_EINVAL, "T is not stored");
        if ((precision == WFQ_PREC_FP64 && !S.T64) || (precision == WFQ_PREC_FP32 && !S.T32) ||
            (precision == WFQ_PREC_BF16 && !S.T16) || precision < 0 || precision > 2)
            fail(WFQ_EINVAL, "that copy of T was not built");
        if (count == 0) return WFQ_OK;
        std::vector<int64_t> ii(count), jj(count);
        for (int64_t k = 0; k < count; ++k) {
            if (i[k] < 0 || i[k] >= S.n || j[k] < 0 || j[k] >= S.n) fail(WFQ_EINVAL, "index out of range");
            ii[k] = S.iperm[i[k]];
            jj[k] = S.iperm[j[k]];
        }
        WFQ_HIP(hipSetDevice(S.device));
        int64_t *di = nullptr, *dj = nullptr;
        double* dout = nullptr;
        WFQ_HIP(hipMalloc(&di, count * 8));
        WFQ_HIP(hipMalloc(&dj, count * 8));
        WFQ_HIP(hipMalloc(&dout, count * 8));
        h2d_sync(h->S, di, ii.data(), count * 8, h->stream);
        h2d_sync(h->S, dj, jj.data(), count * 8, h->stream);
        hipLaunchKernelGGL(sample_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, h->stream, precision,
                           S.T64, S.T32, S.T16, S.npad, di, dj, count, dout);
        WFQ_CHECK_LAUNCH();
        d2h_sync(h->S, out, dout, count * 8, h->stream);
        (void)hipFree(di);
        (void)hipFree(dj);
        (void)hipFree(dout);
        return WFQ_OK;
    });
}

int wfq_export_L(const wfq_handle* h, int64_t* rows, int64_t* cols, double* vals) {
    return guarded([&]() -> int {
        if (!h || !rows || !cols || !vals) fail(WFQ_EINVAL, "bad arguments");
        const Structure& S = h->S;
        WFQ_HIP(hipSetDevice(S.device));
        std::vector<int32_t> rp(S.n + 1), cl(S.nnz);
        std::vector<double> vl(S.nnz);
        d2h_sync(S, rp.data(), S.rowptr, (S.n + 1) * 4, h->stream);
        d2h_sync(S, cl.data(), S.col, S.nnz * 4, h->stream);
        d2h_sync(S, vl.data(), S.val, S.nnz * 8, h->stream);
        for (int64_t i = 0; i < S.n; ++i)
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                rows[p] = S.perm[i];
                cols[p] = S.perm[cl[p]];
                vals[p] = vl[p];
            }
        return WFQ_OK;
    });
}

namespace {
// Y = T X in `precision` through the automatic shape choice (variant < 0) or one registered variant.
int apply_T_impl(wfq_handle* h, int32_t precision, int32_t variant, int32_t ncol, const double* X, double* Y) {
    return guarded([&]() -> int {
        if (!h || !X || !Y || ncol < 1) fail(WFQ_EINVAL, "bad arguments");
        if (precision < 0 || precision > 2) fail(WFQ_EINVAL, "unknown precision");
        Structure& S = h->S;
        if (variant >= 0) {
            if (S.t_mode == WFQ_TMODE_OTF) fail(WFQ_EINVAL, "kernel variants apply to a stored T");
            if (variant >= tx_variant_count(precision)) fail(WFQ_EINVAL, "no such kernel variant");
            if (ncol > tx_variant_max_ncol(precision, variant)) fail(WFQ_EINVAL, "the variant cannot take that many columns");
        }
        WFQ_HIP(hipSetDevice(S.device));
        const int64_t np = S.npad, n = S.n;
        const int64_t rows = round_up(ncol, kColPad);
        std::vector<double> xh((size_t)rows * np, 0.0);
        for (int c = 0; c < ncol; ++c)
            for (int64_t k = 0; k < n; ++k) xh[(size_t)c * np + k] = X[(size_t)c * n + S.perm[k]];
        double *dx64 = nullptr, *dy64 = nullptr;
        void *dx = nullptr, *dy = nullptr;
        WFQ_HIP(hipMalloc(&dx64, rows * np * 8));
        WFQ_HIP(hipMalloc(&dx, rows * np * 8));
        WFQ_HIP(hipMalloc(&dy, rows * np * 8));
        h2d_sync(h->S, dx64, xh.data(), rows * np * 8, h->stream);
        convert_from_f64(precision, dx64, dx, rows * np, h->stream);
        std::vector<double> yh((size_t)ncol * np);
        if (variant >= 0)
            tx_variant_run(S, precision, variant, dx, dy, ncol, h->stream);
        else
            tx_any(S, precision, dx, dy, ncol, h->stream);
        if (precision == WFQ_PREC_FP64) {
            d2h_sync(S, yh.data(), dy, (size_t)ncol * np * 8, h->stream);
        } else {
            std::vector<float> yf((size_t)ncol * np);
            d2h_sync(S, yf.data(), dy, (size_t)ncol * np * 4, h->stream);
            for (size_t q = 0; q < yf.size(); ++q) yh[q] = yf[q];
        }
        WFQ_HIP(hipStreamSynchronize(h->stream));
        (void)dy64;
        (void)hipFree(dx64);
        (void)hipFree(dx);
        (void)hipFree(dy);
        for (int c = 0; c < ncol; ++c)
            for (int64_t k = 0; k < n; ++k) Y[(size_t)c * n + S.perm[k]] = yh[(size_t)c * np + k];
        return WFQ_OK;
    });
}
}  // namespace

int wfq_apply_T(wfq_handle* h, int32_t precision, int32_t ncol, const double* X, double* Y) {
    return apply_T_impl(h, precision, -1, ncol, X, Y);
}

int wfq_apply_T_variant(wfq_handle* h, int32_t precision, int32_t variant, int32_t ncol, const double* X, double* Y) {
    return apply_T_impl(h, precision, variant, ncol, X, Y);
}

}  // extern "C"

// ---- the allocation-free operator entry point (wfq_apply_op_noalloc)
//
// Its scratch (the systems' vectors in the internal order, the shifts, the packed block, the
// product and the split-k partial tiles) lives in one static device array. Every GPU the library
// runs on holds its own copy for the life of the process; the host reaches it only through the
// address hipGetSymbolAddress returns for the current device, kept per device below.
namespace {

constexpr uint64_t kNoAllocScratchBytes = 256ull << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of this device's scratch array (looked up once per device, with it current)
void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) fail(WFQ_EDEVICE, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(WFQ_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

// sys[k] = k, zs[k] = (z_re[k], z_im[k])
__global__ void na_setup_kernel(int nsys, const double* __restrict__ z_re, const double* __restrict__ z_im,
                                double2* __restrict__ zs, int* __restrict__ sys) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsys) return;
    zs[k] = make_double2(z_re[k], z_im[k]);
    sys[k] = k;
}

// slot 0 of system s (re, im planes) = X_s in the internal order, zero padding; slot 1 cleared
__global__ void na_gather_kernel(int64_t n, int64_t npad, const int32_t* __restrict__ perm,
                                 const double* __restrict__ x_re, const double* __restrict__ x_im,
                                 double* __restrict__ V) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npad) return;
    const int64_t s = blockIdx.y;
    double* v = V + s * 4 * npad;
    const bool in = i < n;
    v[i] = in ? x_re[s * n + perm[i]] : 0.0;
    v[npad + i] = in ? x_im[s * n + perm[i]] : 0.0;
    v[2 * npad + i] = 0.0;
    v[3 * npad + i] = 0.0;
}

// zero `words` 16-byte words (a fill kernel rather than a memset node, so the call can be captured)
__global__ void na_zero_kernel(uint4* __restrict__ p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// restores the structure's own split-k work space when the call ends
struct FixedSplit {
    const Structure& S;
    FixedSplit(const Structure& s, void* p, uint64_t bytes) : S(s) {
        S.split_fixed = p;
        S.split_fixed_bytes = bytes;
    }
    ~FixedSplit() {
        S.split_fixed = nullptr;
        S.split_fixed_bytes = 0;
    }
};

}  // namespace

extern "C" {

uint64_t wfq_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int wfq_apply_op_noalloc(wfq_handle* h, int32_t precision, int32_t nsys, const double* z_re_dev,
                         const double* z_im_dev, const double* X_re_dev, const double* X_im_dev, double* Y_re_dev,
                         double* Y_im_dev, void* stream) {
    return guarded([&]() -> int {
        if (!h || !z_re_dev || !z_im_dev || !X_re_dev || !X_im_dev || !Y_re_dev || !Y_im_dev || nsys < 1)
            fail(WFQ_EINVAL, "bad arguments");
        if (precision < 0 || precision > 2) fail(WFQ_EINVAL, "unknown precision");
        Structure& S = h->S;
        if (S.t_mode == WFQ_TMODE_OTF && precision == WFQ_PREC_BF16) fail(WFQ_EINVAL, "matrix-free T runs in FP32 or FP64");
        if (S.t_mode == WFQ_TMODE_STORED &&
            ((precision == WFQ_PREC_FP64 && !S.T64) || (precision == WFQ_PREC_FP32 && !S.T32) ||
             (precision == WFQ_PREC_BF16 && !S.T16)))
            fail(WFQ_EINVAL, "that copy of T was not built");
        const int64_t np = S.npad;
        const int64_t rows = round_up(2 * (int64_t)nsys, kColPad);
        const uint64_t es = precision == WFQ_PREC_FP64 ? 8 : precision == WFQ_PREC_FP32 ? 4 : 2;
        const uint64_t os = precision == WFQ_PREC_FP64 ? 8 : 4;
        auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
        const uint64_t v_bytes = up((uint64_t)nsys * 4 * np * 8), z_bytes = up((uint64_t)nsys * 16),
                       s_bytes = up((uint64_t)nsys * 4), x_bytes = up((uint64_t)rows * np * es),
                       y_bytes = up((uint64_t)rows * np * os);
        const uint64_t need = v_bytes + z_bytes + s_bytes + x_bytes + y_bytes;
        if (need > kNoAllocScratchBytes)
            fail(WFQ_ENOMEM, "wfq_apply_op_noalloc: " + std::to_string(nsys) + " systems of " + std::to_string(S.n) +
                                 " atoms need " + std::to_string(need >> 20) + " MiB of scratch, more than its " +
                                 std::to_string(kNoAllocScratchBytes >> 20) + " MiB");
        WFQ_HIP(hipSetDevice(S.device));
        char* base = static_cast<char*>(scratch_ptr(S.device));
        double* V = reinterpret_cast<double*>(base);
        double2* zs = reinterpret_cast<double2*>(base + v_bytes);
        int* sys = reinterpret_cast<int*>(base + v_bytes + z_bytes);
        void* X = base + v_bytes + z_bytes + s_bytes;
        void* Y = base + v_bytes + z_bytes + s_bytes + x_bytes;
        FixedSplit fs(S, base + need, kNoAllocScratchBytes - need);
        hipStream_t st = static_cast<hipStream_t>(stream);
        hipLaunchKernelGGL(na_setup_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, nsys, z_re_dev, z_im_dev, zs, sys);
        WFQ_CHECK_LAUNCH();
        hipLaunchKernelGGL(na_gather_kernel, dim3((unsigned)(np / 256), (unsigned)nsys), dim3(256), 0, st, S.n, np,
                           S.dperm, X_re_dev, X_im_dev, V);
        WFQ_CHECK_LAUNCH();
        const int64_t words = (int64_t)(x_bytes / 16);
        hipLaunchKernelGGL(na_zero_kernel, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 4096)), dim3(256), 0,
                           st, static_cast<uint4*>(X), words);
        WFQ_CHECK_LAUNCH();
        const Basis Vb{V, 4 * np, 2 * np, np};
        pack_columns(precision, Vb, sys, nsys, 0, nullptr, false, X, np, st);
        tx_any(S, precision, X, Y, 2 * nsys, st);
        spmm_shift(S, precision == WFQ_PREC_FP64, Y, np, sys, nsys, zs, Vb, 0, 1, st);
        scatter_q(S, S.dperm, sys, nsys, Basis{V + 2 * np, 4 * np, 2 * np, np}, Y_re_dev, Y_im_dev, st);
        return WFQ_OK;
    });
}

int wfq_apply_op(wfq_handle* h, int32_t precision, int32_t nsys, const double* z_re, const double* z_im,
                 const double* X_re, const double* X_im, double* Y_re, double* Y_im) {
    return guarded([&]() -> int {
        if (!h || !z_re || !z_im || !X_re || !X_im || !Y_re || !Y_im || nsys < 1) fail(WFQ_EINVAL, "bad arguments");
        if (precision < 0 || precision > 2) fail(WFQ_EINVAL, "unknown precision");
        Structure& S = h->S;
        WFQ_HIP(hipSetDevice(S.device));
        const int64_t np = S.npad, n = S.n;
        // two vector slots per system: 0 = input, 1 = output
        const int64_t sys_stride = 4 * np;
        std::vector<double> vh((size_t)nsys * sys_stride, 0.0);
        for (int s = 0; s < nsys; ++s)
            for (int64_t k = 0; k < n; ++k) {
                vh[(size_t)s * sys_stride + k] = X_re[(size_t)s * n + S.perm[k]];
                vh[(size_t)s * sys_stride + np + k] = X_im[(size_t)s * n + S.perm[k]];
            }
        std::vector<double2> zh(nsys);
        std::vector<int> sl(nsys);
        for (int s = 0; s < nsys; ++s) {
            zh[s] = make_double2(z_re[s], z_im[s]);
            sl[s] = s;
        }
        const int64_t rows = round_up(2 * (int64_t)nsys, kColPad);
        double* dv = nullptr;
        double2* dz = nullptr;
        int* dsys = nullptr;
        void *dx = nullptr, *dy = nullptr;
        WFQ_HIP(hipMalloc(&dv, vh.size() * 8));
        WFQ_HIP(hipMalloc(&dz, nsys * sizeof(double2)));
        WFQ_HIP(hipMalloc(&dsys, nsys * sizeof(int)));
        WFQ_HIP(hipMalloc(&dx, rows * np * 8));
        WFQ_HIP(hipMalloc(&dy, rows * np * 8));
        WFQ_HIP(hipMemsetAsync(dx, 0, rows * np * 8, h->stream));
        h2d_sync(h->S, dv, vh.data(), vh.size() * 8, h->stream);
        h2d_sync(h->S, dz, zh.data(), nsys * sizeof(double2), h->stream);
        h2d_sync(h->S, dsys, sl.data(), nsys * sizeof(int), h->stream);
        Basis V{dv, sys_stride, 2 * np, np};
        pack_columns(precision, V, dsys, nsys, 0, nullptr, false, dx, np, h->stream);
        tx_any(S, precision, dx, dy, 2 * nsys, h->stream);
        spmm_shift(S, precision == WFQ_PREC_FP64, dy, np, dsys, nsys, dz, V, 0, 1, h->stream);
        d2h_sync(S, vh.data(), dv, vh.size() * 8, h->stream);
        (void)hipFree(dv);
        (void)hipFree(dz);
        (void)hipFree(dsys);
        (void)hipFree(dx);
        (void)hipFree(dy);
        for (int s = 0; s < nsys; ++s)
            for (int64_t k = 0; k < n; ++k) {
                Y_re[(size_t)s * n + S.perm[k]] = vh[(size_t)s * sys_stride + 2 * np + k];
                Y_im[(size_t)s * n + S.perm[k]] = vh[(size_t)s * sys_stride + 3 * np + k];
            }
        return WFQ_OK;
    });
}

int wfq_rhs(wfq_handle* h, const double* dirs, int32_t n_dir, double E0, double* out) {
    return guarded([&]() -> int {
        if (!h || !dirs || !out || n_dir < 1) fail(WFQ_EINVAL, "bad arguments");
        Structure& S = h->S;
        WFQ_HIP(hipSetDevice(S.device));
        double *dd = nullptr, *db = nullptr;
        WFQ_HIP(hipMalloc(&dd, 3 * n_dir * 8));
        WFQ_HIP(hipMalloc(&db, (size_t)n_dir * S.npad * 8));
        h2d_sync(h->S, dd, dirs, 3 * n_dir * 8, h->stream);
        build_rhs(S, dd, n_dir, E0 != 0.0 ? E0 : 1.0, db, S.npad, h->stream);
        std::vector<double> bh((size_t)n_dir * S.npad);
        d2h_sync(S, bh.data(), db, bh.size() * 8, h->stream);
        (void)hipFree(dd);
        (void)hipFree(db);
        for (int d = 0; d < n_dir; ++d)
            for (int64_t k = 0; k < S.n; ++k) out[(size_t)d * S.n + S.perm[k]] = bh[(size_t)d * S.npad + k];
        return WFQ_OK;
    });
}

int wfq_tx_variants(int32_t precision, int32_t* count, const char** names, int32_t* max_ncol) {
    return guarded([&]() -> int {
        if (!count) fail(WFQ_EINVAL, "count is NULL");
        if (precision < 0 || precision > 2) fail(WFQ_EINVAL, "unknown precision");
        *count = tx_variant_count(precision);
        for (int k = 0; k < *count; ++k) {
            if (names) names[k] = tx_variant_name(precision, k);
            if (max_ncol) max_ncol[k] = tx_variant_max_ncol(precision, k);
        }
        return WFQ_OK;
    });
}

int wfq_tune(wfq_handle* h, int32_t precision, const int32_t* ncols, int32_t n_ncols, int32_t reps, double* ms,
             int32_t* chosen) {
    return guarded([&]() -> int {
        if (!h || !ncols || n_ncols < 1 || reps < 1) fail(WFQ_EINVAL, "bad arguments");
        if (precision < 0 || precision > 2) fail(WFQ_EINVAL, "unknown precision");
        Structure& S = h->S;
        if (S.t_mode != WFQ_TMODE_STORED) fail(WFQ_EINVAL, "T is not stored");
        WFQ_HIP(hipSetDevice(S.device));
        const int nv = tx_variant_count(precision);
        std::vector<double> row(nv);
        for (int q = 0; q < n_ncols; ++q) {
            if (ncols[q] < 1 || ncols[q] > 4096) fail(WFQ_EINVAL, "ncol must be in [1, 4096]");
            tune_tx(S, precision, ncols[q], reps, row.data(), h->stream);
            if (ms)
                for (int k = 0; k < nv; ++k) ms[(size_t)q * nv + k] = row[k];
            if (chosen) chosen[q] = S.tuned[precision].count(ncols[q]) ? S.tuned[precision][ncols[q]] : -1;
        }
        return WFQ_OK;
    });
}

int wfq_kernel_stats(wfq_handle* h, int32_t* n_classes, const char** names, int64_t* launches, double* total_ms,
                     double* flops, double* bytes, int32_t reset) {
    return guarded([&]() -> int {
        if (!h || !n_classes) fail(WFQ_EINVAL, "bad arguments");
        *n_classes = KC_COUNT;
        for (int k = 0; k < KC_COUNT; ++k) {
            if (names) names[k] = h->stats[k].name;
            if (launches) launches[k] = h->stats[k].launches;
            if (total_ms) total_ms[k] = h->stats[k].ms;
            if (flops) flops[k] = h->stats[k].flops;
            if (bytes) bytes[k] = h->stats[k].bytes;
        }
        if (reset)
            for (int k = 0; k < KC_COUNT; ++k) {
                h->stats[k].launches = 0;
                h->stats[k].ms = h->stats[k].flops = h->stats[k].bytes = 0;
            }
        return WFQ_OK;
    });
}

}  // extern "C"
