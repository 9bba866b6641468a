// Kernels of the J-symmetric QMR-from-BCG iteration with J = T (arXiv 2103.00438, Section
// "Solution strategies", QMR paragraph, and the J-symmetry DA = A^T D of Eq. (a-matrix-d)).
//
// Because M^T T = T M for M = L T + z I, the BCG shadow sequence is T r_k and every inner product is
// the bilinear form x^T T y (no conjugation). Per step the only dense product is T r_k (a block
// product over all active systems); T p_k follows from the recurrence T p_k = T r_k + beta T p_{k-1},
// so M p_k = L (T p_k) + z p_k costs a sparse product only. The QMR iterate comes from the BCG one by
// quasi-minimal residual smoothing: 1/tau_k^2 = 1/tau_{k-1}^2 + 1/||r_k||^2, eta_k = tau_k^2/||r_k||^2,
// xq += eta_k (x_k - xq), s += eta_k (r_k - s).
//
// Vector slots of the per-system basis Q: 0 r, 1 p, 2 T p, 3 q = M p, 4 x (BCG), 5 xq (QMR), 6 s.
#include "device_util.h"
#include "krylov.h"

namespace wfq {

namespace {

__device__ inline double* slot(const Basis& V, int s, int j) {
    return V.base + (int64_t)s * V.sys_stride + (int64_t)j * V.vec_stride;
}

__device__ inline double block_sum4(double v, double* sh) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// partial rho = sum_i r_i (T r)_i, with T r in the packed block Y (rows 2k, 2k + 1)
template <typename YE>
__global__ void __launch_bounds__(256) rho_kernel(const YE* __restrict__ Y, int64_t ld, const int* __restrict__ sys,
                                                  Basis Q, int64_t n, double2* __restrict__ partial, int nblk) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    const int s = sys[k];
    double a = 0.0, b = 0.0;
    if (i < n) {
        const double* r = slot(Q, s, 0);
        const double rr = r[i], ri = r[i + Q.npad];
        const double tr = widen(Y[(int64_t)(2 * k) * ld + i]), ti = widen(Y[(int64_t)(2 * k + 1) * ld + i]);
        a = rr * tr - ri * ti;
        b = rr * ti + ri * tr;
    }
    a = block_sum4(a, sh);
    b = block_sum4(b, sh);
    if (threadIdx.x == 0) partial[(int64_t)s * nblk + blockIdx.x] = make_double2(a, b);
}

// beta = rho_new / rho_old (0 on the first step); p = r + beta p; T p = T r + beta T p
template <typename YE>
__global__ void __launch_bounds__(256) dirs_kernel(const YE* __restrict__ Y, int64_t ld, const int* __restrict__ sys,
                                                   Basis Q, int64_t n, const double2* __restrict__ rho_new,
                                                   const double2* __restrict__ rho_old, const int* __restrict__ first,
                                                   double* __restrict__ tpb) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int k = blockIdx.y;
    const int s = sys[k];
    double br = 0.0, bi = 0.0;
    if (!first[s]) {
        const double2 a = rho_new[s], c = rho_old[s];
        const double dd = c.x * c.x + c.y * c.y;
        br = (a.x * c.x + a.y * c.y) / dd;
        bi = (a.y * c.x - a.x * c.y) / dd;
    }
    const double* r = slot(Q, s, 0);
    double* p = slot(Q, s, 1);
    double* tp = slot(Q, s, 2);
    const int64_t o = Q.npad;
    const double pr = p[i], pi = p[i + o];
    p[i] = r[i] + br * pr - bi * pi;
    p[i + o] = r[i + o] + br * pi + bi * pr;
    const double tr = widen(Y[(int64_t)(2 * k) * ld + i]), ti = widen(Y[(int64_t)(2 * k + 1) * ld + i]);
    const double qr = tp[i], qi = tp[i + o];
    const double nr = tr + br * qr - bi * qi, ni = ti + br * qi + bi * qr;
    tp[i] = nr;
    tp[i + o] = ni;
    reinterpret_cast<double2*>(tpb)[(int64_t)s * ld + i] = make_double2(nr, ni);   // interleaved for the SpMM
}

// partial sums over 256-row blocks of sigma = (T p)^T q, ||T p||^2 and ||q||^2
__global__ void __launch_bounds__(256) q_sums_kernel(int64_t n, const int* __restrict__ sys, Basis Q,
                                                     double2* __restrict__ part_sig, double2* __restrict__ part_nrm,
                                                     int nblk) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int s = sys[blockIdx.y];
    double sr = 0.0, si = 0.0, nt = 0.0, nq = 0.0;
    if (i < n) {
        const int64_t o = Q.npad;
        const double* tp = slot(Q, s, 2);
        const double* q = slot(Q, s, 3);
        const double qr = q[i], qi = q[i + o], tr = tp[i], ti = tp[i + o];
        sr = tr * qr - ti * qi;
        si = tr * qi + ti * qr;
        nt = tr * tr + ti * ti;
        nq = qr * qr + qi * qi;
    }
    sr = block_sum4(sr, sh);
    si = block_sum4(si, sh);
    nt = block_sum4(nt, sh);
    nq = block_sum4(nq, sh);
    if (threadIdx.x == 0) {
        part_sig[(int64_t)s * nblk + blockIdx.x] = make_double2(sr, si);
        part_nrm[(int64_t)s * nblk + blockIdx.x] = make_double2(nt, nq);
    }
}

__global__ void __launch_bounds__(256) xr_kernel(const int* __restrict__ sys, Basis Q, int64_t n,
                                                 const double2* __restrict__ rho, const double2* __restrict__ sigma,
                                                 double* __restrict__ norm2, int nblk) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int s = sys[blockIdx.y];
    const double2 a = rho[s], c = sigma[s];
    const double dd = c.x * c.x + c.y * c.y;
    const double alr = (a.x * c.x + a.y * c.y) / dd, ali = (a.y * c.x - a.x * c.y) / dd;
    double nn = 0.0;
    if (i < n) {
        const int64_t o = Q.npad;
        double* r = slot(Q, s, 0);
        const double* p = slot(Q, s, 1);
        const double* q = slot(Q, s, 3);
        double* x = slot(Q, s, 4);
        const double pr = p[i], pi = p[i + o], qr = q[i], qi = q[i + o];
        x[i] += alr * pr - ali * pi;
        x[i + o] += alr * pi + ali * pr;
        const double rr = r[i] - (alr * qr - ali * qi), ri = r[i + o] - (alr * qi + ali * qr);
        r[i] = rr;
        r[i + o] = ri;
        nn = rr * rr + ri * ri;
    }
    nn = block_sum4(nn, sh);
    if (threadIdx.x == 0) norm2[(int64_t)s * nblk + blockIdx.x] = nn;
}

// per system: sigma = sum of partials and the breakdown test (Lanczos breakdown: no look-ahead)
__global__ void sigma_kernel(const int* __restrict__ sys, int nsys, const double2* __restrict__ part_sig,
                             const double2* __restrict__ part_nrm, int nblk, const double2* __restrict__ rho,
                             double2* __restrict__ sigma, int* __restrict__ flags, double thr) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsys) return;
    const int s = sys[k];
    double sr = 0, si = 0, nt = 0, nq = 0;
    for (int b = 0; b < nblk; ++b) {
        const double2 a = part_sig[(int64_t)s * nblk + b], c = part_nrm[(int64_t)s * nblk + b];
        sr += a.x;
        si += a.y;
        nt += c.x;
        nq += c.y;
    }
    sigma[s] = make_double2(sr, si);
    int f = 0;
    const double sabs = hypot(sr, si), rabs = hypot(rho[s].x, rho[s].y);
    if (!(sabs > thr * sqrt(nt * nq)) || !(rabs > 0.0)) f |= 8;
    if (!(sabs == sabs) || !(rabs == rabs)) f |= 4;
    flags[s] = f;
}

// per system: smoothing weights from the new BCG residual norm; clears the first-step flag
__global__ void weights_kernel(const int* __restrict__ sys, int nsys, const double* __restrict__ rn_part, int nblk,
                               double* __restrict__ tau2, double* __restrict__ eta, int* __restrict__ first) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsys) return;
    const int s = sys[k];
    double nr = 0;
    for (int b = 0; b < nblk; ++b) nr += rn_part[(int64_t)s * nblk + b];
    const double t2 = tau2[s];
    const double t2n = nr > 0.0 ? 1.0 / (1.0 / t2 + 1.0 / nr) : 0.0;
    eta[s] = nr > 0.0 ? t2n / nr : 1.0;
    tau2[s] = t2n;
    first[s] = 0;
}
}  // namespace

// reduce per-block complex partials of the systems in `sys`
__global__ void reduce_complex_kernel(const int* __restrict__ sys, int nsys, const double2* __restrict__ partial,
                                      int nb, double2* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsys) return;
    const int s = sys[k];
    double a = 0, b = 0;
    for (int q = 0; q < nb; ++q) {
        a += partial[(int64_t)s * nb + q].x;
        b += partial[(int64_t)s * nb + q].y;
    }
    out[s] = make_double2(a, b);
}

namespace {
// xq += eta (x - xq); s += eta (r - s); partial ||s||^2
__global__ void __launch_bounds__(256) smooth_kernel(const int* __restrict__ sys, Basis Q, int64_t n,
                                                     const double* __restrict__ eta, double* __restrict__ norm2,
                                                     int nblk) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int s = sys[blockIdx.y];
    const double e = eta[s];
    double nn = 0.0;
    if (i < n) {
        const int64_t o = Q.npad;
        const double* x = slot(Q, s, 4);
        double* xq = slot(Q, s, 5);
        const double* r = slot(Q, s, 0);
        double* sv = slot(Q, s, 6);
        xq[i] += e * (x[i] - xq[i]);
        xq[i + o] += e * (x[i + o] - xq[i + o]);
        const double a = sv[i] + e * (r[i] - sv[i]), b = sv[i + o] + e * (r[i + o] - sv[i + o]);
        sv[i] = a;
        sv[i + o] = b;
        nn = a * a + b * b;
    }
    nn = block_sum4(nn, sh);
    if (threadIdx.x == 0) norm2[(int64_t)s * nblk + blockIdx.x] = nn;
}

// restart: x = xq; p = 0, T p = 0; s = r (r holds the FP64 residual of xq)
__global__ void __launch_bounds__(256) restart_kernel(const int* __restrict__ sys, Basis Q, int64_t npad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int s = sys[blockIdx.y];
    for (int h = 0; h < 2; ++h) {
        const int64_t j = i + h * npad;
        slot(Q, s, 4)[j] = slot(Q, s, 5)[j];
        slot(Q, s, 1)[j] = 0.0;
        slot(Q, s, 2)[j] = 0.0;
        slot(Q, s, 6)[j] = slot(Q, s, 0)[j];
    }
}
}  // namespace

void qmr_rho(bool y_is_f64, const void* Y, int64_t ld, const int* sys, int nsys, const Basis& Q, int64_t n,
             double2* partial, int nblk, hipStream_t st) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)nblk, (unsigned)nsys);
    if (y_is_f64)
        hipLaunchKernelGGL(rho_kernel<double>, grd, dim3(256), 0, st, static_cast<const double*>(Y), ld, sys, Q, n,
                           partial, nblk);
    else
        hipLaunchKernelGGL(rho_kernel<float>, grd, dim3(256), 0, st, static_cast<const float*>(Y), ld, sys, Q, n,
                           partial, nblk);
    WFQ_CHECK_LAUNCH();
}

void qmr_dirs(bool y_is_f64, const void* Y, int64_t ld, const int* sys, int nsys, const Basis& Q, int64_t n,
              const double2* rho_new, const double2* rho_old, const int* first, double* tpb, hipStream_t st) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)((n + 255) / 256), (unsigned)nsys);
    if (y_is_f64)
        hipLaunchKernelGGL(dirs_kernel<double>, grd, dim3(256), 0, st, static_cast<const double*>(Y), ld, sys, Q, n,
                           rho_new, rho_old, first, tpb);
    else
        hipLaunchKernelGGL(dirs_kernel<float>, grd, dim3(256), 0, st, static_cast<const float*>(Y), ld, sys, Q, n,
                           rho_new, rho_old, first, tpb);
    WFQ_CHECK_LAUNCH();
}

void qmr_q(const Structure& S, const int* sys, int nsys, const Basis& Q, const double2* z, const double* tpb,
           double2* part_sig, double2* part_nrm, int nblk, hipStream_t st) {
    if (nsys <= 0) return;
    // q (slot 3) = L (T p) + z p (slot 1), gathering T p from the compact interleaved block that
    // qmr_dirs wrote (one pair of doubles per atom and system)
    spmm_shift_interleaved(S, tpb, S.npad, sys, nsys, z, Q, 1, 3, st);
    dim3 grd((unsigned)nblk, (unsigned)nsys);
    hipLaunchKernelGGL(q_sums_kernel, grd, dim3(256), 0, st, S.n, sys, Q, part_sig, part_nrm, nblk);
    WFQ_CHECK_LAUNCH();
}

void qmr_sigma(const int* sys, int nsys, const double2* part_sig, const double2* part_nrm, int nblk,
               const double2* rho, double2* sigma, int* flags, double thr, hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(sigma_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, sys, nsys, part_sig, part_nrm, nblk, rho,
                       sigma, flags, thr);
    WFQ_CHECK_LAUNCH();
}

void qmr_weights(const int* sys, int nsys, const double* rn_part, int nblk, double* tau2, double* eta, int* first,
                 hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(weights_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, sys, nsys, rn_part, nblk, tau2, eta,
                       first);
    WFQ_CHECK_LAUNCH();
}

void qmr_xr(const int* sys, int nsys, const Basis& Q, int64_t n, const double2* rho, const double2* sigma,
            double* norm2, int nblk, hipStream_t st) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)nblk, (unsigned)nsys);
    hipLaunchKernelGGL(xr_kernel, grd, dim3(256), 0, st, sys, Q, n, rho, sigma, norm2, nblk);
    WFQ_CHECK_LAUNCH();
}

void qmr_smooth(const int* sys, int nsys, const Basis& Q, int64_t n, const double* eta, double* norm2, int nblk,
                hipStream_t st) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)nblk, (unsigned)nsys);
    hipLaunchKernelGGL(smooth_kernel, grd, dim3(256), 0, st, sys, Q, n, eta, norm2, nblk);
    WFQ_CHECK_LAUNCH();
}

void qmr_restart(const int* sys, int nsys, const Basis& Q, hipStream_t st) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)(Q.npad / 256), (unsigned)nsys);
    hipLaunchKernelGGL(restart_kernel, grd, dim3(256), 0, st, sys, Q, Q.npad);
    WFQ_CHECK_LAUNCH();
}

void reduce_complex(const int* sys, int nsys, const double2* partial, int nb, double2* out, hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(reduce_complex_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, sys, nsys, partial, nb, out);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
