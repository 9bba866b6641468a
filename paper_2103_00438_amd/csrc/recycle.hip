// Subspace recycling across neighbouring frequencies (an extension behind a flag; the paper starts
// every solve from q0 = 0 and names recycling as the way to exploit the shift structure of a
// spectrum, in its conclusions).
//
// GMRES augmented with a fixed recycle space (GCRO, de Sturler 1999; Parks, de Sturler, Mackey,
// Johnson and Maiti 2006): for a system A x = b with a recycle space U of k vectors and
// C = A U orthonormalised (C = Q, U' = U R^-1, so A U' = C and C^H C = I),
//   * every cycle starts from the projected residual: x += U' C^H r, r -= C C^H r;
//   * every Arnoldi product is kept orthogonal to C: z -= C (C^H z), with the coefficients
//     B = C^H A Q recorded, so that (I - C C^H) A Q = Q Hbar and A Q = C B + Q Hbar;
//   * at the end of a cycle x += Q y - U' (B y), y the usual Hessenberg least-squares solution.
// The recycle space of a frequency is the span of the solutions at the nearest solved frequencies
// (same field direction). A U needs no product: the final FP64 residual r_a of a solved system
// gives L T q_a = b - r_a - z_a q_a, so A(z) q_a = b - r_a + (z - z_a) q_a.
//
// The Arnoldi process of the batched solver is DCGS2 (dcgs.hip): at step k the product z = A u is
// taken of the first-pass vector u, and q_k = (u - Q a) / rho follows from the step's dots. The
// recorded column is therefore C^H A q_k = (C^H z - B(:, 0:k-1) a) / rho, formed after the step's
// coefficients are known.
//
// Vectors of the recycle space live in the layout of Basis: system s, vector i at
// base + s sys_stride + i vec_stride, real plane then imaginary plane (npad apart). Reductions are
// deterministic: fixed 512-row chunks per wave, chunk partials added in order.
#include "device_util.h"
#include "krylov.h"

namespace wfq {

namespace {

__device__ inline double* vslot(const Basis& V, int s, int j) {
    return V.base + (int64_t)s * V.sys_stride + (int64_t)j * V.vec_stride;
}

__device__ inline double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// part[(s kmax + i) nwc + wc] = sum over chunk wc of conj(C_i) v, v = V(s, j), for i < min(kk[s], lim).
// One wave per (chunk, i, system).
__global__ void __launch_bounds__(64) rc_dots_kernel(Basis C, int kmax, const int* __restrict__ kk, int lim, Basis V,
                                                     int j, const int* __restrict__ sys, const int* __restrict__ run,
                                                     int64_t n, double2* __restrict__ part, int64_t nwc) {
    const int64_t wc = blockIdx.x;
    const int i = blockIdx.y;
    const int s = sys[blockIdx.z];
    if ((run && !run[s]) || i >= min(kk[s], lim)) return;
    const int lane = threadIdx.x;
    const double* cr = vslot(C, s, i);
    const double* vr = vslot(V, s, j);
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t row = wc * kWaveRows + 64 * r + lane;
        if (row < n) {
            const double a = cr[row], b = cr[row + C.npad], x = vr[row], y = vr[row + V.npad];
            sr += a * x + b * y;   // conj(c) v
            si += a * y - b * x;
        }
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) part[((int64_t)s * kmax + i) * nwc + wc] = make_double2(sr, si);
}

// coef[s kmax + i] = sum over chunks of part (chunk order); zero for i >= min(kk[s], lim)
__global__ void __launch_bounds__(64) rc_coef_kernel(int kmax, const int* __restrict__ kk, int lim,
                                                     const int* __restrict__ sys, const int* __restrict__ run,
                                                     const double2* __restrict__ part, int64_t nwc,
                                                     double2* __restrict__ coef) {
    const int i = blockIdx.x;
    const int s = sys[blockIdx.y];
    if (run && !run[s]) return;
    const int lane = threadIdx.x;
    double sr = 0.0, si = 0.0;
    if (i < min(kk[s], lim)) {
        const double2* p = part + ((int64_t)s * kmax + i) * nwc;
        for (int64_t w = lane; w < nwc; w += 64) {   // lane-strided, then a fixed butterfly
            sr += p[w].x;
            si += p[w].y;
        }
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) coef[(int64_t)s * kmax + i] = make_double2(sr, si);
}

// V(s, j) -= sum_{i < min(kk, lim)} C_i coef_i and, with X, X(s, jx) += sgn sum U_i coef_i; with norm2,
// the block partials of |V(s, j)|^2 after the update (rows >= n untouched and counted as 0)
__global__ void __launch_bounds__(256) rc_sub_kernel(Basis C, Basis U, int kmax, const int* __restrict__ kk, int lim,
                                                     Basis V, int j, Basis X, int jx, double sgn,
                                                     const int* __restrict__ sys, const int* __restrict__ run,
                                                     int64_t n, const double2* __restrict__ coef,
                                                     double* __restrict__ norm2, int nblk) {
    __shared__ double sh[4];
    const int s = sys[blockIdx.y];
    if (run && !run[s]) return;   // uniform per block
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int kc = min(kk[s], lim);
    double nn = 0.0;
    if (row < n) {
        double* vr = vslot(V, s, j);
        double re = vr[row], im = vr[row + V.npad];
        double xr = 0.0, xi = 0.0;
        for (int i = 0; i < kc; ++i) {
            const double2 c = coef[(int64_t)s * kmax + i];
            const double* cr = vslot(C, s, i);
            const double a = cr[row], b = cr[row + C.npad];
            re -= a * c.x - b * c.y;
            im -= a * c.y + b * c.x;
            if (X.base) {
                const double* ur = vslot(U, s, i);
                const double p = ur[row], q = ur[row + U.npad];
                xr += p * c.x - q * c.y;
                xi += p * c.y + q * c.x;
            }
        }
        vr[row] = re;
        vr[row + V.npad] = im;
        if (X.base) {
            double* x = vslot(X, s, jx);
            x[row] += sgn * xr;
            x[row + X.npad] += sgn * xi;
        }
        nn = re * re + im * im;
    }
    if (norm2) {
        nn = block_sum256(nn, sh);
        if (threadIdx.x == 0 && (int)blockIdx.x < nblk) norm2[(int64_t)s * nblk + blockIdx.x] = nn;
    }
}

// Column k of B: B[s][i][k] = (cu_i - sum_{t < k} B[s][i][t] a_t) / rho, a_t the first-pass dots of
// step k (dots[s][t]) and 1 / rho from the step's coefficients
__global__ void __launch_bounds__(64) rc_bcol_kernel(int kmax, const int* __restrict__ kk, const int* __restrict__ sys,
                                                     int nsys, const int* __restrict__ run, int k, int mdim,
                                                     const double2* __restrict__ cu, const double2* __restrict__ dots,
                                                     const double* __restrict__ inv_rho, double2* __restrict__ Bm) {
    const int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= nsys * kmax) return;
    const int s = sys[q / kmax], i = q % kmax;
    if ((run && !run[s]) || i >= kk[s]) return;
    const double2* d = dots + (int64_t)s * 2 * mdim;
    double2* b = Bm + ((int64_t)s * kmax + i) * mdim;
    double2 acc = cu[(int64_t)s * kmax + i];
    for (int t = 0; t < k; ++t) {
        const double2 bt = b[t], at = d[t];
        acc.x -= bt.x * at.x - bt.y * at.y;
        acc.y -= bt.x * at.y + bt.y * at.x;
    }
    const double ir = inv_rho[s];
    b[k] = make_double2(acc.x * ir, acc.y * ir);
}

// X(s) -= sum_i U_i (B y)_i over the k[s] completed columns of the cycle
__global__ void __launch_bounds__(256) rc_xfix_kernel(Basis U, int kmax, const int* __restrict__ kk, Basis X,
                                                      const int* __restrict__ sys, const int* __restrict__ ksteps,
                                                      const double2* __restrict__ y, int mdim,
                                                      const double2* __restrict__ Bm, int64_t n) {
    __shared__ double2 c[8];
    const int s = sys[blockIdx.y];
    const int kc = kk[s], K = ksteps[s];
    if (threadIdx.x < kc) {
        const double2* b = Bm + ((int64_t)s * kmax + threadIdx.x) * mdim;
        const double2* ys = y + (int64_t)s * mdim;
        double2 acc = make_double2(0.0, 0.0);
        for (int t = 0; t < K; ++t) {
            acc.x += b[t].x * ys[t].x - b[t].y * ys[t].y;
            acc.y += b[t].x * ys[t].y + b[t].y * ys[t].x;
        }
        c[threadIdx.x] = acc;
    }
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= n || kc == 0) return;
    double xr = 0.0, xi = 0.0;
    for (int i = 0; i < kc; ++i) {
        const double* ur = vslot(U, s, i);
        const double p = ur[row], q = ur[row + U.npad];
        xr += p * c[i].x - q * c[i].y;
        xi += p * c[i].y + q * c[i].x;
    }
    double* x = vslot(X, s, 0);
    x[row] -= xr;
    x[row + X.npad] -= xi;
}

// Recycle space of target system sys[t] from its neighbours nbr[t][i] (-1: none):
// C_i = b_dir - r_a + (z_s - z_a) x_a and U_i = x_a, with r_a = V(a, 0) and x_a = X(a)
__global__ void __launch_bounds__(256) rc_init_kernel(Basis C, Basis U, int kmax, Basis V, Basis X,
                                                      const double* __restrict__ b, const int* __restrict__ dir,
                                                      const double2* __restrict__ z, const int* __restrict__ sys,
                                                      const int* __restrict__ nbr, int64_t n) {
    const int t = blockIdx.z, i = blockIdx.y;
    const int s = sys[t];
    const int a = nbr[t * kmax + i];
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= C.npad) return;
    double* cr = vslot(C, s, i);
    double* ur = vslot(U, s, i);
    if (a < 0 || row >= n) {
        cr[row] = cr[row + C.npad] = 0.0;
        ur[row] = ur[row + U.npad] = 0.0;
        return;
    }
    const double* ra = vslot(V, a, 0);
    const double* xa = vslot(X, a, 0);
    const double dzr = z[s].x - z[a].x, dzi = z[s].y - z[a].y;
    const double xr = xa[row], xi = xa[row + X.npad];
    const double bb = b[(int64_t)dir[s] * V.npad + row];
    cr[row] = bb - ra[row] + dzr * xr - dzi * xi;
    cr[row + C.npad] = -ra[row + V.npad] + dzr * xi + dzi * xr;
    ur[row] = xr;
    ur[row + U.npad] = xi;
}

// C_i *= inv[s], U_i *= inv[s]
__global__ void __launch_bounds__(256) rc_scale_kernel(Basis C, Basis U, int i, const int* __restrict__ sys,
                                                       const double* __restrict__ inv) {
    const int s = sys[blockIdx.y];
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= C.npad) return;
    const double f = inv[s];
    double* cr = vslot(C, s, i);
    double* ur = vslot(U, s, i);
    cr[row] *= f;
    cr[row + C.npad] *= f;
    ur[row] *= f;
    ur[row + U.npad] *= f;
}

}  // namespace

void rc_project(const RecycleSpace& R, const Basis& V, int j, const Basis* X, const int* sys, int nsys,
                const int* run, int64_t n, double* norm2, int nblk, hipStream_t st) {
    if (nsys <= 0 || R.kmax <= 0) return;
    const int64_t nwc = wave_chunks(n);
    hipLaunchKernelGGL(rc_dots_kernel, dim3((unsigned)nwc, (unsigned)R.kmax, (unsigned)nsys), dim3(64), 0, st, R.C,
                       R.kmax, R.kk, R.kmax, V, j, sys, run, n, R.part, nwc);
    WFQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(rc_coef_kernel, dim3((unsigned)R.kmax, (unsigned)nsys), dim3(64), 0, st, R.kmax, R.kk, R.kmax,
                       sys, run, R.part, nwc, R.coef);
    WFQ_CHECK_LAUNCH();
    const Basis none{};
    hipLaunchKernelGGL(rc_sub_kernel, dim3((unsigned)(V.npad / 256), (unsigned)nsys), dim3(256), 0, st, R.C, R.U,
                       R.kmax, R.kk, R.kmax, V, j, X ? *X : none, 0, 1.0, sys, run, n, R.coef, norm2, nblk);
    WFQ_CHECK_LAUNCH();
}

void rc_bcol(const RecycleSpace& R, const int* sys, int nsys, const int* run, int k, int mdim, const double2* dots,
             const double* inv_rho, hipStream_t st) {
    if (nsys <= 0 || R.kmax <= 0) return;
    hipLaunchKernelGGL(rc_bcol_kernel, dim3((unsigned)((nsys * R.kmax + 63) / 64)), dim3(64), 0, st, R.kmax, R.kk, sys,
                       nsys, run, k, mdim, R.coef, dots, inv_rho, R.Bm);
    WFQ_CHECK_LAUNCH();
}

void rc_xfix(const RecycleSpace& R, const Basis& X, const int* sys, int nsys, const int* ksteps, const double2* y,
             int mdim, int64_t n, hipStream_t st) {
    if (nsys <= 0 || R.kmax <= 0) return;
    if (R.kmax > 8) throw Error{WFQ_EINVAL, "recycle space above 8 vectors"};
    hipLaunchKernelGGL(rc_xfix_kernel, dim3((unsigned)(X.npad / 256), (unsigned)nsys), dim3(256), 0, st, R.U, R.kmax,
                       R.kk, X, sys, ksteps, y, mdim, R.Bm, n);
    WFQ_CHECK_LAUNCH();
}

void rc_init(const RecycleSpace& R, const Basis& V, const Basis& X, const double* b, const int* dir, const double2* z,
             const int* sys, int nsys, const int* nbr, int64_t n, hipStream_t st) {
    if (nsys <= 0 || R.kmax <= 0) return;
    hipLaunchKernelGGL(rc_init_kernel, dim3((unsigned)(R.C.npad / 256), (unsigned)R.kmax, (unsigned)nsys), dim3(256), 0,
                       st, R.C, R.U, R.kmax, V, X, b, dir, z, sys, nbr, n);
    WFQ_CHECK_LAUNCH();
}

void rc_orth_step(const RecycleSpace& R, int i, const int* sys, int nsys, int64_t n, double* norm2, int nblk,
                  hipStream_t st) {
    if (nsys <= 0) return;
    const int64_t nwc = wave_chunks(n);
    if (i > 0) {
        hipLaunchKernelGGL(rc_dots_kernel, dim3((unsigned)nwc, (unsigned)i, (unsigned)nsys), dim3(64), 0, st, R.C,
                           R.kmax, R.kk, i, R.C, i, sys, nullptr, n, R.part, nwc);
        WFQ_CHECK_LAUNCH();
        hipLaunchKernelGGL(rc_coef_kernel, dim3((unsigned)i, (unsigned)nsys), dim3(64), 0, st, R.kmax, R.kk, i, sys,
                           nullptr, R.part, nwc, R.coef);
        WFQ_CHECK_LAUNCH();
    }
    // C_i -= sum_{l < i} C_l coef_l, U_i -= sum_{l < i} U_l coef_l, and |C_i|^2 partials
    hipLaunchKernelGGL(rc_sub_kernel, dim3((unsigned)(R.C.npad / 256), (unsigned)nsys), dim3(256), 0, st, R.C, R.U,
                       R.kmax, R.kk, i, R.C, i, R.U, i, -1.0, sys, nullptr, n, R.coef, norm2, nblk);
    WFQ_CHECK_LAUNCH();
}

void rc_scale(const RecycleSpace& R, int i, const int* sys, int nsys, const double* inv, hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(rc_scale_kernel, dim3((unsigned)(R.C.npad / 256), (unsigned)nsys), dim3(256), 0, st, R.C, R.U, i,
                       sys, inv);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
