// Multi-shift GMRES: one Krylov basis for every frequency of a field direction.
//
// The scaled system (L T + z I) q = b_k has a real, frequency-independent matrix L T; the frequency
// only enters as the uniform complex diagonal shift z (arXiv 2103.00438, the remark after Eq.
// wfq-a-matrix), and b_k = E0 L r_k does not depend on it. Krylov spaces are invariant under such
// shifts (the conclusions point to this property for spectra): with the Arnoldi relation
// A V_k = V_{k+1} Hbar_k of A = L T started from b_k,
//     (A + z I) V_k = V_{k+1} (Hbar_k + z Ibar_k),   Ibar_k = [I_k; 0],
// so the GMRES iterate of every shifted system is x = V_k y_z with y_z the least-squares solution of
// (Hbar_k + z Ibar_k) y ~ ||b_k|| e_1. A and b_k are real, hence V and Hbar are real: one real
// Arnoldi process per direction (one T product on a real vector per step, shared by all
// frequencies) and one small complex Givens recurrence per (frequency, direction) system.
//
// Layouts: basis of direction d, slot j at V + (d * mdim1 + j) * npad (FP64, padding rows zero); the
// kept products T u_j (FP64 solves) in the same layout; Hessenberg column j of direction d at
// H + (d * m + j) * (m + 1) (entries 0..j+1), and the triangular factor S of U = Q S likewise.
// Per-system arrays are system-minor (entry e of system s at e * S + s, S = systems of the batch):
// rotations cs/sn (m entries), g (m + 1), R packed by columns (column j from entry j (j + 1) / 2).
// The phase's own orthogonalisation is the one-reduction form below (ms_dcgs_*); ms_dot and ms_update
// serve the starting norms and the relaxed phase's product-error probe.
#include <algorithm>
#include <type_traits>

#include "device_util.h"
#include "krylov.h"

namespace wfq {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cscale(double c, double2 a) { return make_double2(c * a.x, c * a.y); }
__device__ inline double cabs(double2 a) { return hypot(a.x, a.y); }
__device__ inline double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

__device__ inline double* slot(double* V, int64_t npad, int mdim1, int d, int j) {
    return V + ((int64_t)d * mdim1 + j) * npad;
}

// X[c][i] = cast(v) with v = V(d_c, j)[i] * scale[d_c], which is also written back (normalises the
// new basis vector on its way into the product).
template <typename E>
__global__ void __launch_bounds__(256) ms_pack_kernel(double* __restrict__ V, int64_t npad, int mdim1, int j,
                                                      const int* __restrict__ dirs, const double* __restrict__ scale,
                                                      E* __restrict__ X, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    const int d = dirs[c];
    double* v = slot(V, npad, mdim1, d, j);
    const double a = v[i] * scale[d];
    v[i] = a;
    X[(int64_t)c * ld + i] = cast_from_double<E>(a);
}

// V(d_c, jdst) = L Y[c] for the NC columns c0 .. c0 + NC - 1 (real ELL rows; padding rows get 0).
// Each thread reads its row of L once for all NC columns.
template <typename YE, int NC>
__global__ void __launch_bounds__(256) ms_spmm_kernel(int64_t n, int64_t npad, int w, const int32_t* __restrict__ ecol,
                                                      const double* __restrict__ eval, const YE* __restrict__ Y,
                                                      int64_t ld, const int* __restrict__ dirs, double* __restrict__ V,
                                                      int mdim1, int jdst, int c0, double* __restrict__ TV,
                                                      const double* __restrict__ Yi) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    if (i < n) {
        const YE* y = Y + (int64_t)c0 * ld;
        if (Yi) {
            // the interleaved copy: all columns of neighbour j in one aligned 32-byte load
#pragma unroll 4
            for (int e = 0; e < w; ++e) {
                const double v = eval[(int64_t)e * npad + i];
                const int64_t j = ecol[(int64_t)e * npad + i];
                const doublex4 yj = *reinterpret_cast<const doublex4*>(Yi + 4 * j);
                const double yv[4] = {yj.x, yj.y, yj.z, yj.w};
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] += v * yv[c];
            }
        } else {
#pragma unroll 4
            for (int e = 0; e < w; ++e) {
                const double v = eval[(int64_t)e * npad + i];
                const int64_t j = ecol[(int64_t)e * npad + i];
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] += v * widen(y[c * ld + j]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) slot(V, npad, mdim1, dirs[c0 + c], jdst)[i] = acc[c];
    if (TV) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            slot(TV, npad, mdim1, dirs[c0 + c], jdst - 1)[i] = i < n ? widen(Y[(int64_t)(c0 + c) * ld + i]) : 0.0;
    }
}

// partial[d][i][wc] = sum over wave chunk wc (512 rows) of V(d, i) * V(d, jw) for i < nvec; with
// self_norm also partial[d][nvec][wc] = sum of V(d, jw)^2. One wave per (chunk, vector): the
// launch has thousands of waves even for one direction, and each sum has a fixed order.
__global__ void __launch_bounds__(256) ms_dot_kernel(const double* __restrict__ V, int64_t n, int64_t npad, int mdim1,
                                                     int nvec, int jw, const int* __restrict__ dirs,
                                                     double* __restrict__ partial, int pslots, int64_t nwc,
                                                     int self_norm) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wc = blockIdx.x;
    const int i = blockIdx.y * 4 + wave;
    if (i >= nvec + self_norm) return;
    const int d = dirs[blockIdx.z];
    const double* w = V + ((int64_t)d * mdim1 + jw) * npad;
    const double* v = i < nvec ? V + ((int64_t)d * mdim1 + i) * npad : w;
    const int64_t row0 = wc * kWaveRows + lane;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t row = row0 + 64 * r;
        if (row < n) s += v[row] * w[row];
    }
    s = wave_sum(s);
    if (lane == 0) partial[((int64_t)d * pslots + i) * nwc + wc] = s;
}

// h[d][i] = sum_wc partial[d][i][wc], i < count: one wave per (value, direction); lane l adds the
// chunks l, l + 64, ... and the lanes are combined by a fixed butterfly (same order every call)
__global__ void __launch_bounds__(256) ms_reduce_kernel(const int* __restrict__ dirs, const double* __restrict__ partial,
                                                        int pslots, int64_t nwc, int count, double* __restrict__ h) {
    const int d = dirs[blockIdx.y];
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= count) return;   // uniform over the wave
    const double* p = partial + ((int64_t)d * pslots + i) * nwc;
    double s = 0.0;
    for (int64_t q = lane; q < nwc; q += 64) s += p[q];
    s = wave_sum(s);
    if (lane == 0) h[(int64_t)d * pslots + i] = s;
}

// V(d, jw) -= sum_{i < nvec} h[d][i] V(d, i); with norm != NULL also norm[d][blk] = the sum of
// V(d, jw)^2 over the 64 rows of block blk. A block owns 64 rows; its 4 waves take every 4th basis
// vector and their partial sums are combined in LDS in a fixed order.
constexpr int kMsRows = 64;
__global__ void __launch_bounds__(256) ms_update_kernel(double* __restrict__ V, int64_t n, int64_t npad, int mdim1,
                                                        int nvec, int jw, const int* __restrict__ dirs,
                                                        const double* __restrict__ h, int pslots,
                                                        double* __restrict__ norm) {
    __shared__ double part[4][kMsRows];
    const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t row = (int64_t)blockIdx.x * kMsRows + r;
    const int d = dirs[blockIdx.y];
    const double* hd = h + (int64_t)d * pslots;
    double acc = 0.0;
    if (row < n) {
#pragma unroll 4
        for (int i = q; i < nvec; i += 4) acc += hd[i] * V[((int64_t)d * mdim1 + i) * npad + row];
    }
    part[q][r] = acc;
    __syncthreads();
    if (q == 0) {
        double* w = V + ((int64_t)d * mdim1 + jw) * npad;
        double x = 0.0;
        if (row < n) {
            x = w[row] - ((part[0][r] + part[1][r]) + (part[2][r] + part[3][r]));
            w[row] = x;
        }
        if (norm) {
            const double s2 = wave_sum(x * x);
            if (r == 0) norm[(int64_t)d * (npad / kMsRows) + blockIdx.x] = s2;
        }
    }
}

// ---- Arnoldi with one reduction per step on the real basis of each direction: classical
// Gram-Schmidt with delayed reorthogonalisation (DCGS2, Swirydowicz, Langou, Ananthan, Yang and
// Thomas 2020), the real counterpart of the batched GMRES's. At step k, q_0 .. q_{k-1} are final,
// slot k holds u (the previous step's once-projected vector p, normalised by the pack) and slot
// k + 1 holds z = A u. One sweep gives a = Q^T u, alpha = u^T u, b = Q^T z and beta = u^T z
// (dots[d][e]: e = t < k: a_t; e = k: alpha; e = k + 1 + t: b_t; e = 2 k + 1: beta); then with
// rho = sqrt(alpha - |a|^2) and nu = |p|:
//   q_k = (u - Q a) / rho;  H(0:k-1, k-1) = hp + nu a,  H(k, k-1) = nu rho   (column k-1 complete)
//   gamma = q_k^T z = (beta - a^T b) / rho;  p' = (z - Q b - gamma q_k) / rho
//   hp'(0:k-1) = (b - (Hbar a)(0:k-1)) / rho,  hp'(k) = (gamma - H(k, k-1) a_{k-1}) / rho
// since A q_k = (z - Q_{k+1} Hbar a) / rho by A Q_k = Q_{k+1} Hbar. The basis is read twice per step
// instead of four times; column k-1 is complete (and its Givens step taken) at step k, and a last
// step without product completes column m-1. As u_k = rho q_k + Q a, the vectors that entered the
// products relate to the final basis by U = Q S with S upper triangular (S(t, k) = a_t,
// S(k, k) = rho), kept column by column in the layout of H when the products T u_k are kept.

// partial[d][e][wc] for the entries e above over wave chunk wc (512 rows). One wave per (chunk, group
// of kDotGroup basis vectors t <= k, direction): u and z of the chunk stay in registers while the
// wave computes v_t . u and v_t . z for its vectors (t = k: alpha and beta).
constexpr int kDotGroup = 16;
__global__ void __launch_bounds__(256) ms_dcgs_dot_kernel(const double* __restrict__ V, int64_t n, int64_t npad,
                                                          int mdim1, int k, int with_z, const int* __restrict__ dirs,
                                                          double* __restrict__ partial, int ps, int64_t nwc) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wc = (int64_t)blockIdx.x * 4 + wave;
    if (wc >= nwc) return;   // uniform over the wave
    const int t0 = blockIdx.y * kDotGroup, t1 = min(t0 + kDotGroup, k + 1);
    const int d = dirs[blockIdx.z];
    const double* u = V + ((int64_t)d * mdim1 + k) * npad;
    const double* zv = u + npad;   // slot k + 1 (read only with z)
    const int64_t row0 = wc * kWaveRows + lane;
    double xu[8], xz[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t row = row0 + 64 * r;
        xu[r] = row < n ? u[row] : 0.0;
        xz[r] = (with_z && row < n) ? zv[row] : 0.0;
    }
    double* P = partial + (int64_t)d * ps * nwc + wc;
#pragma unroll 2
    for (int t = t0; t < t1; ++t) {
        const double* v = V + ((int64_t)d * mdim1 + t) * npad;
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t row = row0 + 64 * r;
            const double x = row < n ? v[row] : 0.0;
            sa += x * xu[r];
            sb += x * xz[r];
        }
        sa = wave_sum(sa);
        sb = wave_sum(sb);
        if (lane == 0) {
            P[(int64_t)t * nwc] = sa;
            if (with_z) P[(int64_t)(k + 1 + t) * nwc] = sb;
        }
    }
}

// sum over the work-group of one value per thread, in a fixed order (waves' sums in order)
__device__ inline double block_sum256(double x, double* red) {
    x = wave_sum(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// One work-group per direction: column k-1 of H (k >= 1), column k of S (with z, S != NULL), and with
// z gamma and 1 / rho. Without z (the last step) u is the unnormalised p, whose dots are scaled by
// inv_h = 1 / nu.
__global__ void __launch_bounds__(256) ms_dcgs_coeff_kernel(const int* __restrict__ dirs, int k, int with_z, int m,
                                                            const double* __restrict__ dots, int ps,
                                                            double* __restrict__ hp, double* __restrict__ H,
                                                            double* __restrict__ Sm, const double* __restrict__ nu,
                                                            const double* __restrict__ inv_h, double* __restrict__ gam,
                                                            double* __restrict__ inv_rho) {
    __shared__ double red[4];
    const int d = dirs[blockIdx.x];
    const int tid = threadIdx.x;
    const double* dt = dots + (int64_t)d * ps;
    double* hpd = hp + (int64_t)d * (m + 1);
    const double sc = with_z ? 1.0 : inv_h[d];
    double asq = 0.0;
    for (int i = tid; i < k; i += 256) {
        const double ai = sc * dt[i];
        asq += ai * ai;
    }
    asq = block_sum256(asq, red);
    const double r2 = dt[k] * sc * sc - asq;
    const double rho = r2 > 0.0 ? sqrt(r2) : 0.0;
    const double nud = nu[d];
    if (k >= 1) {
        double* col = H + ((int64_t)d * m + (k - 1)) * (m + 1);
        for (int i = tid; i < k; i += 256) col[i] = hpd[i] + nud * sc * dt[i];
        if (tid == 0) col[k] = nud * rho;
    }
    if (!with_z) return;
    if (Sm) {
        double* sk = Sm + ((int64_t)d * m + k) * (m + 1);
        for (int i = tid; i < k; i += 256) sk[i] = dt[i];
        if (tid == 0) sk[k] = rho;
    }
    double ab = 0.0;
    for (int i = tid; i < k; i += 256) ab += dt[i] * dt[k + 1 + i];
    ab = block_sum256(ab, red);
    const double ir = rho > 0.0 ? 1.0 / rho : 0.0;
    if (tid == 0) {
        gam[d] = (dt[2 * k + 1] - ab) * ir;
        inv_rho[d] = ir;
    }
}

// The next column's first-pass coefficients, hp(i) = (b_i - (Hbar a)_i) / rho for i < k and
// hp(k) = (gamma - H(k, k-1) a_{k-1}) / rho, after column k-1 of H is complete. One work-group of
// 16 waves per (64 rows, direction): lane = row, wave w adds the columns c = w, w + 16, ... (Hbar is
// upper Hessenberg: c >= i - 1 only), and the 16 partial sums are added in order.
__global__ void __launch_bounds__(1024) ms_dcgs_hp_kernel(const int* __restrict__ dirs, int k, int m,
                                                          const double* __restrict__ dots, int ps,
                                                          const double* __restrict__ H, const double* __restrict__ gam,
                                                          const double* __restrict__ inv_rho, double* __restrict__ hp) {
    __shared__ double red[16][64];
    const int d = dirs[blockIdx.y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const double* dt = dots + (int64_t)d * ps;
    const double* Hd = H + (int64_t)d * m * (m + 1);
    const int c0 = max(0, (int)blockIdx.x * 64 - 1);
    double acc = 0.0;
    if (i < k) {
#pragma unroll 4
        for (int c = c0 + wave; c < k; c += 16)
            if (c >= i - 1) acc += Hd[(int64_t)c * (m + 1) + i] * dt[c];
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && i <= k) {
        const double ir = inv_rho[d];
        double* hpd = hp + (int64_t)d * (m + 1);
        if (i < k) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < 16; ++w) s += red[w][lane];
            hpd[i] = (dt[k + 1 + i] - s) * ir;
        } else {
            const double last = k >= 1 ? Hd[(int64_t)(k - 1) * (m + 1) + k] * dt[k - 1] : 0.0;
            hpd[k] = (gam[d] - last) * ir;
        }
    }
}

// q_k = (u - Q a) / rho into slot k and p' = (z - Q b - gamma q_k) / rho into slot k + 1, with the
// sums of p'^2 over 64-row blocks in norm[d][blk]. A work-group owns 256 rows (4 per lane); its 4
// waves take every 4th basis vector (both sums from one read) and are combined in LDS in a fixed
// order. Rows past n (below npad) are read but neither written nor counted in the norm.
__global__ void __launch_bounds__(256) ms_dcgs_update_kernel(double* __restrict__ V, int64_t n, int64_t npad,
                                                             int mdim1, int k, const int* __restrict__ dirs,
                                                             const double* __restrict__ dots, int ps,
                                                             const double* __restrict__ gam,
                                                             const double* __restrict__ inv_rho,
                                                             double* __restrict__ norm) {
    __shared__ double pa[4][256], pb[4][256];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * 256;   // npad is a multiple of 256
    const int d = dirs[blockIdx.y];
    const double* dt = dots + (int64_t)d * ps;
    double sa[4] = {0.0, 0.0, 0.0, 0.0}, sb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int i = q; i < k; i += 4) {
        const double* v = V + ((int64_t)d * mdim1 + i) * npad + base + lane;
        const double ai = dt[i], bi = dt[k + 1 + i];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double x = v[64 * r];
            sa[r] += ai * x;
            sb[r] += bi * x;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        pa[q][lane + 64 * r] = sa[r];
        pb[q][lane + 64 * r] = sb[r];
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t row = base + t;
    double* u = V + ((int64_t)d * mdim1 + k) * npad;
    double* zv = u + npad;
    double x = 0.0;
    if (row < n) {
        const double ir = inv_rho[d], g = gam[d];
        const double qk = (u[row] - ((pa[0][t] + pa[1][t]) + (pa[2][t] + pa[3][t]))) * ir;
        x = (zv[row] - ((pb[0][t] + pb[1][t]) + (pb[2][t] + pb[3][t])) - g * qk) * ir;
        u[row] = qk;
        zv[row] = x;
    }
    const double s2 = wave_sum(x * x);
    if (lane == 0) norm[(int64_t)d * (npad / kMsRows) + (base / kMsRows) + q] = s2;
}

// nu[d] = |p'| from the block sums (two waves, fixed order), inv_h[d] = 1 / nu[d] (0 when p' = 0)
__global__ void __launch_bounds__(128) ms_nu_kernel(const int* __restrict__ dirs, const double* __restrict__ norm,
                                                    int64_t nblk, double* __restrict__ nu,
                                                    double* __restrict__ inv_h) {
    __shared__ double sh[2];
    const int d = dirs[blockIdx.x];
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < nblk; q += 128) s += norm[(int64_t)d * nblk + q];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double v = sqrt(sh[0] + sh[1]);
        nu[d] = v;
        inv_h[d] = v > 0.0 ? 1.0 / v : 0.0;
    }
}

// y[s] <- S^-1 y[s] over the first k[s] entries (S of the system's direction; column-oriented back
// substitution, y kept in LDS), one work-group per system
__global__ void __launch_bounds__(256) ms_sinv_kernel(const int* __restrict__ sys, const int* __restrict__ ksteps,
                                                      int m, const double* __restrict__ Sm,
                                                      const int* __restrict__ sdir, double2* __restrict__ y) {
    extern __shared__ double2 ys[];
    const int s = sys[blockIdx.x];
    const int K = ksteps[s];
    const double* Sd = Sm + (int64_t)sdir[s] * m * (m + 1);
    for (int i = threadIdx.x; i < K; i += blockDim.x) ys[i] = y[(int64_t)s * m + i];
    __syncthreads();
    for (int i = K - 1; i >= 0; --i) {
        const double* col = Sd + (int64_t)i * (m + 1);
        const double2 yi = cscale(1.0 / col[i], ys[i]);
        __syncthreads();
        if (threadIdx.x == 0) ys[i] = yi;
        for (int r = threadIdx.x; r < i; r += blockDim.x) ys[r] = csub(ys[r], cscale(col[r], yi));
        __syncthreads();
    }
    for (int i = threadIdx.x; i < K; i += blockDim.x) y[(int64_t)s * m + i] = ys[i];
}

// One Givens step of system s on column j of Hbar + z Ibar (direction sdir[s], shift z[s]): the
// rotations of the earlier steps are applied, a new rotation zeroes the subdiagonal, the rotated
// column is stored as column j of R, and |g_{j+1}| is the residual norm of the shifted system.
// One wave per system. Applying rotation i maps the running entry affinely,
// cur' = -conj(s_i) cur + c_i y_{i+1}, and emits c_i cur + s_i y_{i+1}: each lane composes the maps
// of a contiguous chunk of the rotations, an inclusive scan across the lanes gives every chunk its
// incoming entry, and the lanes then replay their chunks to emit the rotated entries (about
// 2 j / 64 + 6 dependent steps instead of j).
__global__ void __launch_bounds__(64) ms_givens_kernel(const int* __restrict__ sys, int nsys, int j, int m,
                                                       const int* __restrict__ sdir, const double2* __restrict__ z,
                                                       const double* __restrict__ H, double* __restrict__ cs,
                                                       double2* __restrict__ sn, double2* __restrict__ g,
                                                       double2* __restrict__ R, int64_t S, double* __restrict__ est,
                                                       const double* __restrict__ tol_abs, int* __restrict__ flags,
                                                       int* __restrict__ run, int* __restrict__ ksteps) {
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const int s = sys[k];
    if (!run[s]) return;   // stopped earlier in this chunk of steps (uniform over the wave)
    const double* hc = H + ((int64_t)sdir[s] * m + j) * (m + 1);
    double2* col = R + ((int64_t)j * (j + 1) / 2) * S + s;   // entry i of the column at col[i * S]
    const double2 zs = z[s];
    auto yv = [&](int i) {   // entry i + 1 of column j of Hbar + z Ibar
        return make_double2(hc[i + 1] + (i + 1 == j ? zs.x : 0.0), i + 1 == j ? zs.y : 0.0);
    };
    const int L = (j + 63) / 64;
    const int i0 = min(j, lane * L), i1 = min(j, i0 + L);
    // the chunk's map: cur_out = A cur_in + B
    double2 A = make_double2(1.0, 0.0), B = make_double2(0.0, 0.0);
    for (int i = i0; i < i1; ++i) {
        const double2 a = cscale(-1.0, cconj(sn[(int64_t)i * S + s]));
        A = cmul(a, A);
        B = cadd(cmul(a, B), cscale(cs[(int64_t)i * S + s], yv(i)));
    }
    // inclusive scan of the maps over the lanes (lane l: the maps of chunks 0 .. l, applied in order)
    for (int off = 1; off < 64; off <<= 1) {
        const double2 Ap = make_double2(__shfl_up(A.x, off, 64), __shfl_up(A.y, off, 64));
        const double2 Bp = make_double2(__shfl_up(B.x, off, 64), __shfl_up(B.y, off, 64));
        if (lane >= off) {
            B = cadd(cmul(A, Bp), B);
            A = cmul(A, Ap);
        }
    }
    const double2 cur0 = make_double2(hc[0] + (j == 0 ? zs.x : 0.0), j == 0 ? zs.y : 0.0);
    double2 Ae = make_double2(__shfl_up(A.x, 1, 64), __shfl_up(A.y, 1, 64));
    double2 Be = make_double2(__shfl_up(B.x, 1, 64), __shfl_up(B.y, 1, 64));
    if (lane == 0) {
        Ae = make_double2(1.0, 0.0);
        Be = make_double2(0.0, 0.0);
    }
    double2 cur = cadd(cmul(Ae, cur0), Be);
    for (int i = i0; i < i1; ++i) {
        const double2 y = yv(i);
        const double ci = cs[(int64_t)i * S + s];
        const double2 si = sn[(int64_t)i * S + s];
        col[(int64_t)i * S] = cadd(cscale(ci, cur), cmul(si, y));
        cur = cadd(cscale(-1.0, cmul(cconj(si), cur)), cscale(ci, y));
    }
    // entry j after every earlier rotation: the whole composition applied to the first entry
    const double2 At = make_double2(__shfl(A.x, 63, 64), __shfl(A.y, 63, 64));
    const double2 Bt = make_double2(__shfl(B.x, 63, 64), __shfl(B.y, 63, 64));
    if (lane != 0) return;
    const double hn = hc[j + 1];
    const double2 x = cadd(cmul(At, cur0), Bt);
    // rotation [c s; -conj(s) c] with c real zeroing hn below col[j]
    const double ax = cabs(x);
    double c;
    double2 sv;
    if (hn == 0.0) {
        c = 1.0;
        sv = make_double2(0.0, 0.0);
    } else if (ax == 0.0) {
        c = 0.0;
        sv = make_double2(1.0, 0.0);
    } else {
        const double nu = hypot(ax, hn);
        c = ax / nu;
        sv = make_double2(x.x / ax * hn / nu, x.y / ax * hn / nu);
    }
    cs[(int64_t)j * S + s] = c;
    sn[(int64_t)j * S + s] = sv;
    const double2 cj = cadd(cscale(c, x), cscale(hn, sv));
    col[(int64_t)j * S] = cj;
    const double2 gj = g[(int64_t)j * S + s];
    const double2 gn = cscale(-1.0, cmul(cconj(sv), gj));
    g[(int64_t)(j + 1) * S + s] = gn;
    g[(int64_t)j * S + s] = cscale(c, gj);
    const double e = cabs(gn);
    est[s] = e;
    int f = 0;
    if (e <= tol_abs[s]) f |= 1;
    if (hn <= 1e-14 * cabs(cj)) f |= 2;   // the Krylov space is invariant: the iterate is exact
    if (!(e == e) || !(hn == hn)) f |= 4;
    flags[s] = f;
    ksteps[s] = j + 1;
    if (f) run[s] = 0;
}

// y = R^-1 g over the first k[s] columns, one work-group per system: column-oriented back
// substitution on the packed R (entry i of column c at ((c (c + 1) / 2) + i) S + s), y kept in LDS;
__global__ void __launch_bounds__(256) ms_solve_kernel(const int* __restrict__ sys, const int* __restrict__ ksteps,
                                                       int m, const double2* __restrict__ R, int64_t S,
                                                       const double2* __restrict__ g, double2* __restrict__ y) {
    extern __shared__ double2 ys[];
    const int s = sys[blockIdx.x];
    const int K = ksteps[s];
    auto rat = [&](int c, int i) { return R[((int64_t)c * (c + 1) / 2 + i) * S + s]; };
    for (int i = threadIdx.x; i < K; i += blockDim.x) ys[i] = g[(int64_t)i * S + s];
    __syncthreads();
    for (int i = K - 1; i >= 0; --i) {
        const double2 yi = cdiv(ys[i], rat(i, i));   // every thread computes it; ys[i] is final here
        __syncthreads();
        if (threadIdx.x == 0) ys[i] = yi;
        for (int r = threadIdx.x; r < i; r += blockDim.x) ys[r] = csub(ys[r], cmul(rat(i, r), yi));
        __syncthreads();
    }
    for (int i = threadIdx.x; i < K; i += blockDim.x) y[(int64_t)s * m + i] = ys[i];
}

// x(s) = sum_{i < k[s]} y[s][i] V(d, i) for groups of up to 8 systems of one direction (the basis
// is read once per group); rows >= n and systems with k = 0 get 0. Real part at out + col sys_stride,
// imaginary part im_off further, with col = pos[s] (skipped when negative) or s when pos is NULL.
__global__ void __launch_bounds__(256) ms_xupdate_kernel(const double* __restrict__ V, int64_t n, int64_t npad,
                                                         int mdim1, const int* __restrict__ grp_sys,
                                                         const int* __restrict__ grp_dir, const int* __restrict__ ksteps,
                                                         const double2* __restrict__ y, int m,
                                                         double* __restrict__ out, int64_t sys_stride, int64_t im_off,
                                                         const int* __restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int gi = blockIdx.y;
    const int d = grp_dir[gi];
    int sid[kMsGroup], kk[kMsGroup];
    int kmax = 0;
#pragma unroll
    for (int t = 0; t < kMsGroup; ++t) {
        sid[t] = grp_sys[gi * kMsGroup + t];
        kk[t] = sid[t] >= 0 ? ksteps[sid[t]] : 0;
        kmax = max(kmax, kk[t]);
    }
    double ar[kMsGroup], ai[kMsGroup];
#pragma unroll
    for (int t = 0; t < kMsGroup; ++t) ar[t] = ai[t] = 0.0;
    if (i < n) {
        for (int c = 0; c < kmax; ++c) {
            const double v = V[((int64_t)d * mdim1 + c) * npad + i];
#pragma unroll
            for (int t = 0; t < kMsGroup; ++t)
                if (c < kk[t]) {
                    const double2 yc = y[(int64_t)sid[t] * m + c];
                    ar[t] += yc.x * v;
                    ai[t] += yc.y * v;
                }
        }
    }
#pragma unroll
    for (int t = 0; t < kMsGroup; ++t) {
        const int col = sid[t] < 0 ? -1 : pos ? pos[sid[t]] : sid[t];
        if (col >= 0) {
            double* xr = out + (int64_t)col * sys_stride;
            xr[i] = ar[t];
            xr[i + im_off] = ai[t];
        }
    }
}

}  // namespace

void ms_pack(int prec, double* V, int64_t npad, int mdim1, int j, const int* dirs, int ndir, const double* scale,
             void* X, int64_t ld, hipStream_t st) {
    if (ndir <= 0) return;
    dim3 grd((unsigned)(npad / 256), (unsigned)ndir);
    if (prec == WFQ_PREC_FP64)
        hipLaunchKernelGGL(ms_pack_kernel<double>, grd, dim3(256), 0, st, V, npad, mdim1, j, dirs, scale,
                           static_cast<double*>(X), ld);
    else if (prec == WFQ_PREC_FP32)
        hipLaunchKernelGGL(ms_pack_kernel<float>, grd, dim3(256), 0, st, V, npad, mdim1, j, dirs, scale,
                           static_cast<float*>(X), ld);
    else
        hipLaunchKernelGGL(ms_pack_kernel<uint16_t>, grd, dim3(256), 0, st, V, npad, mdim1, j, dirs, scale,
                           static_cast<uint16_t*>(X), ld);
    WFQ_CHECK_LAUNCH();
}

void ms_spmm(const Structure& S, bool y_is_f64, const void* Y, int64_t ld, const int* dirs, int ndir, double* V,
             int mdim1, int jdst, double* TV, hipStream_t st, const double* Yi) {
    if (ndir <= 0) return;
    if (Yi && (!y_is_f64 || ndir > 4)) throw Error{WFQ_EINVAL, "ms_spmm: the interleaved copy holds up to 4 FP64 columns"};
    const dim3 grd((unsigned)(S.npad / 256));
    // columns in chunks of at most 4 (3 for the usual three field directions in one pass)
    for (int c0 = 0; c0 < ndir; c0 += 4) {
        const int nc = std::min(4, ndir - c0);
        auto go = [&](auto tag, auto ncv) {
            using YE = decltype(tag);
            constexpr int NC = decltype(ncv)::value;
            hipLaunchKernelGGL((ms_spmm_kernel<YE, NC>), grd, dim3(256), 0, st, S.n, S.npad, S.ell_w, S.ell_col,
                               S.ell_val, static_cast<const YE*>(Y), ld, dirs, V, mdim1, jdst, c0, TV, Yi);
        };
        auto by_nc = [&](auto tag) {
            if (nc == 1) go(tag, std::integral_constant<int, 1>{});
            else if (nc == 2) go(tag, std::integral_constant<int, 2>{});
            else if (nc == 3) go(tag, std::integral_constant<int, 3>{});
            else go(tag, std::integral_constant<int, 4>{});
        };
        if (y_is_f64)
            by_nc(double{});
        else
            by_nc(float{});
        WFQ_CHECK_LAUNCH();
    }
}

void ms_dot(const double* V, int64_t n, int64_t npad, int mdim1, int nvec, int jw, const int* dirs, int ndir,
            double* partial, int pslots, bool self_norm, hipStream_t st) {
    const int ntot = nvec + (self_norm ? 1 : 0);
    if (ndir <= 0 || ntot <= 0) return;
    const int64_t nwc = wave_chunks(n);
    dim3 grd((unsigned)nwc, (unsigned)((ntot + 3) / 4), (unsigned)ndir);
    hipLaunchKernelGGL(ms_dot_kernel, grd, dim3(256), 0, st, V, n, npad, mdim1, nvec, jw, dirs, partial, pslots, nwc,
                       (int)self_norm);
    WFQ_CHECK_LAUNCH();
}

void ms_reduce(const int* dirs, int ndir, const double* partial, int pslots, int64_t n, int count, double* h,
               hipStream_t st) {
    if (ndir <= 0 || count <= 0) return;
    hipLaunchKernelGGL(ms_reduce_kernel, dim3((unsigned)((count + 3) / 4), (unsigned)ndir), dim3(256), 0, st, dirs,
                       partial, pslots, wave_chunks(n), count, h);
    WFQ_CHECK_LAUNCH();
}

void ms_update(double* V, int64_t n, int64_t npad, int mdim1, int nvec, int jw, const int* dirs, int ndir,
               const double* h, int pslots, double* norm, hipStream_t st) {
    if (ndir <= 0) return;
    dim3 grd((unsigned)(npad / kMsRows), (unsigned)ndir);
    hipLaunchKernelGGL(ms_update_kernel, grd, dim3(256), 0, st, V, n, npad, mdim1, nvec, jw, dirs, h, pslots, norm);
    WFQ_CHECK_LAUNCH();
}

void ms_givens(const int* sys, int nsys, int j, int m, const int* sdir, const double2* z, const double* H, double* cs,
               double2* sn, double2* g, double2* R, int64_t S, double* est, const double* tol_abs, int* flags,
               int* run, int* ksteps, hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(ms_givens_kernel, dim3((unsigned)nsys), dim3(64), 0, st, sys, nsys, j, m, sdir, z, H, cs, sn, g,
                       R, S, est, tol_abs, flags, run, ksteps);
    WFQ_CHECK_LAUNCH();
}

void ms_dcgs_dot(const double* V, int64_t n, int64_t npad, int mdim1, int k, bool with_z, const int* dirs, int ndir,
                 double* partial, int ps, hipStream_t st) {
    if (ndir <= 0) return;
    if (2 * k + 2 > ps) throw Error{WFQ_EINVAL, "ms_dcgs_dot: too few partial slots"};
    const int64_t nwc = wave_chunks(n);
    dim3 grd((unsigned)((nwc + 3) / 4), (unsigned)(k / kDotGroup + 1), (unsigned)ndir);
    hipLaunchKernelGGL(ms_dcgs_dot_kernel, grd, dim3(256), 0, st, V, n, npad, mdim1, k, with_z ? 1 : 0, dirs, partial,
                       ps, nwc);
    WFQ_CHECK_LAUNCH();
}

void ms_dcgs_coeff(const int* dirs, int ndir, int k, bool with_z, int m, const double* dots, int ps, double* hp,
                   double* H, double* Sm, const double* nu, const double* inv_h, double* gam, double* inv_rho,
                   hipStream_t st) {
    if (ndir <= 0) return;
    hipLaunchKernelGGL(ms_dcgs_coeff_kernel, dim3((unsigned)ndir), dim3(256), 0, st, dirs, k, with_z ? 1 : 0, m, dots,
                       ps, hp, H, Sm, nu, inv_h, gam, inv_rho);
    WFQ_CHECK_LAUNCH();
    if (!with_z) return;
    hipLaunchKernelGGL(ms_dcgs_hp_kernel, dim3((unsigned)(k / 64 + 1), (unsigned)ndir), dim3(1024), 0, st, dirs, k, m,
                       dots, ps, H, gam, inv_rho, hp);
    WFQ_CHECK_LAUNCH();
}

void ms_dcgs_update(double* V, int64_t n, int64_t npad, int mdim1, int k, const int* dirs, int ndir,
                    const double* dots, int ps, const double* gam, const double* inv_rho, double* norm,
                    double* nu, double* inv_h, hipStream_t st) {
    if (ndir <= 0) return;
    dim3 grd((unsigned)(npad / 256), (unsigned)ndir);
    hipLaunchKernelGGL(ms_dcgs_update_kernel, grd, dim3(256), 0, st, V, n, npad, mdim1, k, dirs, dots, ps, gam, inv_rho,
                       norm);
    WFQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(ms_nu_kernel, dim3((unsigned)ndir), dim3(128), 0, st, dirs, norm, npad / kMsRows, nu, inv_h);
    WFQ_CHECK_LAUNCH();
}

void ms_sinv(const int* sys, int nsys, const int* ksteps, int m, const double* Sm, const int* sdir, double2* y,
             hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(ms_sinv_kernel, dim3((unsigned)nsys), dim3(256), (size_t)m * sizeof(double2), st, sys, ksteps,
                       m, Sm, sdir, y);
    WFQ_CHECK_LAUNCH();
}

void ms_solve(const int* sys, int nsys, const int* ksteps, int m, const double2* R, int64_t S, const double2* g,
              double2* y, hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(ms_solve_kernel, dim3((unsigned)nsys), dim3(256), (size_t)m * sizeof(double2), st, sys, ksteps,
                       m, R, S, g, y);
    WFQ_CHECK_LAUNCH();
}

void ms_xupdate(const double* V, int64_t n, int64_t npad, int mdim1, const int* grp_sys, const int* grp_dir, int ngrp,
                const int* ksteps, const double2* y, int m, const Basis& X, hipStream_t st) {
    if (ngrp <= 0) return;
    dim3 grd((unsigned)(npad / 256), (unsigned)ngrp);
    hipLaunchKernelGGL(ms_xupdate_kernel, grd, dim3(256), 0, st, V, n, npad, mdim1, grp_sys, grp_dir, ksteps, y, m,
                       X.base, X.sys_stride, X.npad, nullptr);
    WFQ_CHECK_LAUNCH();
}

void ms_txupdate(const double* TV, int64_t n, int64_t npad, int mdim1, const int* grp_sys, const int* grp_dir,
                 int ngrp, const int* ksteps, const double2* y, int m, const int* pos, double* Y, int64_t ld,
                 hipStream_t st) {
    if (ngrp <= 0) return;
    if (ld < npad) throw Error{WFQ_EINVAL, "ms_txupdate: leading dimension below the padded length"};
    dim3 grd((unsigned)(npad / 256), (unsigned)ngrp);
    hipLaunchKernelGGL(ms_xupdate_kernel, grd, dim3(256), 0, st, TV, n, npad, mdim1, grp_sys, grp_dir, ksteps, y, m, Y,
                       2 * ld, ld, pos);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
