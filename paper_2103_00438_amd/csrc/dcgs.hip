// Arnoldi orthogonalisation for batched GMRES with one reduction per step: classical Gram-Schmidt
// with delayed reorthogonalisation (DCGS2, Swirydowicz, Langou, Ananthan, Yang and Thomas 2020),
// the low-synchronisation form of the two-pass Gram-Schmidt process that the GMRES paragraph of the
// paper's "Solution strategies" section relies on for the orthonormal Krylov basis.
//
// Step k of a cycle (k = 0 .. m) holds, per system: q_0 .. q_{k-1} final; u (slot k) = the new
// direction after one projection pass, scaled to unit norm; z = A u (slot k + 1, absent at k = m).
// One fused sweep over the basis gives a = Q^H u, alpha = u^H u, b = Q^H z and beta = u^H z. Then
//   rho = sqrt(alpha - |a|^2),  q_k = (u - Q a) / rho                     (second pass of u, delayed)
//   H(0:k, k-1) = hp + nu a,    H(k, k-1) = nu rho                          (column k-1 completed)
//   w' = (z - Q b - q_k gamma) / rho,  gamma = (beta - a^H b) / rho        (first pass of A q_k)
// with hp the first-pass coefficients of the previous step and nu = |w'| of the previous step; the
// first-pass coefficients of A q_k follow from A Q = Q H:
//   hp'(0:k-1) = (b - H(0:k-1, 0:k-1) a) / rho,  hp'(k) = (gamma - nu rho a_{k-1}) / rho.
// A second sweep applies both updates. The basis is read twice per step instead of four times, and
// each cycle applies the operator once more than it has columns (the last product only completes
// the last column). Column k-1 is completed, and its Givens rotation taken, at step k.
#include "device_util.h"
#include "krylov.h"

namespace wfq {

namespace {

__device__ inline double* slot(const Basis& V, int s, int j) {
    return V.base + (int64_t)s * V.sys_stride + (int64_t)j * V.vec_stride;
}
__device__ inline double2 c_mul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 c_conj_mul(double2 a, double2 b) {   // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 c_scale(double c, double2 a) { return make_double2(c * a.x, c * a.y); }
__device__ inline double c_abs(double2 a) { return hypot(a.x, a.y); }

// entry layout of the fused dots of one system (2 mdim slots): t < k: a_t; t = k: alpha;
// k + 1 + t (t < k): b_t; 2 k + 1: beta
__device__ inline int dot_a(int t) { return t; }
__device__ inline int dot_b(int k, int t) { return k + 1 + t; }

// Wide form: one wave per (512-row chunk, system); u and z of the chunk in registers. FULL: every
// row of the chunk is below n (all chunks but the last), so the loads need no per-row guard.
template <bool FULL>
__device__ inline void dot_rows_body(const Basis& V, int64_t n, int s, int k, int with_z, double2* __restrict__ partial,
                                     int pstride, int64_t nwc, int64_t wc, int lane) {
    const double* ur = slot(V, s, k);
    const double* zr = with_z ? slot(V, s, k + 1) : ur;
    const int64_t row0 = wc * kWaveRows + lane;
    double xr[8], xi[8], yr[8], yi[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t row = row0 + 64 * r;
        const bool in = FULL || row < n;
        xr[r] = in ? ur[row] : 0.0;
        xi[r] = in ? ur[row + V.npad] : 0.0;
        yr[r] = (in && with_z) ? zr[row] : 0.0;
        yi[r] = (in && with_z) ? zr[row + V.npad] : 0.0;
    }
    double2* P = partial + (int64_t)s * pstride * nwc + wc;
    // in full chunks the rows of basis vector i + 1 are loaded before the sums of vector i are
    // reduced, so a wave keeps loads in flight across its reductions (rows past n read as zero:
    // same sums)
    double va[8], vb[8];
    auto load_v = [&](int i, double (&ra)[8], double (&rb)[8]) {
        const double* vr = slot(V, s, i);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t row = row0 + 64 * r;
            const bool in = FULL || row < n;
            ra[r] = in ? vr[row] : 0.0;
            rb[r] = in ? vr[row + V.npad] : 0.0;
        }
    };
    if (k > 0) load_v(0, va, vb);
    for (int i = 0; i < k; ++i) {
        double na[8], nb[8];
        if constexpr (FULL) load_v(min(i + 1, k - 1), na, nb);   // the last step re-reads its own vector
        else if (i > 0) load_v(i, va, vb);                       // the tail chunk: no prefetch
        double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const double a = va[r], b = vb[r];
            ar += a * xr[r] + b * xi[r];   // conj(v) u
            ai += a * xi[r] - b * xr[r];
            br += a * yr[r] + b * yi[r];   // conj(v) z
            bi += a * yi[r] - b * yr[r];
        }
        if constexpr (FULL) {
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                va[r] = na[r];
                vb[r] = nb[r];
            }
        }
        ar = wave_sum(ar);
        ai = wave_sum(ai);
        br = wave_sum(br);
        bi = wave_sum(bi);
        if (lane == 0) {
            P[(int64_t)dot_a(i) * nwc] = make_double2(ar, ai);
            if (with_z) P[(int64_t)dot_b(k, i) * nwc] = make_double2(br, bi);
        }
    }
    double al = 0.0, br = 0.0, bi = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        al += xr[r] * xr[r] + xi[r] * xi[r];
        br += xr[r] * yr[r] + xi[r] * yi[r];
        bi += xr[r] * yi[r] - xi[r] * yr[r];
    }
    al = wave_sum(al);
    br = wave_sum(br);
    bi = wave_sum(bi);
    if (lane == 0) {
        P[(int64_t)k * nwc] = make_double2(al, 0.0);
        if (with_z) P[(int64_t)(2 * k + 1) * nwc] = make_double2(br, bi);
    }
}

__global__ void __launch_bounds__(256) dcgs_dot_rows_kernel(Basis V, int64_t n, const int* __restrict__ sys, int k,
                                                       int with_z, double2* __restrict__ partial, int pstride,
                                                       int64_t nwc, const int* __restrict__ run) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wc = (int64_t)blockIdx.x * 4 + wave;
    if (wc >= nwc) return;
    const int s = sys[blockIdx.y];
    if (run && !run[s]) return;
    if ((wc + 1) * kWaveRows <= n)
        dot_rows_body<true>(V, n, s, k, with_z, partial, pstride, nwc, wc, lane);
    else
        dot_rows_body<false>(V, n, s, k, with_z, partial, pstride, nwc, wc, lane);
}

// Narrow form: one wave per (512-row chunk, basis vector t <= k, system), so that a few systems
// still spread over many waves; t = k computes alpha and beta.
__global__ void __launch_bounds__(256) dcgs_dot_kernel(Basis V, int64_t n, const int* __restrict__ sys, int k,
                                                  int with_z, double2* __restrict__ partial, int pstride, int64_t nwc,
                                                  const int* __restrict__ run) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wc = blockIdx.x;
    const int t = blockIdx.y * 4 + wave;
    if (t > k) return;
    const int s = sys[blockIdx.z];
    if (run && !run[s]) return;
    const double* ur = slot(V, s, k);
    const double* zr = with_z ? slot(V, s, k + 1) : ur;
    const double* vr = slot(V, s, t);
    const int64_t row0 = wc * kWaveRows + lane;
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t row = row0 + 64 * r;
        if (row < n) {
            const double a = vr[row], b = vr[row + V.npad];
            const double x = ur[row], y = ur[row + V.npad];
            ar += a * x + b * y;
            ai += a * y - b * x;
            if (with_z) {
                const double p = zr[row], q = zr[row + V.npad];
                br += a * p + b * q;
                bi += a * q - b * p;
            }
        }
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    br = wave_sum(br);
    bi = wave_sum(bi);
    if (lane == 0) {
        double2* P = partial + (int64_t)s * pstride * nwc + wc;
        if (t < k) {
            P[(int64_t)dot_a(t) * nwc] = make_double2(ar, ai);
            if (with_z) P[(int64_t)dot_b(k, t) * nwc] = make_double2(br, bi);
        } else {
            P[(int64_t)k * nwc] = make_double2(ar, 0.0);
            if (with_z) P[(int64_t)(2 * k + 1) * nwc] = make_double2(br, bi);
        }
    }
}

// One wave per system: complete column k-1 of the Hessenberg matrix, rotate it into R, and form the
// coefficients of the update sweep and the first-pass coefficients of the next column.
__global__ void __launch_bounds__(64) dcgs_coeff_kernel(const int* __restrict__ sys, int k, int with_z, int mdim,
                                                        DcgsArgs a) {
    const int s = sys[blockIdx.x];
    const int lane = threadIdx.x;
    if (a.run && !a.run[s]) return;
    const double2* d = a.dots + (int64_t)s * 2 * mdim;
    double2* hp = a.hp + (int64_t)s * mdim;
    double2* Hs = a.H + (int64_t)s * mdim * mdim;   // column-major: Hs[c * mdim + i] = H(i, c)
    // at the last step u is the unnormalised w' (no product was formed to normalise it)
    const double sc = with_z ? 1.0 : a.inv_h[s];
    double asq = 0.0;
    for (int i = lane; i < k; i += 64) {
        const double2 ai = c_scale(sc, d[dot_a(i)]);
        asq += ai.x * ai.x + ai.y * ai.y;
    }
    asq = wave_sum(asq);
    const double alpha = d[k].x * sc * sc;
    const double r2 = alpha - asq;
    const double rho = r2 > 0.0 ? sqrt(r2) : 0.0;
    const double nu = a.nu[s];
    if (k == 0) {
        if (lane == 0) {
            a.flags[s] = 0;
            a.ksteps[s] = 0;
        }
    } else {
        const int c = k - 1;
        double2* col = a.R + ((int64_t)s * mdim + c) * mdim;
        for (int i = lane; i < k; i += 64) {
            const double2 h = c_add(hp[i], c_scale(nu * sc, d[dot_a(i)]));
            Hs[(int64_t)c * mdim + i] = h;
            col[i] = h;
        }
        const double hn = nu * rho;
        if (lane == 0) Hs[(int64_t)c * mdim + k] = make_double2(hn, 0.0);
        __syncthreads();
        if (lane == 0) {
            // previous rotations, then the one that zeroes hn below col[c]: [cs sn; -conj(sn) cs]
            double* cs = a.cs + (int64_t)s * mdim;
            double2* sn = a.sn + (int64_t)s * mdim;
            // the running entry stays in registers; the unrotated entries are loaded ahead of it
            double2 cur = col[0];
            for (int i = 0; i < c; ++i) {
                const double2 y = col[i + 1];
                col[i] = c_add(c_scale(cs[i], cur), c_mul(sn[i], y));
                cur = c_sub(c_scale(cs[i], y), c_conj_mul(sn[i], cur));
            }
            const double2 x = cur;
            const double ax = c_abs(x);
            double cr;
            double2 sv;
            if (hn == 0.0) {
                cr = 1.0;
                sv = make_double2(0.0, 0.0);
            } else if (ax == 0.0) {
                cr = 0.0;
                sv = make_double2(1.0, 0.0);
            } else {
                const double nrm = hypot(ax, hn);
                cr = ax / nrm;
                sv = make_double2(x.x / ax * hn / nrm, x.y / ax * hn / nrm);
            }
            cs[c] = cr;
            sn[c] = sv;
            col[c] = c_add(c_scale(cr, x), c_scale(hn, sv));
            double2* g = a.g + (int64_t)s * (mdim + 1);
            const double2 gc = g[c];
            g[c + 1] = c_scale(-1.0, c_conj_mul(sv, gc));
            g[c] = c_scale(cr, gc);
            const double est = c_abs(g[c + 1]);
            a.est[s] = est;
            int f = 0;
            if (est <= a.tol_abs[s]) f |= 1;
            if (hn <= 1e-14 * c_abs(col[c])) f |= 2;
            if (!(est == est) || !(hn == hn) || !(rho == rho)) f |= 4;
            a.flags[s] = f;
            a.ksteps[s] = k;
            if (f && a.run) a.run[s] = 0;
        }
    }
    if (!with_z) return;
    // gamma = (beta - a^H b) / rho and the next column's first-pass coefficients
    double2 ab = make_double2(0.0, 0.0);
    for (int i = lane; i < k; i += 64) ab = c_add(ab, c_conj_mul(d[dot_a(i)], d[dot_b(k, i)]));
    ab.x = wave_sum(ab.x);
    ab.y = wave_sum(ab.y);
    const double ir = rho > 0.0 ? 1.0 / rho : 0.0;
    const double2 gamma = c_scale(ir, c_sub(d[2 * k + 1], ab));
    __syncthreads();   // column k-1 of H is complete
    for (int i = lane; i < k; i += 64) {
        // (H(0:k-1, 0:k-1) a)_i: H is upper Hessenberg, so columns c >= i - 1 only
        double2 acc = make_double2(0.0, 0.0);
        for (int c = (i > 0 ? i - 1 : 0); c < k; ++c) acc = c_add(acc, c_mul(Hs[(int64_t)c * mdim + i], d[dot_a(c)]));
        hp[i] = c_scale(ir, c_sub(d[dot_b(k, i)], acc));
    }
    if (lane == 0) {
        const double2 last = k > 0 ? c_scale(nu * rho, d[dot_a(k - 1)]) : make_double2(0.0, 0.0);
        hp[k] = c_scale(ir, c_sub(gamma, last));
        a.gamma[s] = gamma;
        a.inv_rho[s] = ir;
    }
}

// Wide update: one wave per (512-row chunk, system): q_k = (u - Q a) / rho into slot k and
// w' = (z - Q b - q_k gamma) / rho into slot k + 1, with the chunk's |w'|^2. FULL: every row of the chunk is
// below n (all chunks but the last).
template <bool FULL>
__device__ inline void update_rows_body(const Basis& V, int64_t n, int s, int k, int mdim, const DcgsArgs& a,
                                        int64_t nwc, int64_t wc, int lane) {
    double* ur = slot(V, s, k);
    double* zr = slot(V, s, k + 1);
    const int64_t row0 = wc * kWaveRows + lane;
    double xr[8], xi[8], yr[8], yi[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t row = row0 + 64 * r;
        const bool in = FULL || row < n;
        xr[r] = in ? ur[row] : 0.0;
        xi[r] = in ? ur[row + V.npad] : 0.0;
        yr[r] = in ? zr[row] : 0.0;
        yi[r] = in ? zr[row + V.npad] : 0.0;
    }
    const double2* d = a.dots + (int64_t)s * 2 * mdim;
    // in full chunks the rows of basis vector i + 1 are loaded while vector i is applied (rows past
    // n read as zero and are not stored)
    double va[8], vb[8];
    auto load_v = [&](int i, double (&ra)[8], double (&rb)[8]) {
        const double* vr = slot(V, s, i);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t row = row0 + 64 * r;
            const bool in = FULL || row < n;
            ra[r] = in ? vr[row] : 0.0;
            rb[r] = in ? vr[row + V.npad] : 0.0;
        }
    };
    if (k > 0) load_v(0, va, vb);
    for (int i = 0; i < k; ++i) {
        double na[8], nb[8];
        if constexpr (FULL) load_v(min(i + 1, k - 1), na, nb);   // the last step re-reads its own vector
        else if (i > 0) load_v(i, va, vb);                       // the tail chunk: no prefetch
        const double2 ca = d[dot_a(i)], cb = d[dot_b(k, i)];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const double p = va[r], q = vb[r];
            xr[r] -= ca.x * p - ca.y * q;
            xi[r] -= ca.x * q + ca.y * p;
            yr[r] -= cb.x * p - cb.y * q;
            yi[r] -= cb.x * q + cb.y * p;
            if constexpr (FULL) {
                va[r] = na[r];
                vb[r] = nb[r];
            }
        }
    }
    const double ir = a.inv_rho[s];
    const double2 gm = a.gamma[s];
    double nn = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t row = row0 + 64 * r;
        if (FULL || row < n) {
            const double qr = xr[r] * ir, qi = xi[r] * ir;
            const double wr = (yr[r] - (gm.x * qr - gm.y * qi)) * ir;
            const double wi = (yi[r] - (gm.x * qi + gm.y * qr)) * ir;
            ur[row] = qr;
            ur[row + V.npad] = qi;
            zr[row] = wr;
            zr[row + V.npad] = wi;
            nn += wr * wr + wi * wi;
        }
    }
    nn = wave_sum(nn);
    if (lane == 0) a.norm2[(int64_t)s * nwc + wc] = nn;
}

__global__ void __launch_bounds__(256) dcgs_update_rows_kernel(Basis V, int64_t n, const int* __restrict__ sys, int k,
                                                          int mdim, DcgsArgs a, int64_t nwc) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wc = (int64_t)blockIdx.x * 4 + wave;
    if (wc >= nwc) return;
    const int s = sys[blockIdx.y];
    if (a.run && !a.run[s]) return;
    if ((wc + 1) * kWaveRows <= n)
        update_rows_body<true>(V, n, s, k, mdim, a, nwc, wc, lane);
    else
        update_rows_body<false>(V, n, s, k, mdim, a, nwc, wc, lane);
}

// Narrow update: one 512-row chunk per work-group; each of the 4 waves sums every 4th basis vector
// over the whole chunk, and the partial sums meet in LDS in a fixed order.
__global__ void __launch_bounds__(256) dcgs_update_kernel(Basis V, int64_t n, const int* __restrict__ sys, int k,
                                                     int mdim, DcgsArgs a, int64_t nwc) {
    __shared__ double part[2][4][kWaveRows];   // (re, im) per wave: Q a first, then Q b
    __shared__ double red[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wc = blockIdx.x;
    const int s = sys[blockIdx.y];
    if (a.run && !a.run[s]) return;   // whole work-group
    const int64_t row0 = wc * kWaveRows;
    const double2* d = a.dots + (int64_t)s * 2 * mdim;
    double sar[8], sai[8], sbr[8], sbi[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) sar[r] = sai[r] = sbr[r] = sbi[r] = 0.0;
    for (int i = wave; i < k; i += 4) {
        const double2 ca = d[dot_a(i)], cb = d[dot_b(k, i)];
        const double* vr = slot(V, s, i);
        const double* vi = vr + V.npad;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t row = row0 + lane + 64 * r;
            if (row < n) {
                const double p = vr[row], q = vi[row];
                sar[r] += ca.x * p - ca.y * q;
                sai[r] += ca.x * q + ca.y * p;
                sbr[r] += cb.x * p - cb.y * q;
                sbi[r] += cb.x * q + cb.y * p;
            }
        }
    }
    // combine the four waves' sums for the two rows each thread finishes, Q a then Q b
    double qa[2][2], qb[2][2];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        part[0][wave][lane + 64 * r] = sar[r];
        part[1][wave][lane + 64 * r] = sai[r];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int q = threadIdx.x + 256 * t;
#pragma unroll
        for (int c = 0; c < 2; ++c) qa[t][c] = (part[c][0][q] + part[c][1][q]) + (part[c][2][q] + part[c][3][q]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        part[0][wave][lane + 64 * r] = sbr[r];
        part[1][wave][lane + 64 * r] = sbi[r];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int q = threadIdx.x + 256 * t;
#pragma unroll
        for (int c = 0; c < 2; ++c) qb[t][c] = (part[c][0][q] + part[c][1][q]) + (part[c][2][q] + part[c][3][q]);
    }
    double* ur = slot(V, s, k);
    double* zr = slot(V, s, k + 1);
    const double ir = a.inv_rho[s];
    const double2 gm = a.gamma[s];
    double nn = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int64_t row = row0 + threadIdx.x + 256 * t;
        if (row < n) {
            const double qr = (ur[row] - qa[t][0]) * ir, qi = (ur[row + V.npad] - qa[t][1]) * ir;
            const double wr = (zr[row] - qb[t][0] - (gm.x * qr - gm.y * qi)) * ir;
            const double wi = (zr[row + V.npad] - qb[t][1] - (gm.x * qi + gm.y * qr)) * ir;
            ur[row] = qr;
            ur[row + V.npad] = qi;
            zr[row] = wr;
            zr[row + V.npad] = wi;
            nn += wr * wr + wi * wi;
        }
    }
    nn = wave_sum(nn);
    if (lane == 0) red[wave] = nn;
    __syncthreads();
    if (threadIdx.x == 0) a.norm2[(int64_t)s * nwc + wc] = (red[0] + red[1]) + (red[2] + red[3]);
}

// nu = |w'| from the chunk partials (fixed order); the next step's product is taken of w' / nu
__global__ void dcgs_nu_kernel(const int* __restrict__ sys, int nsys, DcgsArgs a, int64_t nwc) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nsys) return;
    const int s = sys[q];
    if (a.run && !a.run[s]) return;
    double acc = 0.0;
    for (int64_t w = 0; w < nwc; ++w) acc += a.norm2[(int64_t)s * nwc + w];
    const double nu = sqrt(acc);
    a.nu[s] = nu;
    a.inv_h[s] = nu > 0.0 ? 1.0 / nu : 0.0;
}

// chunks x systems from which the one-wave-per-(chunk, system) forms fill the chip
constexpr int64_t kWideDcgs = 4096;

}  // namespace

void dcgs_dots(const Basis& V, int64_t n, const int* sys, int nsys, int k, bool with_z, double2* partial, int mdim,
               const int* run, hipStream_t st) {
    if (nsys <= 0) return;
    const int64_t nwc = wave_chunks(n);
    const int pstride = 2 * mdim;
    if (nwc * nsys >= kWideDcgs) {
        dim3 grd((unsigned)((nwc + 3) / 4), (unsigned)nsys);
        hipLaunchKernelGGL(dcgs_dot_rows_kernel, grd, dim3(256), 0, st, V, n, sys, k, (int)with_z, partial, pstride,
                           nwc, run);
    } else {
        dim3 grd((unsigned)nwc, (unsigned)((k + 1 + 3) / 4), (unsigned)nsys);
        hipLaunchKernelGGL(dcgs_dot_kernel, grd, dim3(256), 0, st, V, n, sys, k, (int)with_z, partial, pstride, nwc,
                           run);
    }
    WFQ_CHECK_LAUNCH();
}

void dcgs_coeff(const int* sys, int nsys, int k, bool with_z, int mdim, const DcgsArgs& a, hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(dcgs_coeff_kernel, dim3(nsys), dim3(64), 0, st, sys, k, (int)with_z, mdim, a);
    WFQ_CHECK_LAUNCH();
}

void dcgs_update(const Basis& V, int64_t n, const int* sys, int nsys, int k, int mdim, const DcgsArgs& a,
                 hipStream_t st) {
    if (nsys <= 0) return;
    const int64_t nwc = wave_chunks(n);
    if (nwc * nsys >= kWideDcgs) {
        dim3 grd((unsigned)((nwc + 3) / 4), (unsigned)nsys);
        hipLaunchKernelGGL(dcgs_update_rows_kernel, grd, dim3(256), 0, st, V, n, sys, k, mdim, a, nwc);
    } else {
        dim3 grd((unsigned)nwc, (unsigned)nsys);
        hipLaunchKernelGGL(dcgs_update_kernel, grd, dim3(256), 0, st, V, n, sys, k, mdim, a, nwc);
    }
    WFQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(dcgs_nu_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, sys, nsys, a, nwc);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
