// Block-Jacobi right preconditioning of the batched GMRES (a project extension: the paper applies
// its Krylov solvers without preconditioning, reports that the diagonal of the matrix did not help,
// and names the missing preconditioner as a bottleneck in its conclusions).
//
// Blocks are 64 consecutive atoms of the internal, spatially sorted order. For block b the
// frequency-independent part is C_b = (L T)_bb, C_b[r][c] = sum_k L_{ik} T_{kj} (i = 64 b + r,
// j = 64 b + c); for system s the block of the operator is C_b + z_s I, inverted once per solve by
// Gauss-Jordan elimination with partial pivoting in LDS. GMRES then runs on (L T + z I) M^-1 with
// the true residual; the product input is u = M^-1 v (block by block), and the iterate update is
// x += M^-1 (V y). Padding atoms have zero rows and columns in C, so their diagonal is z and the
// padding of every vector stays zero.
#include "device_util.h"
#include "krylov.h"

namespace wfq {

namespace {

constexpr int kB = 64;   // atoms per block

__device__ inline double* vslot(const Basis& V, int s, int j) {
    return V.base + (int64_t)s * V.sys_stride + (int64_t)j * V.vec_stride;
}

// C_b, one work-group per block: thread (row r = tid / 4, quarter q = tid % 4) forms the 16 entries
// C_b[r][16 q .. 16 q + 15] from the ELL entries of row r (padding entries have value 0).
__global__ void __launch_bounds__(256) bj_blocks_kernel(int64_t npad, int w, const int32_t* __restrict__ ecol,
                                                        const double* __restrict__ eval,
                                                        const double* __restrict__ T64, double* __restrict__ C) {
    const int64_t b = blockIdx.x;
    const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int64_t i = b * kB + r;
    const int64_t j0 = b * kB + q * 16;
    double acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;
    for (int e = 0; e < w; ++e) {
        const double v = eval[(int64_t)e * npad + i];
        const int64_t k = ecol[(int64_t)e * npad + i];
        const double* trow = T64 + k * npad + j0;   // T is symmetric: row k holds T_{kj}
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] += v * trow[c];
    }
    double* out = C + (b * kB + r) * kB + q * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) out[c] = acc[c];
}

__device__ inline double2 c_mul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 c_inv(double2 a) {
    const double d = a.x * a.x + a.y * a.y;
    return make_double2(a.x / d, -a.y / d);
}

// P_sb = (C_b + z_s I)^-1, one work-group of 256 threads per (block, listed system): Gauss-Jordan
// elimination with partial pivoting on [M | I] (64 x 128 complex in LDS; pivot = the largest
// modulus in the column, the first row on ties). Output column-major: P[(s nblk + b) 4096 + c 64 + r].
__global__ void __launch_bounds__(256) bj_invert_kernel(const double* __restrict__ C, const int* __restrict__ sys,
                                                        const double2* __restrict__ z, int64_t nblk,
                                                        double2* __restrict__ P) {
    __shared__ double2 A[kB][2 * kB + 1];
    __shared__ double2 fcol[kB];
    __shared__ int piv;
    const int64_t b = blockIdx.x;
    const int s = sys[blockIdx.y];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double2 zs = z[s];
    for (int idx = tid; idx < kB * 2 * kB; idx += 256) {
        const int r = idx / (2 * kB), c = idx % (2 * kB);
        double2 v;
        if (c < kB) {
            v = make_double2(C[(b * kB + r) * kB + c], 0.0);
            if (r == c) {
                v.x += zs.x;
                v.y += zs.y;
            }
        } else {
            v = make_double2(c - kB == r ? 1.0 : 0.0, 0.0);
        }
        A[r][c] = v;
    }
    __syncthreads();
    for (int p = 0; p < kB; ++p) {
        if (wave == 0) {
            // argmax over rows p .. 63 of |A[r][p]|^2; lane r holds row r
            double val = -1.0;
            if (lane >= p) val = A[lane][p].x * A[lane][p].x + A[lane][p].y * A[lane][p].y;
            int idx = lane;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(val, off, 64);
                const int oi = __shfl_xor(idx, off, 64);
                if (ov > val || (ov == val && oi < idx)) {
                    val = ov;
                    idx = oi;
                }
            }
            if (lane == 0) piv = idx;
        }
        __syncthreads();
        const int q = piv;
        if (q != p)
            for (int c = tid; c < 2 * kB; c += 256) {
                const double2 t = A[p][c];
                A[p][c] = A[q][c];
                A[q][c] = t;
            }
        __syncthreads();
        const double2 ip = c_inv(A[p][p]);
        __syncthreads();   // every thread has read the pivot before row p is scaled
        for (int c = tid; c < 2 * kB; c += 256) A[p][c] = c_mul(A[p][c], ip);
        if (tid < kB) fcol[tid] = A[tid][p];
        __syncthreads();
        for (int idx = tid; idx < kB * 2 * kB; idx += 256) {
            const int r = idx / (2 * kB), c = idx % (2 * kB);
            if (r == p) continue;
            const double2 f = fcol[r], a = A[p][c];
            A[r][c] = make_double2(A[r][c].x - (f.x * a.x - f.y * a.y), A[r][c].y - (f.x * a.y + f.y * a.x));
        }
        __syncthreads();
    }
    double2* out = P + ((int64_t)s * nblk + b) * kB * kB;
    for (int idx = tid; idx < kB * kB; idx += 256) {
        const int c = idx / kB, r = idx % kB;
        out[idx] = A[r][kB + c];
    }
}

// The preconditioned product input for block b of listed system k: v = V(s, j) * scale[s] is
// written back (the normalised basis vector), u = P_sb v goes to U(s) and to columns 2k, 2k+1 of
// the packed block X. A system with run[s] == 0 gets zero columns.
template <typename E>
__global__ void __launch_bounds__(64) bj_pack_kernel(Basis V, int j, const int* __restrict__ sys,
                                                     const double* __restrict__ scale, const double2* __restrict__ P,
                                                     int64_t nblk, Basis U, E* __restrict__ X, int64_t ld,
                                                     const int* __restrict__ run) {
    __shared__ double2 v[kB];
    const int64_t b = blockIdx.x;
    const int k = blockIdx.y;
    const int s = sys[k];
    const int r = threadIdx.x;
    const int64_t i = b * kB + r;
    if (run && !run[s]) {   // uniform over the work-group
        X[(int64_t)(2 * k) * ld + i] = cast_from_double<E>(0.0);
        X[(int64_t)(2 * k + 1) * ld + i] = cast_from_double<E>(0.0);
        return;
    }
    double* vr = vslot(V, s, j);
    const double sc = scale ? scale[s] : 1.0;
    const double a = vr[i] * sc, bb = vr[i + V.npad] * sc;
    vr[i] = a;
    vr[i + V.npad] = bb;
    v[r] = make_double2(a, bb);
    __syncthreads();
    const double2* Pb = P + ((int64_t)s * nblk + b) * kB * kB;
    double ar = 0.0, ai = 0.0;
    for (int c = 0; c < kB; ++c) {
        const double2 p = Pb[c * kB + r], x = v[c];
        ar += p.x * x.x - p.y * x.y;
        ai += p.x * x.y + p.y * x.x;
    }
    double* ur = vslot(U, s, 0);
    ur[i] = ar;
    ur[i + U.npad] = ai;
    X[(int64_t)(2 * k) * ld + i] = cast_from_double<E>(ar);
    X[(int64_t)(2 * k + 1) * ld + i] = cast_from_double<E>(ai);
}

// X(s) += P_s U(s) over block b of listed system k (the iterate update through the preconditioner)
__global__ void __launch_bounds__(64) bj_add_kernel(const int* __restrict__ sys, const double2* __restrict__ P,
                                                    int64_t nblk, Basis U, Basis X) {
    __shared__ double2 t[kB];
    const int64_t b = blockIdx.x;
    const int s = sys[blockIdx.y];
    const int r = threadIdx.x;
    const int64_t i = b * kB + r;
    const double* ur = vslot(U, s, 0);
    t[r] = make_double2(ur[i], ur[i + U.npad]);
    __syncthreads();
    const double2* Pb = P + ((int64_t)s * nblk + b) * kB * kB;
    double ar = 0.0, ai = 0.0;
    for (int c = 0; c < kB; ++c) {
        const double2 p = Pb[c * kB + r], x = t[c];
        ar += p.x * x.x - p.y * x.y;
        ai += p.x * x.y + p.y * x.x;
    }
    double* xr = vslot(X, s, 0);
    xr[i] += ar;
    xr[i + X.npad] += ai;
}

}  // namespace

void bj_setup(const Structure& S, const int* sys, int nsys, const double2* z, double* C, double2* P,
              hipStream_t st) {
    if (!S.T64) throw Error{WFQ_EINVAL, "block-Jacobi preconditioning needs the stored FP64 T"};
    const int64_t nblk = S.npad / kB;
    hipLaunchKernelGGL(bj_blocks_kernel, dim3((unsigned)nblk), dim3(256), 0, st, S.npad, S.ell_w, S.ell_col, S.ell_val,
                       S.T64, C);
    WFQ_CHECK_LAUNCH();
    if (nsys <= 0) return;
    hipLaunchKernelGGL(bj_invert_kernel, dim3((unsigned)nblk, (unsigned)nsys), dim3(256), 0, st, C, sys, z, nblk, P);
    WFQ_CHECK_LAUNCH();
}

void bj_pack(int prec, const Basis& V, int j, const int* sys, int nsys, const double* scale, const double2* P,
             int64_t npad, const Basis& U, void* X, int64_t ld, const int* run, hipStream_t st) {
    if (nsys <= 0) return;
    const int64_t nblk = npad / kB;
    dim3 grd((unsigned)nblk, (unsigned)nsys);
    if (prec == WFQ_PREC_FP64)
        hipLaunchKernelGGL(bj_pack_kernel<double>, grd, dim3(kB), 0, st, V, j, sys, scale, P, nblk, U,
                           static_cast<double*>(X), ld, run);
    else if (prec == WFQ_PREC_FP32)
        hipLaunchKernelGGL(bj_pack_kernel<float>, grd, dim3(kB), 0, st, V, j, sys, scale, P, nblk, U,
                           static_cast<float*>(X), ld, run);
    else
        hipLaunchKernelGGL(bj_pack_kernel<uint16_t>, grd, dim3(kB), 0, st, V, j, sys, scale, P, nblk, U,
                           static_cast<uint16_t*>(X), ld, run);
    WFQ_CHECK_LAUNCH();
}

void bj_add(const int* sys, int nsys, const double2* P, int64_t npad, const Basis& U, const Basis& X, hipStream_t st) {
    if (nsys <= 0) return;
    const int64_t nblk = npad / kB;
    hipLaunchKernelGGL(bj_add_kernel, dim3((unsigned)nblk, (unsigned)nsys), dim3(kB), 0, st, sys, P, nblk, U, X);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
