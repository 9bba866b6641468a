// Block-Jacobi right preconditioning of the batched GMRES (a project extension: the paper applies
// its Krylov solvers without preconditioning, reports that the diagonal of the matrix did not help,
// and names the missing preconditioner as a bottleneck in its conclusions).
//
// Blocks are 64 consecutive atoms of the internal, spatially sorted order. For block b the
// frequency-independent part is C_b = (L T)_bb, C_b[r][c] = sum_k L_{ik} T_{kj} (i = 64 b + r,
// j = 64 b + c); for system s the block of the operator is C_b + z_s I, inverted once per solve by
// Gauss-Jordan elimination with partial pivoting (FP64, in registers) and stored in complex FP32.
// GMRES then runs on (L T + z I) M^-1 with the true residual; the product input is u = M^-1 v
// (block by block), and the iterate update is x += M^-1 (V y). Padding atoms have zero rows and
// columns in C, so their diagonal is z and the padding of every vector stays zero.
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

constexpr int kG = 8;        // inversion: threads per row
constexpr int kJ = kB / kG;  // inversion: entries per thread

// P_sb = (C_b + z_s I)^-1, one work-group of 512 threads per (block, listed system): Gauss-Jordan
// elimination in place with partial pivoting (pivot = the largest modulus in the column, the first
// row on ties), in FP64 and in registers: thread (row r = tid / 8, g = tid % 8) holds the 8 entries
// of row r in the columns g + 8 j. Step p shares only the pivot column, the pivot row and the row it
// is swapped with through LDS (double-buffered by p % 2, so two barriers a step). The row swaps make
// the result the inverse of the row-permuted matrix; the columns are put back in place when the
// result is written. To keep the register indices compile-time constants, the 8 steps of column
// group jp run unrolled with the pivot column in a[0], and the row array is rotated by one after each
// group (8 rotations restore the original order).
// Output rounded to complex FP32, column-major: P[(s nblk + b) 4096 + c 64 + r]. The rounded inverse
// is the preconditioner (the same one in the product and in the iterate update), so the rounding
// changes the step count at most marginally and the solution not at all.
__global__ void __launch_bounds__(512) bj_invert_kernel(const double* __restrict__ C, const int* __restrict__ sys,
                                                        const double2* __restrict__ z, int64_t nblk,
                                                        float2* __restrict__ P) {
    __shared__ double mag[2][kB];
    __shared__ double2 colv[2][kB];
    __shared__ double2 prow[2][kB];
    __shared__ double2 srow[2][kB];
    __shared__ int qs[kB];
    __shared__ int dest[kB];
    const int64_t b = blockIdx.x;
    const int s = sys[blockIdx.y];
    const int tid = threadIdx.x, r = tid >> 3, g = tid & 7, lane = tid & 63;
    const double2 zs = z[s];
    double2 a[kJ];
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        const int c = g + kG * j;
        double2 v = make_double2(C[(b * kB + r) * kB + c], 0.0);
        if (c == r) {
            v.x += zs.x;
            v.y += zs.y;
        }
        a[j] = v;
    }
#pragma unroll 1
    for (int jp = 0; jp < kJ; ++jp) {
#pragma unroll
        for (int gp = 0; gp < kG; ++gp) {
            const int p = kG * jp + gp;
            const int buf = gp & 1;
            if (g == gp) {   // the owners of column p (held in a[0])
                const double2 v = a[0];
                mag[buf][r] = r >= p ? v.x * v.x + v.y * v.y : -1.0;
                colv[buf][r] = v;
            }
            __syncthreads();
            // argmax over the rows, the same in every wave (a total order: larger value, then lower row)
            double val = mag[buf][lane];
            int q = lane;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(val, off, 64);
                const int oq = __shfl_xor(q, off, 64);
                if (ov > val || (ov == val && oq < q)) {
                    val = ov;
                    q = oq;
                }
            }
            if (r == q) {
#pragma unroll
                for (int j = 0; j < kJ; ++j) prow[buf][g + kG * ((j + jp) & (kJ - 1))] = a[j];
            }
            if (r == p && q != p) {
#pragma unroll
                for (int j = 0; j < kJ; ++j) srow[buf][g + kG * ((j + jp) & (kJ - 1))] = a[j];
            }
            if (tid == 0) qs[p] = q;
            __syncthreads();
            const double2 inv = c_inv(prow[buf][p]);
            if (r == p) {
                // the (swapped-in) pivot row, scaled; its column p becomes 1 / pivot
#pragma unroll
                for (int j = 0; j < kJ; ++j) {
                    const int c = g + kG * ((j + jp) & (kJ - 1));
                    a[j] = c == p ? inv : c_mul(prow[buf][c], inv);
                }
            } else {
                double2 f = colv[buf][r];
                if (r == q) {   // this row now holds the old row p
                    f = colv[buf][p];
#pragma unroll
                    for (int j = 0; j < kJ; ++j) a[j] = srow[buf][g + kG * ((j + jp) & (kJ - 1))];
                }
                const double2 fi = c_mul(f, inv);
#pragma unroll
                for (int j = 0; j < kJ; ++j) {
                    const int c = g + kG * ((j + jp) & (kJ - 1));
                    const double2 pr = prow[buf][c];
                    a[j] = c == p ? make_double2(-fi.x, -fi.y)
                                  : make_double2(a[j].x - (fi.x * pr.x - fi.y * pr.y),
                                                 a[j].y - (fi.x * pr.y + fi.y * pr.x));
                }
            }
        }
        // rotate so that the next group's pivot column sits in a[0]
        const double2 t = a[0];
#pragma unroll
        for (int j = 0; j < kJ - 1; ++j) a[j] = a[j + 1];
        a[kJ - 1] = t;
    }
    __syncthreads();
    // inverse = X S_63 ... S_0 (S_p: the row swap of step p, applied to columns): output column j is
    // computed column sigma(j), with sigma(j) = j carried through the swaps of steps 0 .. 63 in order
    if (tid < kB) {
        int idx = tid;
        for (int p = 0; p < kB; ++p) {
            const int q = qs[p];
            idx = idx == p ? q : (idx == q ? p : idx);
        }
        dest[idx] = tid;
    }
    __syncthreads();
    float2* out = P + ((int64_t)s * nblk + b) * kB * kB;
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        const int c = g + kG * j;
        out[dest[c] * kB + r] = make_float2((float)a[j].x, (float)a[j].y);
    }
}

// Lane c's value of x, for a wave-uniform c (two 32-bit lane reads).
__device__ inline double lane_value(double x, int c) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), c);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), c);
    return __hiloint2double(hi, lo);
}

// y[r] = sum_c P_sb[c][r] x[c] for the 64 rows of one block, x held one entry per lane; the 64
// columns are read as 4 groups of 16 loads in flight (coalesced 512-byte rows of P).
__device__ inline void block_apply(const float2* __restrict__ Pb, int r, double xr, double xi, double& ar,
                                   double& ai) {
    ar = 0.0;
    ai = 0.0;
#pragma unroll
    for (int c0 = 0; c0 < kB; c0 += 16) {
        float2 p[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) p[t] = Pb[(c0 + t) * kB + r];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const double vr = lane_value(xr, c0 + t), vi = lane_value(xi, c0 + t);
            const double pr = p[t].x, pi = p[t].y;
            ar += pr * vr - pi * vi;
            ai += pr * vi + pi * vr;
        }
    }
}

// The preconditioned product input, one wave per (block b, listed system k): v = V(s, j) * scale[s]
// is written back (the normalised basis vector), u = P_sb v goes to U(s) and to columns 2k, 2k+1
// of the packed block X. A system with run[s] == 0 gets zero columns.
template <typename E>
__global__ void __launch_bounds__(256) bj_pack_kernel(Basis V, int j, const int* __restrict__ sys, int nsys,
                                                      const double* __restrict__ scale, const float2* __restrict__ P,
                                                      int64_t nblk, Basis U, E* __restrict__ X, int64_t ld,
                                                      const int* __restrict__ run) {
    const int64_t b = blockIdx.x;
    const int k = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (k >= nsys) return;   // whole waves; no work-group barrier below
    const int s = sys[k];
    const int r = threadIdx.x & 63;
    const int64_t i = b * kB + r;
    if (run && !run[s]) {
        X[(int64_t)(2 * k) * ld + i] = cast_from_double<E>(0.0);
        X[(int64_t)(2 * k + 1) * ld + i] = cast_from_double<E>(0.0);
        return;
    }
    double* vr = vslot(V, s, j);
    const double sc = scale ? scale[s] : 1.0;
    const double a = vr[i] * sc, bb = vr[i + V.npad] * sc;
    vr[i] = a;
    vr[i + V.npad] = bb;
    double ar, ai;
    block_apply(P + ((int64_t)s * nblk + b) * kB * kB, r, a, bb, ar, ai);
    double* ur = vslot(U, s, 0);
    ur[i] = ar;
    ur[i + U.npad] = ai;
    X[(int64_t)(2 * k) * ld + i] = cast_from_double<E>(ar);
    X[(int64_t)(2 * k + 1) * ld + i] = cast_from_double<E>(ai);
}

// X(s) += P_s U(s), one wave per (block b, listed system k) (the iterate update through M^-1)
__global__ void __launch_bounds__(256) bj_add_kernel(const int* __restrict__ sys, int nsys,
                                                     const float2* __restrict__ P, int64_t nblk, Basis U, Basis X) {
    const int64_t b = blockIdx.x;
    const int k = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (k >= nsys) return;
    const int s = sys[k];
    const int r = threadIdx.x & 63;
    const int64_t i = b * kB + r;
    const double* ur = vslot(U, s, 0);
    double ar, ai;
    block_apply(P + ((int64_t)s * nblk + b) * kB * kB, r, ur[i], ur[i + U.npad], ar, ai);
    double* xr = vslot(X, s, 0);
    xr[i] += ar;
    xr[i + X.npad] += ai;
}

}  // namespace

void bj_setup(const Structure& S, const int* sys, int nsys, const double2* z, double* C, float2* P,
              hipStream_t st) {
    if (!S.T64) throw Error{WFQ_EINVAL, "block-Jacobi preconditioning needs the stored FP64 T"};
    const int64_t nblk = S.npad / kB;
    hipLaunchKernelGGL(bj_blocks_kernel, dim3((unsigned)nblk), dim3(256), 0, st, S.npad, S.ell_w, S.ell_col, S.ell_val,
                       S.T64, C);
    WFQ_CHECK_LAUNCH();
    if (nsys <= 0) return;
    hipLaunchKernelGGL(bj_invert_kernel, dim3((unsigned)nblk, (unsigned)nsys), dim3(64 * kG), 0, st, C, sys, z, nblk,
                       P);
    WFQ_CHECK_LAUNCH();
}

void bj_pack(int prec, const Basis& V, int j, const int* sys, int nsys, const double* scale, const float2* P,
             int64_t npad, const Basis& U, void* X, int64_t ld, const int* run, hipStream_t st) {
    if (nsys <= 0) return;
    const int64_t nblk = npad / kB;
    dim3 grd((unsigned)nblk, (unsigned)((nsys + 3) / 4));
    if (prec == WFQ_PREC_FP64)
        hipLaunchKernelGGL(bj_pack_kernel<double>, grd, dim3(256), 0, st, V, j, sys, nsys, scale, P, nblk, U,
                           static_cast<double*>(X), ld, run);
    else if (prec == WFQ_PREC_FP32)
        hipLaunchKernelGGL(bj_pack_kernel<float>, grd, dim3(256), 0, st, V, j, sys, nsys, scale, P, nblk, U,
                           static_cast<float*>(X), ld, run);
    else
        hipLaunchKernelGGL(bj_pack_kernel<uint16_t>, grd, dim3(256), 0, st, V, j, sys, nsys, scale, P, nblk, U,
                           static_cast<uint16_t*>(X), ld, run);
    WFQ_CHECK_LAUNCH();
}

void bj_add(const int* sys, int nsys, const float2* P, int64_t npad, const Basis& U, const Basis& X, hipStream_t st) {
    if (nsys <= 0) return;
    const int64_t nblk = npad / kB;
    hipLaunchKernelGGL(bj_add_kernel, dim3((unsigned)nblk, (unsigned)((nsys + 3) / 4)), dim3(256), 0, st, sys, nsys, P,
                       nblk, U, X);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
