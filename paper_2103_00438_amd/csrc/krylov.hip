// Krylov-side kernels: the sparse half of the operator (L Y + z V), the reduction of Gram-Schmidt
// partial dots (the Arnoldi sweeps themselves are in dcgs.hip), the Hessenberg least-squares solve,
// the solution update, the FP64 refinement residual and the observables (arXiv 2103.00438, Section
// "Solution strategies": GMRES paragraph and restarted GMRES(k); Eq. (long-cross) for the dipole).
//
// All of these are bandwidth-bound vector sweeps. Reductions are deterministic: each wave sums a
// fixed 512-row chunk with a fixed butterfly, and per-chunk partials are added in chunk order.
#include "device_util.h"
#include "krylov.h"

namespace wfq {

namespace {

__device__ inline double* vre(const Basis& V, int s, int j) { return V.base + (int64_t)s * V.sys_stride + (int64_t)j * V.vec_stride; }

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// block of 256 threads -> one value, fixed order
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = sh[0] + sh[1] + sh[2] + sh[3];
    return t;
}

template <typename E>
__global__ void __launch_bounds__(256) pack_kernel(Basis V, const int* __restrict__ sys, int j,
                                                   const double* __restrict__ scale, int write_back, E* __restrict__ X,
                                                   int64_t ld, const int* __restrict__ run) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    const int s = sys[k];
    if (run && !run[s]) {   // a system that stopped inside this chunk of steps: zero columns
        X[(int64_t)(2 * k) * ld + i] = cast_from_double<E>(0.0);
        X[(int64_t)(2 * k + 1) * ld + i] = cast_from_double<E>(0.0);
        return;
    }
    double* re = vre(V, s, j);
    double* im = re + V.npad;
    const double sc = scale ? scale[s] : 1.0;
    const double a = re[i] * sc, b = im[i] * sc;
    if (write_back) {
        re[i] = a;
        im[i] = b;
    }
    X[(int64_t)(2 * k) * ld + i] = cast_from_double<E>(a);
    X[(int64_t)(2 * k + 1) * ld + i] = cast_from_double<E>(b);
}

// Each thread owns one row of L and up to NS systems, so the row's (col, val) pairs are read once
// for NS right-hand sides; L is read in the transposed ELL layout (coalesced across rows).
template <typename YE, int NS>
__global__ void __launch_bounds__(256) spmm_kernel(int64_t n, int64_t npad, int w, const int32_t* __restrict__ ecol,
                                                   const double* __restrict__ eval, const YE* __restrict__ Y,
                                                   int64_t ld, const int* __restrict__ sys, int nsys,
                                                   const double2* __restrict__ z, Basis Vs, Basis V, int jsrc,
                                                   int jdst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int k0 = blockIdx.y * NS;
    const int kn = min(NS, nsys - k0);
    double ar[NS], ai[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) ar[t] = ai[t] = 0.0;
    for (int p = 0; p < w; ++p) {
        const int c = ecol[(int64_t)p * npad + i];
        const double v = eval[(int64_t)p * npad + i];
#pragma unroll
        for (int t = 0; t < NS; ++t)
            if (t < kn) {
                ar[t] += v * widen(Y[(int64_t)(2 * (k0 + t)) * ld + c]);
                ai[t] += v * widen(Y[(int64_t)(2 * (k0 + t) + 1) * ld + c]);
            }
    }
#pragma unroll
    for (int t = 0; t < NS; ++t)
        if (t < kn) {
            const int s = sys[k0 + t];
            const double* sr = vre(Vs, s, jsrc);
            const double vr = sr[i], vi = sr[i + Vs.npad];
            const double2 zz = z[s];
            double* dr = vre(V, s, jdst);
            dr[i] = ar[t] + zz.x * vr - zz.y * vi;
            dr[i + V.npad] = ai[t] + zz.x * vi + zz.y * vr;
        }
}

// Row-block variant. A work-group owns R consecutive rows for one group of systems. Their ELL
// rows are staged once in LDS ([entry][row], so lanes read consecutive words) and reused for every
// system of the group; each wave works on 64 / R systems at a time, one lane per (row, system).
// The neighbour window of each Y plane is then gathered by the work-groups of neighbouring row
// blocks at about the same time: row blocks are laid out so that the work-groups of one XCD (ids
// congruent mod 8) own one contiguous run of rows, and that XCD's L2 serves the overlapping windows.
template <typename YE> struct Pair2;
template <> struct Pair2<float> { using type = float2; };
template <> struct Pair2<double> { using type = double2; };

// Yp[k][i] = (Y[2k][i], Y[2k+1][i]): the real and imaginary planes of each system's product side
// by side, so that the SpMM fetches both with one load per neighbour
template <typename YE>
__global__ void __launch_bounds__(256) pair_kernel(const YE* __restrict__ Y, int64_t ld,
                                                   typename Pair2<YE>::type* __restrict__ Yp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;   // grid: ld / 256 blocks (ld % 256 == 0)
    const int64_t k = blockIdx.y;
    typename Pair2<YE>::type v;
    v.x = Y[(2 * k) * ld + i];
    v.y = Y[(2 * k + 1) * ld + i];
    Yp[k * ld + i] = v;
}

// PAIRS: Y is the interleaved form (row k = ld pairs) instead of two planes per system
template <typename YE, int R, bool PAIRS = false>
__global__ void __launch_bounds__(256) spmm_rows_kernel(int64_t n, int64_t npad, int w,
                                                        const int32_t* __restrict__ ecol,
                                                        const double* __restrict__ eval, const YE* __restrict__ Y,
                                                        int64_t ld, const int* __restrict__ sys, int nsys, int per_group,
                                                        const double2* __restrict__ z, Basis Vs, Basis V, int jsrc,
                                                        int jdst,
                                                        int y_by_sys) {
    extern __shared__ char smem[];
    double* lval = reinterpret_cast<double*>(smem);
    int32_t* lcol = reinterpret_cast<int32_t*>(smem + (size_t)w * R * sizeof(double));
    constexpr int G = 64 / R;
    const int per_xcd = (int)(gridDim.x >> 3);
    const int64_t rb = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const int64_t r0 = rb * R;
    if (r0 >= n) return;   // whole work-group: grid padded to a multiple of 8 row blocks
    for (int q = threadIdx.x; q < w * R; q += 256) {
        const int e = q / R, r = q % R;
        const int64_t i = r0 + r;   // < npad: npad is a multiple of R
        lcol[q] = ecol[(int64_t)e * npad + i];
        lval[q] = eval[(int64_t)e * npad + i];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane % R, g = lane / R;
    const int64_t i = r0 + r;
    if (i >= n) return;
    const int k_end = min(nsys, (int)(blockIdx.y + 1) * per_group);
    for (int k = (int)blockIdx.y * per_group + wave * G + g; k < k_end; k += 4 * G) {
        double ar = 0.0, ai = 0.0;
        if constexpr (PAIRS) {
            const typename Pair2<YE>::type* yp =
                reinterpret_cast<const typename Pair2<YE>::type*>(Y) + (int64_t)(y_by_sys ? sys[k] : k) * ld;
#pragma unroll 4
            for (int e = 0; e < w; ++e) {
                const int c = lcol[e * R + r];
                const double v = lval[e * R + r];
                const typename Pair2<YE>::type y = yp[c];
                ar += v * widen(y.x);
                ai += v * widen(y.y);
            }
        } else {
            const YE* yr = Y + (int64_t)(2 * (y_by_sys ? sys[k] : k)) * ld;
            const YE* yi = yr + ld;
#pragma unroll 4
            for (int e = 0; e < w; ++e) {
                const int c = lcol[e * R + r];
                const double v = lval[e * R + r];
                ar += v * widen(yr[c]);
                ai += v * widen(yi[c]);
            }
        }
        const int s = sys[k];
        const double* sr = vre(Vs, s, jsrc);
        const double vr = sr[i], vi = sr[i + Vs.npad];
        const double2 zz = z[s];
        double* dr = vre(V, s, jdst);
        dr[i] = ar + zz.x * vr - zz.y * vi;
        dr[i + V.npad] = ai + zz.x * vi + zz.y * vr;
    }
}

template <typename YE, int R, bool PAIRS = false>
void launch_spmm_rows(const Structure& S, const YE* Y, int64_t ld, const int* sys, int nsys, const double2* z,
                      const Basis& Vs, const Basis& V, int jsrc, int jdst, bool y_by_sys, hipStream_t st) {
    constexpr int G = 64 / R;
    const int64_t nb = S.npad / R;
    const int64_t nb8 = (nb + 7) / 8 * 8;
    // enough work-groups to fill the chip (about 8 per CU), but at least one system per wave
    const int64_t want = (2048 + nb8 - 1) / nb8;
    const int gy = (int)std::max<int64_t>(1, std::min<int64_t>(want, (nsys + 4 * G - 1) / (4 * G)));
    const int per_group = (nsys + gy - 1) / gy;
    const size_t lds = (size_t)S.ell_w * R * 12;
    hipLaunchKernelGGL((spmm_rows_kernel<YE, R, PAIRS>), dim3((unsigned)nb8, (unsigned)gy), dim3(256), lds, st, S.n, S.npad,
                       S.ell_w, S.ell_col, S.ell_val, Y, ld, sys, nsys, per_group, z, Vs, V, jsrc, jdst,
                       (int)y_by_sys);
}

__global__ void reduce_dots_kernel(const int* __restrict__ sys, int j, const double2* __restrict__ partial, int mdim,
                                   int64_t nwc, double2* __restrict__ h, const int* __restrict__ active) {
    const int s = sys[blockIdx.x];
    if (active && !active[s]) return;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        const double2* p = partial + ((int64_t)s * mdim + i) * nwc;
        double sr = 0.0, si = 0.0;
        for (int64_t w = 0; w < nwc; ++w) {
            sr += p[w].x;
            si += p[w].y;
        }
        h[(int64_t)s * mdim + i] = make_double2(sr, si);
    }
}

// One wave per system: column-oriented back substitution on R y = g (k <= mdim - 1 steps).
__global__ void __launch_bounds__(64) tri_solve_kernel(const int* __restrict__ sys, const int* __restrict__ ksteps,
                                                       int mdim, const double2* __restrict__ R,
                                                       const double2* __restrict__ g, double2* __restrict__ y) {
    const int s = sys[blockIdx.x];
    const int lane = threadIdx.x;
    const int kk = ksteps[s];
    const double2* Rs = R + (int64_t)s * mdim * mdim;
    const double2* gs = g + (int64_t)s * (mdim + 1);
    double2* ys = y + (int64_t)s * mdim;
    // each lane keeps the right-hand side entries l = lane, lane + 64, ...
    double2 rhs[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int l = lane + 64 * q;
        rhs[q] = l < kk ? gs[l] : make_double2(0.0, 0.0);
    }
    for (int i = kk - 1; i >= 0; --i) {
        const int owner = i & 63, slot = i >> 6;
        double2 ri = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q == slot) ri = rhs[q];
        ri.x = __shfl(ri.x, owner, 64);
        ri.y = __shfl(ri.y, owner, 64);
        const double2 d = Rs[(int64_t)i * mdim + i];
        const double dd = d.x * d.x + d.y * d.y;
        const double2 yi = make_double2((ri.x * d.x + ri.y * d.y) / dd, (ri.y * d.x - ri.x * d.y) / dd);
        if (lane == 0) ys[i] = yi;
        // rhs_l -= R_li y_i for l < i (column i of R)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int l = lane + 64 * q;
            if (l < i) {
                const double2 t = cmul(Rs[(int64_t)i * mdim + l], yi);
                rhs[q].x -= t.x;
                rhs[q].y -= t.y;
            }
        }
    }
}

__global__ void __launch_bounds__(256) x_update_kernel(Basis V, Basis X, int64_t n, const int* __restrict__ sys,
                                                       const int* __restrict__ ksteps, const double2* __restrict__ y,
                                                       int mdim) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int s = sys[blockIdx.y];
    const int kk = ksteps[s];
    double ar = 0.0, ai = 0.0;
    for (int l = 0; l < kk; ++l) {
        const double2 yy = y[(int64_t)s * mdim + l];
        const double* vr = vre(V, s, l);
        const double a = vr[i], b = vr[i + V.npad];
        ar += yy.x * a - yy.y * b;
        ai += yy.x * b + yy.y * a;
    }
    double* xr = vre(X, s, 0);
    xr[i] += ar;
    xr[i + X.npad] += ai;
}

// V(s, 0) = b_dir(s) - (L Y_s + z_s x_s), system s = sys[k] with its product in columns 2k and 2k + 1 of
// Y; norm2[s][blk] = the block's sum of |r_i|^2 and qtq[s][blk] (if not NULL) that of
// Re(conj(x_i) (T x)_i). The grid's x index is the system and its y index the row block, so the
// work-groups of one row block run together and read its rows of L through the L2 cache once.
__global__ void __launch_bounds__(256) residual_kernel(int64_t n, int64_t npad, int w,
                                                       const int32_t* __restrict__ ecol,
                                                       const double* __restrict__ eval,
                                                       const double* __restrict__ Y, int64_t ld,
                                                       const int* __restrict__ sys, const double2* __restrict__ z,
                                                       Basis X, const double* __restrict__ b, const int* __restrict__ dir,
                                                       Basis V, double* __restrict__ norm2, int nblk,
                                                       double* __restrict__ qtq) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.y * 256 + threadIdx.x;
    const int k = blockIdx.x;
    const int s = sys[k];
    double nn = 0.0, et = 0.0;
    if (i < n) {
        double ar = 0.0, ai = 0.0;
        for (int p = 0; p < w; ++p) {
            const int c = ecol[(int64_t)p * npad + i];
            const double v = eval[(int64_t)p * npad + i];
            ar += v * Y[(int64_t)(2 * k) * ld + c];
            ai += v * Y[(int64_t)(2 * k + 1) * ld + c];
        }
        const double* xr = vre(X, s, 0);
        const double xre = xr[i], xim = xr[i + X.npad];
        const double2 zz = z[s];
        const double rr = b[(int64_t)dir[s] * V.npad + i] - (ar + zz.x * xre - zz.y * xim);
        const double ri = -(ai + zz.x * xim + zz.y * xre);
        double* vr = vre(V, s, 0);
        vr[i] = rr;
        vr[i + V.npad] = ri;
        nn = rr * rr + ri * ri;
        // Re(conj(x_i) (T x)_i); T is real and symmetric, so the sum over i is x^H T x
        et = xre * Y[(int64_t)(2 * k) * ld + i] + xim * Y[(int64_t)(2 * k + 1) * ld + i];
    }
    nn = block_sum(nn, sh);
    if (threadIdx.x == 0) norm2[(int64_t)s * nblk + blockIdx.y] = nn;
    if (qtq) {
        et = block_sum(et, sh);   // block_sum synchronises before it reuses sh
        if (threadIdx.x == 0) qtq[(int64_t)s * nblk + blockIdx.y] = et;
    }
}

__global__ void __launch_bounds__(256) copy_rhs_kernel(int64_t n, const int* __restrict__ sys,
                                                       const double* __restrict__ b, const int* __restrict__ dir, Basis V,
                                                       double* __restrict__ norm2, int nblk) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int s = sys[blockIdx.y];
    double nn = 0.0;
    if (i < n) {
        const double v = b[(int64_t)dir[s] * V.npad + i];
        double* vr = vre(V, s, 0);
        vr[i] = v;
        vr[i + V.npad] = 0.0;
        nn = v * v;
    }
    nn = block_sum(nn, sh);
    if (threadIdx.x == 0) norm2[(int64_t)s * nblk + blockIdx.x] = nn;
}

__global__ void sumsq_kernel(const int* __restrict__ sys, int nsys, const double* __restrict__ norm2, int nb,
                             double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsys) return;
    const int s = sys[k];
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += norm2[(int64_t)s * nb + b];
    out[s] = sqrt(acc);
}

__global__ void __launch_bounds__(256) observables_kernel(int64_t n, int64_t npad, const double* __restrict__ pos,
                                                          const int* __restrict__ sys, Basis X, double E0,
                                                          double2* __restrict__ alpha) {
    __shared__ double sh[4];
    const int s = sys[blockIdx.x];
    const double* xr = vre(X, s, 0);
    const double* xi = xr + X.npad;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double a = xr[i], b = xi[i];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double r = pos[l * npad + i];
            acc[2 * l] += r * a;
            acc[2 * l + 1] += r * b;
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] = block_sum(acc[q], sh);
    if (threadIdx.x == 0)
        for (int l = 0; l < 3; ++l) alpha[(int64_t)s * 3 + l] = make_double2(acc[2 * l] / E0, acc[2 * l + 1] / E0);
}

__global__ void __launch_bounds__(256) scatter_kernel(int64_t n, const int32_t* __restrict__ perm,
                                                      const int* __restrict__ sys, Basis X, double* __restrict__ qr,
                                                      double* __restrict__ qi) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int s = sys[blockIdx.y];
    const double* xr = vre(X, s, 0);
    const int64_t o = (int64_t)s * n + perm[i];
    if (qr) qr[o] = xr[i];
    if (qi) qi[o] = xr[i + X.npad];
}

// x(sys[k]) = x(src_a[k]) + t[k] (x(src_b[k]) - x(src_a[k])), complex t (the targets are distinct from
// every source)
__global__ void __launch_bounds__(256) interp_kernel(int64_t n, const int* __restrict__ sys,
                                                     const int* __restrict__ src_a, const int* __restrict__ src_b,
                                                     const double2* __restrict__ t, Basis X) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int k = blockIdx.y;
    const double* ar = vre(X, src_a[k], 0);
    const double* br = vre(X, src_b[k], 0);
    double* xr = vre(X, sys[k], 0);
    const double2 tk = t[k];
    const double dr = br[i] - ar[i], di = br[i + X.npad] - ar[i + X.npad];
    xr[i] = ar[i] + (tk.x * dr - tk.y * di);
    xr[i + X.npad] = ar[i + X.npad] + (tk.x * di + tk.y * dr);
}

}  // namespace

void interp_start(const int* sys, int nsys, const int* src_a, const int* src_b, const double2* t, const Basis& x,
                  int64_t n, hipStream_t st) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)((n + 255) / 256), (unsigned)nsys);
    hipLaunchKernelGGL(interp_kernel, grd, dim3(256), 0, st, n, sys, src_a, src_b, t, x);
    WFQ_CHECK_LAUNCH();
}

void pack_columns(int prec, const Basis& V, const int* sys, int nsys, int j, const double* scale, bool write_back,
                  void* X, int64_t ld, hipStream_t st, const int* run) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)(V.npad / 256), (unsigned)nsys);
    if (prec == WFQ_PREC_FP64)
        hipLaunchKernelGGL(pack_kernel<double>, grd, dim3(256), 0, st, V, sys, j, scale, (int)write_back,
                           static_cast<double*>(X), ld, run);
    else if (prec == WFQ_PREC_FP32)
        hipLaunchKernelGGL(pack_kernel<float>, grd, dim3(256), 0, st, V, sys, j, scale, (int)write_back,
                           static_cast<float*>(X), ld, run);
    else
        hipLaunchKernelGGL(pack_kernel<uint16_t>, grd, dim3(256), 0, st, V, sys, j, scale, (int)write_back,
                           static_cast<uint16_t*>(X), ld, run);
    WFQ_CHECK_LAUNCH();
}

void spmm_shift(const Structure& S, bool y_is_f64, const void* Y, int64_t ld, const int* sys, int nsys,
                const double2* z, const Basis& V, int jsrc, int jdst, hipStream_t st, bool y_by_sys,
                const Basis* shift_src) {
    if (nsys <= 0) return;
    const Basis& Vs = shift_src ? *shift_src : V;
    // row-block kernel with the largest row block whose ELL rows fit in 40 KB of LDS (4 work-groups
    // per CU); the per-thread kernel only for neighbour lists too long even for 8 rows
    const size_t per_row = (size_t)S.ell_w * 12;
    const int R = per_row * 64 <= 40960 ? 64 : per_row * 32 <= 40960 ? 32 : per_row * 16 <= 40960 ? 16
                  : per_row * 8 <= 40960 ? 8 : 0;
    if (R > 0) {
        if (y_is_f64) {
            const double* Yd = static_cast<const double*>(Y);
            if (R == 64) launch_spmm_rows<double, 64>(S, Yd, ld, sys, nsys, z, Vs, V, jsrc, jdst, y_by_sys, st);
            else if (R == 32) launch_spmm_rows<double, 32>(S, Yd, ld, sys, nsys, z, Vs, V, jsrc, jdst, y_by_sys, st);
            else if (R == 16) launch_spmm_rows<double, 16>(S, Yd, ld, sys, nsys, z, Vs, V, jsrc, jdst, y_by_sys, st);
            else launch_spmm_rows<double, 8>(S, Yd, ld, sys, nsys, z, Vs, V, jsrc, jdst, y_by_sys, st);
        } else {
            const float* Yf = static_cast<const float*>(Y);
            if (R == 64) launch_spmm_rows<float, 64>(S, Yf, ld, sys, nsys, z, Vs, V, jsrc, jdst, y_by_sys, st);
            else if (R == 32) launch_spmm_rows<float, 32>(S, Yf, ld, sys, nsys, z, Vs, V, jsrc, jdst, y_by_sys, st);
            else if (R == 16) launch_spmm_rows<float, 16>(S, Yf, ld, sys, nsys, z, Vs, V, jsrc, jdst, y_by_sys, st);
            else launch_spmm_rows<float, 8>(S, Yf, ld, sys, nsys, z, Vs, V, jsrc, jdst, y_by_sys, st);
        }
        WFQ_CHECK_LAUNCH();
        return;
    }
    if (y_by_sys) throw Error{WFQ_EINVAL, "neighbour lists too long for the sparse product"};
    constexpr int NS = 8;
    dim3 grd((unsigned)((S.n + 255) / 256), (unsigned)((nsys + NS - 1) / NS));
    if (y_is_f64)
        hipLaunchKernelGGL((spmm_kernel<double, NS>), grd, dim3(256), 0, st, S.n, S.npad, S.ell_w, S.ell_col,
                           S.ell_val, static_cast<const double*>(Y), ld, sys, nsys, z, Vs, V, jsrc, jdst);
    else
        hipLaunchKernelGGL((spmm_kernel<float, NS>), grd, dim3(256), 0, st, S.n, S.npad, S.ell_w, S.ell_col,
                           S.ell_val, static_cast<const float*>(Y), ld, sys, nsys, z, Vs, V, jsrc, jdst);
    WFQ_CHECK_LAUNCH();
}

void spmm_shift_pairs(const Structure& S, bool y_is_f64, const void* Y, int64_t ld, void* Yp, const int* sys,
                      int nsys, const double2* z, const Basis& V, int jsrc, int jdst, hipStream_t st,
                      const Basis* shift_src) {
    if (nsys <= 0) return;
    // the row block of spmm_shift; the per-thread form (R = 0) reads the two planes
    const size_t per_row = (size_t)S.ell_w * 12;
    const int R = per_row * 64 <= 40960 ? 64 : per_row * 32 <= 40960 ? 32 : per_row * 16 <= 40960 ? 16
                  : per_row * 8 <= 40960 ? 8 : 0;
    if (R == 0 || ld != S.npad) {
        spmm_shift(S, y_is_f64, Y, ld, sys, nsys, z, V, jsrc, jdst, st, false, shift_src);
        return;
    }
    const Basis& Vs = shift_src ? *shift_src : V;
    dim3 pg((unsigned)(ld / 256), (unsigned)nsys);
    if (y_is_f64) {
        hipLaunchKernelGGL(pair_kernel<double>, pg, dim3(256), 0, st, static_cast<const double*>(Y), ld,
                           static_cast<double2*>(Yp));
        WFQ_CHECK_LAUNCH();
        const double* P = static_cast<const double*>(Yp);
        if (R == 64) launch_spmm_rows<double, 64, true>(S, P, ld, sys, nsys, z, Vs, V, jsrc, jdst, false, st);
        else if (R == 32) launch_spmm_rows<double, 32, true>(S, P, ld, sys, nsys, z, Vs, V, jsrc, jdst, false, st);
        else if (R == 16) launch_spmm_rows<double, 16, true>(S, P, ld, sys, nsys, z, Vs, V, jsrc, jdst, false, st);
        else launch_spmm_rows<double, 8, true>(S, P, ld, sys, nsys, z, Vs, V, jsrc, jdst, false, st);
    } else {
        hipLaunchKernelGGL(pair_kernel<float>, pg, dim3(256), 0, st, static_cast<const float*>(Y), ld,
                           static_cast<float2*>(Yp));
        WFQ_CHECK_LAUNCH();
        const float* P = static_cast<const float*>(Yp);
        if (R == 64) launch_spmm_rows<float, 64, true>(S, P, ld, sys, nsys, z, Vs, V, jsrc, jdst, false, st);
        else if (R == 32) launch_spmm_rows<float, 32, true>(S, P, ld, sys, nsys, z, Vs, V, jsrc, jdst, false, st);
        else if (R == 16) launch_spmm_rows<float, 16, true>(S, P, ld, sys, nsys, z, Vs, V, jsrc, jdst, false, st);
        else launch_spmm_rows<float, 8, true>(S, P, ld, sys, nsys, z, Vs, V, jsrc, jdst, false, st);
    }
    WFQ_CHECK_LAUNCH();
}

void spmm_shift_interleaved(const Structure& S, const double* Yp, int64_t ld, const int* sys, int nsys,
                            const double2* z, const Basis& V, int jsrc, int jdst, hipStream_t st) {
    if (nsys <= 0) return;
    const size_t per_row = (size_t)S.ell_w * 12;
    const int R = per_row * 64 <= 40960 ? 64 : per_row * 32 <= 40960 ? 32 : per_row * 16 <= 40960 ? 16
                  : per_row * 8 <= 40960 ? 8 : 0;
    if (R == 0) throw Error{WFQ_EINVAL, "neighbour lists too long for the sparse product"};
    if (R == 64) launch_spmm_rows<double, 64, true>(S, Yp, ld, sys, nsys, z, V, V, jsrc, jdst, true, st);
    else if (R == 32) launch_spmm_rows<double, 32, true>(S, Yp, ld, sys, nsys, z, V, V, jsrc, jdst, true, st);
    else if (R == 16) launch_spmm_rows<double, 16, true>(S, Yp, ld, sys, nsys, z, V, V, jsrc, jdst, true, st);
    else launch_spmm_rows<double, 8, true>(S, Yp, ld, sys, nsys, z, V, V, jsrc, jdst, true, st);
    WFQ_CHECK_LAUNCH();
}

void reduce_dots(int64_t n, const int* sys, int nsys, int j, const double2* partial, int mdim, double2* h,
                 hipStream_t st, const int* active) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(reduce_dots_kernel, dim3(nsys), dim3(128), 0, st, sys, j, partial, mdim, wave_chunks(n), h,
                       active);
    WFQ_CHECK_LAUNCH();
}

void tri_solve(const int* sys, int nsys, const int* ksteps, int mdim, const double2* R, const double2* g,
               double2* y, hipStream_t st) {
    if (nsys <= 0) return;
    if (mdim > 257) throw Error{WFQ_EINVAL, "restart length above 256 is not supported"};
    hipLaunchKernelGGL(tri_solve_kernel, dim3(nsys), dim3(64), 0, st, sys, ksteps, mdim, R, g, y);
    WFQ_CHECK_LAUNCH();
}

void x_update(const Basis& V, const Basis& x, int64_t n, const int* sys, int nsys, const int* ksteps,
              const double2* y, int mdim, hipStream_t st) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)((n + 255) / 256), (unsigned)nsys);
    hipLaunchKernelGGL(x_update_kernel, grd, dim3(256), 0, st, V, x, n, sys, ksteps, y, mdim);
    WFQ_CHECK_LAUNCH();
}

void residual(const Structure& S, const double* Y, int64_t ld, const int* sys, int nsys, const double2* z,
              const Basis& x, const double* b, const int* dir, const Basis& V, double* norm2, int nblk,
              double* qtq, hipStream_t st) {
    if (nsys <= 0) return;
    if (nblk > 65535) throw Error{WFQ_EINVAL, "residual: more row blocks than the grid's y dimension holds"};
    dim3 grd((unsigned)nsys, (unsigned)nblk);
    hipLaunchKernelGGL(residual_kernel, grd, dim3(256), 0, st, S.n, S.npad, S.ell_w, S.ell_col, S.ell_val, Y, ld, sys,
                       z, x, b, dir, V, norm2, nblk, qtq);
    WFQ_CHECK_LAUNCH();
}

void sumsq(const int* sys, int nsys, const double* norm2, int nb, double* out, hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(sumsq_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, sys, nsys, norm2, nb, out);
    WFQ_CHECK_LAUNCH();
}

void copy_rhs(const Structure& S, const int* sys, int nsys, const double* b, const int* dir, const Basis& V,
              double* norm2, int nblk, hipStream_t st) {
    if (nsys <= 0) return;
    dim3 grd((unsigned)nblk, (unsigned)nsys);
    hipLaunchKernelGGL(copy_rhs_kernel, grd, dim3(256), 0, st, S.n, sys, b, dir, V, norm2, nblk);
    WFQ_CHECK_LAUNCH();
}

void observables(const Structure& S, const int* sys, int nsys, const Basis& x, double E0, double2* alpha,
                 hipStream_t st) {
    if (nsys <= 0) return;
    hipLaunchKernelGGL(observables_kernel, dim3(nsys), dim3(256), 0, st, S.n, S.npad, S.pos, sys, x, E0, alpha);
    WFQ_CHECK_LAUNCH();
}

void scatter_q(const Structure& S, const int32_t* perm, const int* sys, int nsys, const Basis& x, double* q_re,
               double* q_im, hipStream_t st) {
    if (nsys <= 0 || (!q_re && !q_im)) return;
    dim3 grd((unsigned)((S.n + 255) / 256), (unsigned)nsys);
    hipLaunchKernelGGL(scatter_kernel, grd, dim3(256), 0, st, S.n, perm, sys, x, q_re, q_im);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
