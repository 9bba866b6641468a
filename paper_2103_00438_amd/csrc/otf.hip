// Matrix-free block products Y = T X: the damped Coulomb elements of Eq. (d-matrix) are recomputed
// in every product instead of being stored (arXiv 2103.00438, subsection "Large systems": the
// on-the-fly matrix-vector product). The sparse half L is still applied from its stored rows.
//
// A work-group owns BI = 128 target atoms and BC columns of X. It walks over the sources in tiles of
// BJ atoms; per tile it stages the source positions (relative to the centre of its target block,
// so that coordinate differences keep full relative precision in FP32) and the X tile in LDS,
// evaluates the T tile on the vector ALUs, and accumulates the tile product on the matrix cores
// (the same fragment layout as the stored-T kernels). Tile sums are added to the running sum with
// Kahan compensation, so the FP32 result does not drift over ~10^4 source tiles.
//
// FP32 elements use erf(x) = 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p x) (Abramowitz &
// Stegun, Handbook of Mathematical Functions, formula 7.1.26; absolute error <= 1.5e-7) for
// x >= 1/2 and the Maclaurin series of erf below; FP64 elements use the device library's erf.
#include <algorithm>

#include "common.h"
#include "device_util.h"

namespace wfq {

namespace {

constexpr int kBI = 128;   // targets per work-group (4 waves x 32)

__device__ inline float erf_f32(float x) {
    if (x < 0.5f) {
        const float x2 = x * x;
        // 2/sqrt(pi) * (x - x^3/3 + x^5/10 - x^7/42 + x^9/216 - x^11/1320 + x^13/9360)
        float p = 1.2055332981789664e-4f;
        p = p * x2 - 8.5483270234508645e-4f;
        p = p * x2 + 5.2239776254421878e-3f;
        p = p * x2 - 2.6866170645131252e-2f;
        p = p * x2 + 1.1283791670955126e-1f;
        p = p * x2 - 3.7612638903183752e-1f;
        p = p * x2 + 1.1283791670955126f;
        return x * p;
    }
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
    float p = 1.061405429f;
    p = p * t - 1.453152027f;
    p = p * t + 1.421413741f;
    p = p * t - 0.284496736f;
    p = p * t + 0.254829592f;
    p = p * t;
    return 1.0f - p * __expf(-x * x);
}

template <int P>
struct OtfT;
template <>
struct OtfT<WFQ_PREC_FP32> {
    using elem = float;
    using acc = floatx4;
    using vec4 = floatx4;           // (x, y, z, d^2) of one source atom
    static constexpr int BJ = 64;   // 256-byte rows
};
template <>
struct OtfT<WFQ_PREC_FP64> {
    using elem = double;
    using acc = doublex4;
    using vec4 = doublex4;
    static constexpr int BJ = 32;
};

__device__ inline void mma_otf(floatx4& c, const uint4& a, const uint4& b) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
}
__device__ inline void mma_otf(doublex4& c, const uint4& a, const uint4& b) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(__hiloint2double(a.y, a.x), __hiloint2double(b.y, b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(__hiloint2double(a.w, a.z), __hiloint2double(b.w, b.z), c, 0, 0, 0);
}

// 1 / r_ij, the far-field value of T_ij
__device__ inline float inv_dist(float xi, float yi, float zi, float xj, float yj, float zj) {
    const float dx = xi - xj, dy = yi - yj, dz = zi - zj;
    return __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
}
__device__ inline double inv_dist(double xi, double yi, double zi, double xj, double yj, double zj) {
    const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
    return 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
}

// T_ij for one pair from coordinates relative to a common centre
__device__ inline float t_elem(float xi, float yi, float zi, float di2, float xj, float yj, float zj, float dj2) {
    const float dx = xi - xj, dy = yi - yj, dz = zi - zj;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float inv_r = __builtin_amdgcn_rsqf(r2);
    const float x = r2 * inv_r * __builtin_amdgcn_rsqf(di2 + dj2);
    return erf_f32(x) * inv_r;
}
__device__ inline double t_elem(double xi, double yi, double zi, double di2, double xj, double yj, double zj,
                                double dj2) {
    const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    return erf(r / sqrt(di2 + dj2)) / r;
}

// Far-field test of a (target block, source tile) pair from the bounding spheres of their 64-atom
// blocks: true when every pair is at least rfar apart, i.e. erf(r / sqrt(d_i^2 + d_j^2)) rounds to 1
// in the element precision (rfar = 4.5 sqrt(2) d_max for FP32, erfc(4.5) = 2e-10; 6 sqrt(2) d_max for
// FP64, erfc(6) = 2e-17), so T_ij = 1 / r_ij exactly as the full evaluation would round it.
__device__ inline bool far_apart(const double* __restrict__ sph, int64_t bt, int64_t bs, double rfar) {
    const double* a = sph + bt * 4;
    const double* b = sph + bs * 4;
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz) - a[3] - b[3] >= rfar;
}

template <int P, int BC>
__global__ void __launch_bounds__(256) otf_kernel(int64_t n, int64_t npad, const double* __restrict__ pos,
                                                  const double* __restrict__ width, const double* __restrict__ eta,
                                                  const double* __restrict__ sphere, double rfar,
                                                  const typename OtfT<P>::elem* __restrict__ X,
                                                  typename OtfT<P>::elem* __restrict__ Y) {
    using E = typename OtfT<P>::elem;
    using acc_t = typename OtfT<P>::acc;
    constexpr int BJ = OtfT<P>::BJ;
    constexpr int KB = BJ * (int)sizeof(E);   // 256 bytes of k per row
    constexpr int RS = KB + 16;
    constexpr int WM = BC / 16;               // column blocks
    constexpr int WN = 2;                     // 32 target rows per wave
    constexpr int XCH = BC * (KB / 16);       // 16-byte chunks of the X tile
    using V4 = typename OtfT<P>::vec4;
    __shared__ __attribute__((aligned(16))) char lds[(BC + kBI) * RS];
    __shared__ V4 src[BJ];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kBI;
    const int64_t c0 = (int64_t)blockIdx.y * BC;
    const int64_t ic = min(i0 + kBI / 2, n - 1);
    const double cx = pos[ic], cy = pos[npad + ic], cz = pos[2 * npad + ic];

    // this thread evaluates row `it` of the T tile, half `jh` of its columns
    const int it = tid >> 1, jh = tid & 1;
    const int64_t ti = i0 + it;
    const bool tin = ti < n;
    const E xi = tin ? (E)(pos[ti] - cx) : E(0), yi = tin ? (E)(pos[npad + ti] - cy) : E(0);
    const E zi = tin ? (E)(pos[2 * npad + ti] - cz) : E(0);
    const E di2 = tin ? (E)(width[ti] * width[ti]) : E(1);
    const E etai = tin ? (E)eta[ti] : E(0);

    acc_t sum[WM][WN], comp[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) {
            sum[a][b] = acc_t{0, 0, 0, 0};
            comp[a][b] = acc_t{0, 0, 0, 0};
        }
    char* XT = lds;
    char* TT = lds + BC * RS;
    const int frag_row = lane & 15, frag_chunk = lane >> 4;

    for (int64_t j0 = 0; j0 < npad; j0 += BJ) {
        __syncthreads();
        if (tid < BJ) {
            const int64_t j = j0 + tid;
            const bool jin = j < n;
            V4 p;
            p.x = jin ? (E)(pos[j] - cx) : E(0);
            p.y = jin ? (E)(pos[npad + j] - cy) : E(0);
            p.z = jin ? (E)(pos[2 * npad + j] - cz) : E(0);
            p.w = jin ? (E)(width[j] * width[j]) : E(1);
            src[tid] = p;
        }
        for (int q = tid; q < XCH; q += 256) {
            const int row = q / (KB / 16), cc = q % (KB / 16);
            *reinterpret_cast<uint4*>(XT + row * RS + cc * 16) =
                *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(X + (c0 + row) * npad + j0) + cc * 16);
        }
        __syncthreads();
        // T tile: row it, columns jh * BJ/2 .. + BJ/2 (zero outside the atoms, eta on the diagonal)
        E* trow = reinterpret_cast<E*>(TT + it * RS);
        const int64_t bs = j0 / 64, bt = i0 / 64;
        const bool full = tin && j0 + BJ <= n;   // no padding atom in this row of the tile
        if (far_apart(sphere, bt, bs, rfar) && far_apart(sphere, bt + 1, bs, rfar)) {
            if (full) {
#pragma unroll 8
                for (int jj = 0; jj < BJ / 2; ++jj) {
                    const int jl = jh * (BJ / 2) + jj;
                    const V4 p = src[jl];
                    trow[jl] = inv_dist(xi, yi, zi, p.x, p.y, p.z);
                }
            } else {
                for (int jj = 0; jj < BJ / 2; ++jj) {
                    const int jl = jh * (BJ / 2) + jj;
                    const V4 p = src[jl];
                    trow[jl] = (tin && j0 + jl < n) ? inv_dist(xi, yi, zi, p.x, p.y, p.z) : E(0);
                }
            }
        } else {
#pragma unroll 4
            for (int jj = 0; jj < BJ / 2; ++jj) {
                const int jl = jh * (BJ / 2) + jj;
                const int64_t j = j0 + jl;
                const V4 p = src[jl];
                E v;
                if (!tin || j >= n)
                    v = E(0);
                else if (j == ti)
                    v = etai;
                else
                    v = t_elem(xi, yi, zi, di2, p.x, p.y, p.z, p.w);
                trow[jl] = v;
            }
        }
        __syncthreads();
        acc_t tile[WM][WN];
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b) tile[a][b] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int cg = 0; cg < KB / 64; ++cg) {
            uint4 af[WM], bf[WN];
            const int coff = (cg * 4 + frag_chunk) * 16;
#pragma unroll
            for (int a = 0; a < WM; ++a) af[a] = *reinterpret_cast<const uint4*>(XT + (a * 16 + frag_row) * RS + coff);
#pragma unroll
            for (int b = 0; b < WN; ++b)
                bf[b] = *reinterpret_cast<const uint4*>(TT + (wave * 32 + b * 16 + frag_row) * RS + coff);
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int b = 0; b < WN; ++b) mma_otf(tile[a][b], af[a], bf[b]);
        }
        // compensated accumulation of the tile sums
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const E y = tile[a][b][r] - comp[a][b][r];
                    const E t = sum[a][b][r] + y;
                    comp[a][b][r] = (t - sum[a][b][r]) - y;
                    sum[a][b][r] = t;
                }
    }
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = P == WFQ_PREC_FP64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
                const int64_t c = c0 + a * 16 + row;
                const int64_t i = i0 + wave * 32 + b * 16 + (lane & 15);
                Y[c * npad + i] = sum[a][b][r];
            }
}

// ---- narrow matrix-free FP64 product: at most NC real columns (multi-shift and single-system steps)
//
// A product with a few columns is bound by the element evaluations, not by the accumulation, so
// there are no matrix-core tiles here: each thread owns TK target atoms (64 apart), evaluates T_ij
// for a run of source atoms and accumulates T_ij x_j for every column in FP64 registers. The grid's
// second dimension splits the sources into parts so that thousands of waves are in flight; each
// part's sums go to a work space and a second kernel adds the parts in order (deterministic).
// Sources come in tiles of 256 atoms (coordinates relative to the work-group's first atom, their squared
// norms and the X values staged in LDS and read by broadcast; every LDS read serves TK pairs); a tile
// far from a wave's targets takes r^2 by the expansion described below. Every pair takes the far-field value
// T_ij = 1 / r_ij (hardware reciprocal square root refined by one Newton step; 0 on the diagonal),
// with no branch; the sum kernel then adds the structure's sparse near-field correction
// C = T - 1/r (pairs closer than rfar, eta_i on the diagonal), so the result is T X.
constexpr int kNarrowTile = 256;
constexpr int kNarrowTK = 4;   // targets per thread: a work-group covers 1024 consecutive atoms
constexpr int64_t kSymFrom = 65536;   // the symmetric form from here: at least 2 080 block pairs
constexpr int kSymTK = 4;                 // symmetric form: targets per thread
constexpr int kSymBlock = 256 * kSymTK;   // atoms per block (one work-group's targets)

// Distances by expansion. Coordinates inside a work-group are taken relative to an origin o near its
// atoms. For a pair whose atoms are far apart compared with their distance from o, r^2 is expanded as
// |x_i - o|^2 + |x_j - o|^2 - 2 (x_i - o).(x_j - o): one addition and three fused multiply-adds instead of
// three subtractions, a product and two fused multiply-adds. Its rounding error grows with
// kappa = (|x_i - o|^2 + |x_j - o|^2) / r^2, so it is used only where the bounding spheres of the two
// 64-atom blocks keep kappa <= kExpKappa for every pair of their atoms (relative error of the element
// below about 4 kappa u in the worst case, u = 2^-53); other pairs take the differences. A thread holds
// its targets as a = -2 (x_i - o), from which x_i - o is recovered exactly, and |x_i - o|^2; LDS holds the
// sources' x_j - o and |x_j - o|^2.
constexpr double kExpKappa = 256.0;

// Whether the 64-atom blocks tb (targets) and sb (sources) keep kappa <= kExpKappa for every
// pair of their atoms, by their bounding spheres (centre c, radius R): with gap = |c_t - c_s| - R_t -
// R_s > 0, r >= gap and |x - o| <= |c - o| + R on each side. The radii are widened by a relative 1e-12
// for their own rounding.
__device__ inline bool expansion_ok(const double* __restrict__ sph, int64_t tb, int64_t sb, double ox, double oy,
                                    double oz) {
    const double* a = sph + tb * 4;
    const double* b = sph + sb * 4;
    const double ra = a[3] * (1.0 + 1e-12), rb = b[3] * (1.0 + 1e-12);
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    const double gap = sqrt(dx * dx + dy * dy + dz * dz) - ra - rb;
    const double ea = sqrt((a[0] - ox) * (a[0] - ox) + (a[1] - oy) * (a[1] - oy) + (a[2] - oz) * (a[2] - oz)) + ra;
    const double eb = sqrt((b[0] - ox) * (b[0] - ox) + (b[1] - oy) * (b[1] - oy) + (b[2] - oz) * (b[2] - oz)) + rb;
    return gap > 0.0 && ea * ea + eb * eb <= kExpKappa * gap * gap;
}

// The pairs of one staged source tile with this thread's TK targets. kDiag: the tile may hold one of
// the targets themselves (r = 0), whose far-field value is replaced by 0 (the diagonal is in the
// near-field correction); other tiles skip that test. kExp: r^2 by the expansion.
template <int NC, bool kDiag, bool kExp>
__device__ __forceinline__ void narrow_tile(const double* __restrict__ sx, const double* __restrict__ sy,
                                            const double* __restrict__ sz, const double* __restrict__ sn,
                                            const double (*sX)[kNarrowTile], int cnt, const double (&ax)[kNarrowTK],
                                            const double (&ay)[kNarrowTK], const double (&az)[kNarrowTK],
                                            const double (&ni)[kNarrowTK], double (&acc)[kNarrowTK][NC]) {
#pragma unroll 2
    for (int q = 0; q < cnt; ++q) {
        const double xs = sx[q], ys = sy[q], zs = sz[q];
        double xv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) xv[c] = sX[c][q];
#pragma unroll
        for (int k = 0; k < kNarrowTK; ++k) {
            double r2;
            if (kExp) {
                r2 = fma(ax[k], xs, fma(ay[k], ys, fma(az[k], zs, ni[k] + sn[q])));
            } else {
                const double dx = fma(-0.5, ax[k], -xs), dy = fma(-0.5, ay[k], -ys), dz = fma(-0.5, az[k], -zs);
                r2 = dx * dx + dy * dy + dz * dz;
            }
            double g = __builtin_amdgcn_rsq(r2);
            // one Newton step for 1/sqrt(r2): g <- g (3 - r2 g^2) / 2
            g = g * fma(-0.5 * r2, g * g, 1.5);
            if (kDiag) g = r2 > 0.0 ? g : 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[k][c] = fma(g, xv[c], acc[k][c]);
        }
    }
}

template <int NC>
__global__ void __launch_bounds__(256) otf_narrow_f64_kernel(int64_t n, int64_t npad, const double* __restrict__ pos,
                                                             const double* __restrict__ sph,
                                                             const double* __restrict__ X, int64_t ldx,
                                                             double* __restrict__ part, int64_t src_per_part) {
    constexpr int TK = kNarrowTK;
    __shared__ double sx[kNarrowTile], sy[kNarrowTile], sz[kNarrowTile], sn[kNarrowTile];
    __shared__ double sX[NC][kNarrowTile];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // targets of the work-group: [it0, it0 + 256 TK); of this thread: ib + 64 k + lane
    const int64_t it0 = (int64_t)blockIdx.x * 256 * TK;
    const int64_t ib = it0 + (int64_t)wave * 64 * TK;
    // the origin: the work-group's first atom
    const int64_t i0 = min(it0, n - 1);
    const double ox = pos[i0], oy = pos[npad + i0], oz = pos[2 * npad + i0];
    double ax[TK], ay[TK], az[TK], ni[TK];
    bool tin[TK];
    double acc[TK][NC];
#pragma unroll
    for (int k = 0; k < TK; ++k) {
        const int64_t i = ib + 64 * k + lane;
        const int64_t ii = i < npad ? i : 0;
        tin[k] = i < n;
        const double x = pos[ii] - ox, y = pos[npad + ii] - oy, z = pos[2 * npad + ii] - oz;
        ax[k] = -2.0 * x;
        ay[k] = -2.0 * y;
        az[k] = -2.0 * z;
        ni[k] = x * x + y * y + z * z;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[k][c] = 0.0;
    }
    const int64_t jb = (int64_t)blockIdx.y * src_per_part;
    const int64_t je = min(n, jb + src_per_part);   // padding sources contribute nothing
    for (int64_t j0 = jb; j0 < je; j0 += kNarrowTile) {
        // lane 4 q + k (< 16) checks the wave's target block k against the tile's source block q
        const int64_t tb = ib / 64 + (lane & 3), sb = j0 / 64 + ((lane >> 2) & 3);
        const bool ok = lane >= 16 || tb * 64 >= n || sb * 64 >= n || expansion_ok(sph, tb, sb, ox, oy, oz);
        const bool use_exp = __ballot(ok) == ~0ull;
        __syncthreads();
        {
            const int64_t j = j0 + tid;   // < npad
            const double x = pos[j] - ox, y = pos[npad + j] - oy, z = pos[2 * npad + j] - oz;
            sx[tid] = x;
            sy[tid] = y;
            sz[tid] = z;
            sn[tid] = x * x + y * y + z * z;
#pragma unroll
            for (int c = 0; c < NC; ++c) sX[c][tid] = X[c * ldx + j];
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)kNarrowTile, je - j0);
        if (j0 < it0 + 256 * TK && j0 + kNarrowTile > it0)
            narrow_tile<NC, true, false>(sx, sy, sz, sn, sX, cnt, ax, ay, az, ni, acc);
        else if (use_exp)
            narrow_tile<NC, false, true>(sx, sy, sz, sn, sX, cnt, ax, ay, az, ni, acc);
        else
            narrow_tile<NC, false, false>(sx, sy, sz, sn, sX, cnt, ax, ay, az, ni, acc);
    }
#pragma unroll
    for (int k = 0; k < TK; ++k) {
        const int64_t i = ib + 64 * k + lane;
        if (i < npad)
#pragma unroll
            for (int c = 0; c < NC; ++c) part[((int64_t)blockIdx.y * NC + c) * npad + i] = tin[k] ? acc[k][c] : 0.0;
    }
}

// Y[c][i] = sum over the source parts + sum_e C[e][i] X[c][col[e][i]] (near field). A work-group owns
// 64 rows: its 4 waves take every 4th correction entry and every 4th part (all columns of a row in one
// thread, so each entry is read once), and their sums are added in LDS in a fixed order.
template <int NC>
__global__ void __launch_bounds__(256) otf_narrow_sum_kernel(int64_t npad, int nparts, int ncol,
                                                             const double* __restrict__ part, int w,
                                                             const int32_t* __restrict__ ncolv,
                                                             const double* __restrict__ nval,
                                                             const double* __restrict__ X, int64_t ldx,
                                                             double* __restrict__ Y, int64_t ldy,
                                                             double* __restrict__ Yi) {
    __shared__ double red[4][NC][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;   // npad is a multiple of 64
    double t[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) t[c] = 0.0;
#pragma unroll 4
    for (int e = q; e < w; e += 4) {
        const double v = nval[(int64_t)e * npad + i];
        const int64_t j = ncolv[(int64_t)e * npad + i];
#pragma unroll
        for (int c = 0; c < NC; ++c) t[c] = fma(v, X[c * ldx + j], t[c]);
    }
#pragma unroll 4
    for (int p = q; p < nparts; p += 4) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < ncol) t[c] += part[((int64_t)p * NC + c) * npad + i];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) red[q][c][lane] = t[c];
    __syncthreads();
    if (q == 0) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < ncol) {
                v[c] = (red[0][c][lane] + red[1][c][lane]) + (red[2][c][lane] + red[3][c][lane]);
                Y[c * ldy + i] = v[c];
            }
        if (Yi) *reinterpret_cast<doublex4*>(Yi + 4 * i) = doublex4{v[0], v[1], v[2], v[3]};
    }
}

template <int NC>
void launch_otf_narrow(const Structure& s, const double* X, double* Y, int64_t ld, int ncol, int cus, double* Yi,
                       hipStream_t st) {
    const int64_t tblocks = (s.npad + 256 * kNarrowTK - 1) / (256 * kNarrowTK);
    // about 8 work-groups per compute unit in total, each part at least one source tile
    int nparts = (int)std::max<int64_t>(1, std::min<int64_t>((8LL * cus + tblocks - 1) / tblocks, 64));
    const int64_t per = round_up((s.npad + nparts - 1) / nparts, kNarrowTile);
    nparts = (int)((s.npad + per - 1) / per);
    double* part = static_cast<double*>(split_workspace(s, (uint64_t)nparts * NC * s.npad * sizeof(double)));
    if (!s.near_col || !s.sphere) throw Error{WFQ_EDEVICE, "the structure has no near-field correction or block spheres"};
    hipLaunchKernelGGL((otf_narrow_f64_kernel<NC>), dim3((unsigned)tblocks, (unsigned)nparts), dim3(256), 0, st, s.n,
                       s.npad, s.pos, s.sphere, X, ld, part, per);
    WFQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(otf_narrow_sum_kernel<NC>, dim3((unsigned)(s.npad / 64)), dim3(256), 0, st, s.npad, nparts,
                       ncol, part, s.near_w, s.near_col, s.near_val, X, ld, Y, ld, Yi);
    WFQ_CHECK_LAUNCH();
}

// ---- symmetric narrow product: each unordered pair of atoms evaluated once
//
// T is symmetric, so T_ij serves both rows: y_i += T_ij x_j and y_j += T_ij x_i. Atoms are grouped
// in blocks of 1 024 (the internal, Morton-cell order). One work-group per pair of blocks I <= J:
// its 256 threads own the 1 024 atoms of I (4 each, 64 apart, as in the one-sided kernel) and
// stream the atoms of J through LDS in tiles of 256. The target side accumulates in registers. For
// the source side, each wave takes the tile's sources in groups of 64 and rotates them across its
// lanes: at step t lane l pairs its targets with source (l + t) mod 64 and adds their contributions
// to that source's running sum, which then moves one lane down (l <- l + 1); after 64 steps every
// lane holds the wave's sum for its own source. The four waves' sums are added in order in LDS.
// No atomics: block K's contribution to row i is stored once, in P[K][c][i] (the target side of the
// pair (B(i), K) or the source side of (K, B(i)); a diagonal pair (I, I) computes its rows one-sided
// over all of I), and the sum kernel adds the blocks in order with the near-field correction.
// kMask: the pair involves the last block, which holds padding atoms (their contributions are 0).
// The symmetric kernel takes the origin midway between the first atoms of its two blocks, and one LDS
// row per source: x_j - o, |x_j - o|^2 and the NC columns of X, padded to an odd number of doubles so
// that the 64 lanes' rows fall in distinct LDS banks.
template <int NC>
constexpr int sym_row() { return (4 + NC) | 1; }

// One group of 64 sources against the thread's TK targets; with SIDE the source-side sums rotate as
// described above and land in red[wave][c][g + lane]. The group sits twice in a row in LDS (rows
// 2g .. 2g + 127, row 2g + 64 + q a copy of row 2g + q), so step t reads row 2g + lane + t with no
// wrap-around. The element is taken as G = y (3 - r^2 y^2), twice the Newton-refined 1/r (one
// operation fewer); the sums are halved when they are stored. EXP: r^2 by the expansion.
template <int NC, bool SIDE, bool DIAG, bool MASK, bool EXP>
__device__ __forceinline__ void sym_group(const double* __restrict__ srow, int g, int lane, int64_t j0, int64_t n,
                                          const double (&ax)[kSymTK], const double (&ay)[kSymTK],
                                          const double (&az)[kSymTK], const double (&ni)[kSymTK],
                                          const double (&xt)[kSymTK][NC], const bool (&tin)[kSymTK],
                                          double (&acc)[kSymTK][NC], double (*red)[256], int wave) {
    constexpr int ROW = sym_row<NC>();
    double ps[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) ps[c] = 0.0;
    const double* rp = srow + (2 * g + lane) * ROW;
    constexpr int kUnroll = NC <= 3 ? 4 : 2;   // measured best; 4 columns need the registers
#pragma unroll kUnroll
    for (int t = 0; t < 64; ++t) {
        const double* r = rp + t * ROW;
        const double xs = r[0], ys = r[1], zs = r[2];
        double xv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) xv[c] = r[4 + c];
        const bool sv = !MASK || j0 + g + ((lane + t) & 63) < n;
#pragma unroll
        for (int k = 0; k < kSymTK; ++k) {
            double r2;
            if (EXP) {
                r2 = fma(ax[k], xs, fma(ay[k], ys, fma(az[k], zs, ni[k] + r[3])));
            } else {
                const double dx = fma(-0.5, ax[k], -xs), dy = fma(-0.5, ay[k], -ys), dz = fma(-0.5, az[k], -zs);
                r2 = dx * dx + dy * dy + dz * dz;
            }
            double gk = __builtin_amdgcn_rsq(r2);
            gk = gk * fma(-r2, gk * gk, 3.0);
            if (DIAG) gk = r2 > 0.0 ? gk : 0.0;
            if (MASK) gk = (tin[k] && sv) ? gk : 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                acc[k][c] = fma(gk, xv[c], acc[k][c]);
                if (SIDE) ps[c] = fma(gk, xt[k][c], ps[c]);
            }
        }
        if (SIDE) {
#pragma unroll
            for (int c = 0; c < NC; ++c) ps[c] = __shfl(ps[c], (lane + 1) & 63, 64);
        }
    }
    if (SIDE) {
#pragma unroll
        for (int c = 0; c < NC; ++c) red[wave * NC + c][g + lane] = ps[c];
    }
}

// jfix < 0: the work-group index enumerates the pairs I <= J < nbt in row-major order of I;
// jfix >= 0: the pair is (blockIdx.x, jfix)
template <int NC, bool MASK>
__global__ void __launch_bounds__(256) otf_sym_kernel(int64_t n, int64_t npad, int nbt, int jfix,
                                                      const double* __restrict__ pos,
                                                      const double* __restrict__ sph, const double* __restrict__ X,
                                                      int64_t ldx, double* __restrict__ P) {
    constexpr int TK = kSymTK, TILE = 256, BS = kSymBlock, ROW = sym_row<NC>();
    __shared__ double srow[2 * TILE * ROW];   // each group of 64 twice
    __shared__ double red[4 * NC][TILE];
    int I = 0, J = 0;
    if (jfix >= 0) {
        I = blockIdx.x;
        J = jfix;
    } else {
        int64_t p = blockIdx.x;
        while (p >= nbt - I) {
            p -= nbt - I;
            ++I;
        }
        J = I + (int)p;
    }
    const bool diag = I == J;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // the origin: midpoint of the first atoms of I and J (both < n)
    const int64_t i0 = (int64_t)I * BS, j00 = min((int64_t)J * BS, n - 1);
    const double ox = 0.5 * (pos[i0] + pos[j00]), oy = 0.5 * (pos[npad + i0] + pos[npad + j00]),
                 oz = 0.5 * (pos[2 * npad + i0] + pos[2 * npad + j00]);
    // expansion flags of this wave: lane 16 t + 4 q + k checks target block k of the wave against
    // source group q of tile t; group q of tile t may use the expansion when all four of its bits are set
    uint64_t eflags = 0;
    if (!diag) {
        const int64_t tb = (i0 + wave * 64 * TK) / 64 + (lane & 3);
        const int64_t sb = (int64_t)J * BS / 64 + (lane >> 2);
        // blocks without atoms have no sphere to test; nothing of theirs is used
        const bool ok = tb * 64 >= n || sb * 64 >= n || expansion_ok(sph, tb, sb, ox, oy, oz);
        eflags = __ballot(ok);
    }
    const int64_t ib = i0 + wave * 64 * TK + lane;   // target k: ib + 64 k
    double ax[TK], ay[TK], az[TK], ni[TK], xt[TK][NC], acc[TK][NC];
    bool tin[TK];
#pragma unroll
    for (int k = 0; k < TK; ++k) {
        const int64_t i = ib + 64 * k;
        const int64_t ii = i < npad ? i : 0;
        tin[k] = i < n;
        const double x = pos[ii] - ox, y = pos[npad + ii] - oy, z = pos[2 * npad + ii] - oz;
        ax[k] = -2.0 * x;
        ay[k] = -2.0 * y;
        az[k] = -2.0 * z;
        ni[k] = x * x + y * y + z * z;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            xt[k][c] = tin[k] ? X[c * ldx + ii] : 0.0;
            acc[k][c] = 0.0;
        }
    }
    for (int t0 = 0; t0 < BS; t0 += TILE) {
        const int64_t j0 = (int64_t)J * BS + t0;
        if (j0 >= n) break;   // uniform: the rest of block J is padding
        __syncthreads();
        {
            const int64_t j = j0 + tid;
            const int64_t jj = j < npad ? j : 0;
            const int r0 = 2 * (tid & ~63) + (tid & 63);   // row of source tid, and its copy 64 later
            const double x = pos[jj] - ox, y = pos[npad + jj] - oy, z = pos[2 * npad + jj] - oz;
            double v[ROW] = {};
            v[0] = x;
            v[1] = y;
            v[2] = z;
            v[3] = x * x + y * y + z * z;
#pragma unroll
            for (int c = 0; c < NC; ++c) v[4 + c] = j < n ? X[c * ldx + jj] : 0.0;
#pragma unroll
            for (int f = 0; f < ROW; ++f) srow[r0 * ROW + f] = srow[(r0 + 64) * ROW + f] = v[f];
        }
        __syncthreads();
        for (int g = 0; g < TILE; g += 64) {
            if (MASK && j0 + g >= n) break;   // uniform: the rest of the tile is padding
            const int q = (t0 + g) / 64;
            if (diag)
                sym_group<NC, false, true, MASK, false>(srow, g, lane, j0, n, ax, ay, az, ni, xt, tin, acc, red, wave);
            else if (((eflags >> (4 * q)) & 0xF) == 0xF)
                sym_group<NC, true, false, MASK, true>(srow, g, lane, j0, n, ax, ay, az, ni, xt, tin, acc, red, wave);
            else
                sym_group<NC, true, false, MASK, false>(srow, g, lane, j0, n, ax, ay, az, ni, xt, tin, acc, red, wave);
        }
        if (!diag) {
            __syncthreads();
            const int64_t j = j0 + tid;
            if (j < npad) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double v = ((red[c][tid] + red[NC + c][tid]) + red[2 * NC + c][tid]) + red[3 * NC + c][tid];
                    P[((int64_t)I * NC + c) * npad + j] = j < n ? 0.5 * v : 0.0;
                }
            }
        }
    }
    if (!diag) {
        // rows of J at or beyond n that no tile above reached still get their zeros (same thread per row)
        for (int64_t j = (int64_t)J * BS + tid; j < (int64_t)(J + 1) * BS && j < npad; j += 256)
            if (j >= n)
#pragma unroll
                for (int c = 0; c < NC; ++c) P[((int64_t)I * NC + c) * npad + j] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < TK; ++k) {
        const int64_t i = ib + 64 * k;
        if (i < npad)
#pragma unroll
            for (int c = 0; c < NC; ++c) P[((int64_t)J * NC + c) * npad + i] = tin[k] ? 0.5 * acc[k][c] : 0.0;
    }
}

template <int NC>
void launch_otf_sym(const Structure& s, const double* X, double* Y, int64_t ld, int ncol, double* Yi, hipStream_t st) {
    const int nb = (int)((s.npad + kSymBlock - 1) / kSymBlock);
    double* P = static_cast<double*>(split_workspace(s, (uint64_t)nb * NC * s.npad * sizeof(double)));
    if (!s.near_col || !s.sphere) throw Error{WFQ_EDEVICE, "the structure has no near-field correction or block spheres"};
    // pairs within the full blocks need no masks; the pairs with the last block (which holds the
    // padding when n is not a multiple of 1024) run the masked variant
    const bool partial = (int64_t)nb * kSymBlock > s.n;
    const int nbt = partial ? nb - 1 : nb;
    const int64_t pairs = (int64_t)nbt * (nbt + 1) / 2;
    if (pairs > 0)
        hipLaunchKernelGGL((otf_sym_kernel<NC, false>), dim3((unsigned)pairs), dim3(256), 0, st, s.n, s.npad, nbt, -1,
                           s.pos, s.sphere, X, ld, P);
    if (partial)
        hipLaunchKernelGGL((otf_sym_kernel<NC, true>), dim3((unsigned)nb), dim3(256), 0, st, s.n, s.npad, nb, nb - 1,
                           s.pos, s.sphere, X, ld, P);
    WFQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(otf_narrow_sum_kernel<NC>, dim3((unsigned)(s.npad / 64)), dim3(256), 0, st, s.npad, nb, ncol,
                       P, s.near_w, s.near_col, s.near_val, X, ld, Y, ld, Yi);
    WFQ_CHECK_LAUNCH();
}

}  // namespace

uint64_t otf_sym_bytes(const Structure& s, int ncol) {
    if (s.n < kSymFrom) return 0;
    const int64_t nb = (s.npad + kSymBlock - 1) / kSymBlock;
    return (uint64_t)nb * ncol * s.npad * sizeof(double);
}

bool otf_sym_fits(const Structure& s, int ncol) {
    const uint64_t cap = s.split_fixed ? s.split_fixed_bytes : std::max(kSplitWsCap, s.sym_ws_allowed);
    return s.n >= kSymFrom && otf_sym_bytes(s, ncol) <= cap;
}

void otf_narrow_f64(const Structure& s, const double* X, double* Y, int64_t ld, int ncol, int cus, hipStream_t st,
                    double* Yi) {
    if (ncol <= 0) return;
    if (ncol > 4) throw Error{WFQ_EINVAL, "the narrow matrix-free product takes at most 4 columns"};
    if (otf_sym_fits(s, ncol)) {
        if (ncol == 1)
            launch_otf_sym<1>(s, X, Y, ld, ncol, Yi, st);
        else if (ncol == 2)
            launch_otf_sym<2>(s, X, Y, ld, ncol, Yi, st);
        else if (ncol == 3)
            launch_otf_sym<3>(s, X, Y, ld, ncol, Yi, st);
        else
            launch_otf_sym<4>(s, X, Y, ld, ncol, Yi, st);
        return;
    }
    if (ncol == 1)
        launch_otf_narrow<1>(s, X, Y, ld, ncol, cus, Yi, st);
    else if (ncol == 2)
        launch_otf_narrow<2>(s, X, Y, ld, ncol, cus, Yi, st);
    else if (ncol == 3)
        launch_otf_narrow<3>(s, X, Y, ld, ncol, cus, Yi, st);
    else
        launch_otf_narrow<4>(s, X, Y, ld, ncol, cus, Yi, st);
}

void otf_tx_f32(const Structure& s, const float* X, float* Y, int ncol, hipStream_t st) {
    if (ncol <= 0) return;
    constexpr int BC = 32;
    dim3 grd((unsigned)(s.npad / kBI), (unsigned)((ncol + BC - 1) / BC));
    const double rfar = 4.5 * std::sqrt(2.0) * s.width_max;
    hipLaunchKernelGGL((otf_kernel<WFQ_PREC_FP32, BC>), grd, dim3(256), 0, st, s.n, s.npad, s.pos, s.width, s.eta,
                       s.sphere, rfar, X, Y);
    WFQ_CHECK_LAUNCH();
}

void otf_tx_f64(const Structure& s, const double* X, double* Y, int ncol, hipStream_t st) {
    if (ncol <= 0) return;
    constexpr int BC = 32;
    dim3 grd((unsigned)(s.npad / kBI), (unsigned)((ncol + BC - 1) / BC));
    const double rfar = 6.0 * std::sqrt(2.0) * s.width_max;
    hipLaunchKernelGGL((otf_kernel<WFQ_PREC_FP64, BC>), grd, dim3(256), 0, st, s.n, s.npad, s.pos, s.width, s.eta,
                       s.sphere, rfar, X, Y);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
