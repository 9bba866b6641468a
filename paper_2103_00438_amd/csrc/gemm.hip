// Block products Y = T X with the stored damped Coulomb matrix (the dense half of the operator
// A = (Kbar - P) D of Eq. (a-matrix-product); arXiv 2103.00438). T is symmetric, so each output
// column is a row-times-row product: Y[c][i] = sum_k T[i][k] X[c][k]. Both operands are contiguous
// along k, which is the layout the matrix cores want.
//
// Wide blocks (many Krylov columns) run on MFMA: FP64 v_mfma_f64_16x16x4, FP32 v_mfma_f32_16x16x4,
// BF16 v_mfma_f32_16x16x32 (FP32 accumulation). A work-group (4 or 8 waves) owns a BM x BN output
// tile, stages 64-, 128- or 256-byte k-slices of its X rows and T rows in LDS (double buffered,
// rows padded by 16 bytes so that each group of 8 lanes reading 16 bytes covers all 32 banks) and
// each wave computes a (16 WM) x (16 WN) sub-tile. Each lane feeds the matrix core 16 bytes of k per operand; the k
// order inside a slice is a permutation that is the same for both operands, so the sum is exact.
// Narrow blocks (<= 8 columns, e.g. one frequency at a time) stream T once with vector loads.
#include <cstring>
#include <iterator>

#include "common.h"
#include "device_util.h"

namespace wfq {

namespace {

template <int P>
struct Prec;
template <>
struct Prec<WFQ_PREC_FP64> {
    using elem = double;
    using out = double;
    using acc = doublex4;
    using sacc = double;
};
template <>
struct Prec<WFQ_PREC_FP32> {
    using elem = float;
    using out = float;
    using acc = floatx4;
    using sacc = float;
};
template <>
struct Prec<WFQ_PREC_BF16> {
    using elem = uint16_t;
    using out = float;
    using acc = floatx4;
    using sacc = float;
};

__device__ inline void mma(doublex4& c, const u32x4& a, const u32x4& b) {
    double a0 = __hiloint2double(a.y, a.x), a1 = __hiloint2double(a.w, a.z);
    double b0 = __hiloint2double(b.y, b.x), b1 = __hiloint2double(b.w, b.z);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c, 0, 0, 0);
}

template <int P>
__device__ inline void mma(floatx4& c, const u32x4& a, const u32x4& b);

template <>
__device__ inline void mma<WFQ_PREC_FP32>(floatx4& c, const u32x4& a, const u32x4& b) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
}

template <>
__device__ inline void mma<WFQ_PREC_BF16>(floatx4& c, const u32x4& a, const u32x4& b) {
    bf16x8 av = __builtin_bit_cast(bf16x8, a);
    bf16x8 bv = __builtin_bit_cast(bf16x8, b);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}

// Element-outer issue order: for each k element, one MFMA into every accumulator in turn, so
// consecutive MFMAs never depend on each other.
template <int P, int WM, int WN, typename A>
__device__ inline void mma_block_interleaved(A (&acc)[WM][WN], const u32x4 (&af)[WM], const u32x4 (&bf)[WN]) {
    if constexpr (P == WFQ_PREC_FP32) {
        float a[WM][4], b[WN][4];
#pragma unroll
        for (int x = 0; x < WM; ++x) {
            a[x][0] = __uint_as_float(af[x].x); a[x][1] = __uint_as_float(af[x].y);
            a[x][2] = __uint_as_float(af[x].z); a[x][3] = __uint_as_float(af[x].w);
        }
#pragma unroll
        for (int y = 0; y < WN; ++y) {
            b[y][0] = __uint_as_float(bf[y].x); b[y][1] = __uint_as_float(bf[y].y);
            b[y][2] = __uint_as_float(bf[y].z); b[y][3] = __uint_as_float(bf[y].w);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int x = 0; x < WM; ++x)
#pragma unroll
                for (int y = 0; y < WN; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x][e], b[y][e], acc[x][y], 0, 0, 0);
    } else if constexpr (P == WFQ_PREC_FP64) {
        double a[WM][2], b[WN][2];
#pragma unroll
        for (int x = 0; x < WM; ++x) {
            a[x][0] = __hiloint2double(af[x].y, af[x].x);
            a[x][1] = __hiloint2double(af[x].w, af[x].z);
        }
#pragma unroll
        for (int y = 0; y < WN; ++y) {
            b[y][0] = __hiloint2double(bf[y].y, bf[y].x);
            b[y][1] = __hiloint2double(bf[y].w, bf[y].z);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int x = 0; x < WM; ++x)
#pragma unroll
                for (int y = 0; y < WN; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x][e], b[y][e], acc[x][y], 0, 0, 0);
    } else {
#pragma unroll
        for (int x = 0; x < WM; ++x)
#pragma unroll
            for (int y = 0; y < WN; ++y) mma<P>(acc[x][y], af[x], bf[y]);
    }
}

template <int P, typename A>
__device__ inline void mma_any(A& c, const u32x4& a, const u32x4& b) {
    if constexpr (P == WFQ_PREC_FP64)
        mma(c, a, b);
    else
        mma<P>(c, a, b);
}

constexpr int kRowStride = 144;  // bytes per staged row (128 data + 16 pad)

// Map a linear work-group id to a (m-tile, n-tile) pair so that the work-groups dispatched to one
// XCD (ids congruent mod 8) get a contiguous run of tiles, m fastest: the m-tiles that share one
// slab of T rows then run on the same XCD and reuse it from that XCD's L2.
__device__ inline int xcd_logical(int b, int total) {
    int xcd = b & 7, slot = b >> 3;
    int q = total >> 3, r = total & 7;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// KB = bytes of k staged per row and stage (64, 128 or 256); rows are padded by 16 bytes in LDS.
//
// Split k: with split > 1 the k range is cut into `split` equal parts and each (m-tile, part,
// n-tile) is one work-group, m fastest, so the m-tiles that share one slab of T and one k part
// stay adjacent (same XCD, same time) and T is still read once. Part 0 writes Y, part p > 0 writes
// its partial tile to ws + (p - 1) * mrows * ld in the layout of Y; split_reduce_kernel then adds
// the parts to Y in part order (a fixed summation order, so results are reproducible).
template <int P, int WM, int WN, int WAVES_M, int WAVES_N, int KB, int OCC, int ILV>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N, OCC)
    tx_mfma_kernel(const typename Prec<P>::elem* __restrict__ X, const typename Prec<P>::elem* __restrict__ T,
                   typename Prec<P>::out* __restrict__ Y, int64_t ld, int ncol, int mt_count, int nt_count, int split,
                   typename Prec<P>::out* __restrict__ ws) {
    using elem = typename Prec<P>::elem;
    using acc_t = typename Prec<P>::acc;
    constexpr int NT = 64 * WAVES_M * WAVES_N;
    constexpr int BM = 16 * WM * WAVES_M;
    constexpr int BN = 16 * WN * WAVES_N;
    constexpr int ROWS = BM + BN;
    constexpr int CH = KB / 16;          // 16-byte chunks per staged row
    constexpr int RS = KB + 16;          // padded LDS row stride
    constexpr int TOTAL = ROWS * CH;     // 16-byte chunks per stage
    constexpr int PER_T = (TOTAL + NT - 1) / NT;
    // chunk u of this thread exists (only the last one can be missing)
#define WFQ_CHUNK_OK(u) (TOTAL % NT == 0 || (u) < PER_T - 1 || r0 + (u) * RSTEP < ROWS)
    __shared__ __attribute__((aligned(16))) char lds[2 * ROWS * RS];

    const int logical = xcd_logical(blockIdx.x, mt_count * nt_count * split);
    const int mt = logical % mt_count;
    const int part = (logical / mt_count) % split;
    const int nt = logical / (mt_count * split);
    const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;

    // chunk u of this thread: row r0 + u * RSTEP (X rows first, then T rows), byte column cc * 16
    static_assert(NT % CH == 0, "whole rows per pass");
    constexpr int RSTEP = NT / CH;
    const int r0 = tid / CH, cc = tid % CH;
    const int64_t ldb = ld * (int64_t)sizeof(elem);
    const char* xb = reinterpret_cast<const char*>(X) + m0 * ldb + cc * 16;
    const char* tb = reinterpret_cast<const char*>(T) + n0 * ldb + cc * 16;
    const int dst0 = r0 * RS + cc * 16;
    // A missing last chunk re-reads the last row, and X rows past the last column (the tile can
    // be wider than the rows the caller holds) re-read the last column: loads stay unconditional
    // and in bounds; what they feed lands only in Y rows >= ncol, which are not stored.
    const int xlast = ncol - 1 - (int)m0;
    auto src_of = [&](int u) {
        const int row = min(r0 + u * RSTEP, ROWS - 1);
        return row < BM ? xb + min(row, xlast) * ldb : tb + (row - BM) * ldb;
    };

    acc_t acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int nk_all = (int)(ld * (int64_t)sizeof(elem) / KB);
    const int kb = (int)((int64_t)nk_all * part / split), ke = (int)((int64_t)nk_all * (part + 1) / split);
    u32x4 reg[PER_T];
#pragma unroll
    for (int u = 0; u < PER_T; ++u)
        reg[u] = *reinterpret_cast<const u32x4*>(src_of(u) + (int64_t)kb * KB);
#pragma unroll
    for (int u = 0; u < PER_T; ++u)
        if (WFQ_CHUNK_OK(u)) *reinterpret_cast<u32x4*>(lds + dst0 + u * RSTEP * RS) = reg[u];
    __syncthreads();

    const int frag_row = lane & 15, frag_chunk = lane >> 4;
    for (int kt = kb; kt < ke; ++kt) {
        // prefetch the next k-step (the last step re-reads its own: loads stay unconditional, so
        // the staging registers live in VGPRs across the MFMA block instead of going to scratch)
        {
            const int64_t off = (int64_t)min(kt + 1, ke - 1) * KB;
#pragma unroll
            for (int u = 0; u < PER_T; ++u)
                reg[u] = *reinterpret_cast<const u32x4*>(src_of(u) + off);
        }
        // keep the loads ahead of the MFMA block: issued late, their latency is not hidden
        __builtin_amdgcn_sched_barrier(0);
        const char* L = lds + ((kt - kb) & 1) * ROWS * RS;
#pragma unroll
        for (int cg = 0; cg < CH / 4; ++cg) {
            u32x4 af[WM], bf[WN];
            const int coff = (cg * 4 + frag_chunk) * 16;
#pragma unroll
            for (int a = 0; a < WM; ++a)
                af[a] = *reinterpret_cast<const u32x4*>(L + (wm * 16 * WM + a * 16 + frag_row) * RS + coff);
#pragma unroll
            for (int b = 0; b < WN; ++b)
                bf[b] = *reinterpret_cast<const u32x4*>(L + (BM + wn * 16 * WN + b * 16 + frag_row) * RS + coff);
            if constexpr (ILV) {
                mma_block_interleaved<P, WM, WN>(acc, af, bf);
            } else {
#pragma unroll
                for (int a = 0; a < WM; ++a)
#pragma unroll
                    for (int b = 0; b < WN; ++b) mma_any<P>(acc[a][b], af[a], bf[b]);
            }
        }
        // the other buffer was last read in step kt - 1, which every wave left at its barrier;
        // the stores wait for the loads, so they stay behind the MFMA block
        __builtin_amdgcn_sched_barrier(0);
        {
            char* S = lds + ((kt + 1 - kb) & 1) * ROWS * RS;
#pragma unroll
            for (int u = 0; u < PER_T; ++u)
                if (WFQ_CHUNK_OK(u)) *reinterpret_cast<u32x4*>(S + dst0 + u * RSTEP * RS) = reg[u];
        }
        __syncthreads();
    }

    // Accumulator layout of one 16 x 16 block: column j = lane % 16 in every case; the row of
    // element r is 4 (lane / 16) + r for the FP32 and BF16 instructions and lane / 16 + 4 r for
    // the FP64 one.
    typename Prec<P>::out* out = part == 0 ? Y : ws + (int64_t)(part - 1) * mt_count * BM * ld;
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = P == WFQ_PREC_FP64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
                int64_t c = m0 + wm * 16 * WM + a * 16 + row;
                int64_t i = n0 + wn * 16 * WN + b * 16 + (lane & 15);
                if (c < ncol) out[c * ld + i] = acc[a][b][r];
            }
}

#undef WFQ_CHUNK_OK

// Y[q] += ws_1[q] + ws_2[q] + ... for the first `count` elements, parts added in order.
template <typename O>
__global__ void __launch_bounds__(256) split_reduce_kernel(O* __restrict__ Y, const O* __restrict__ ws,
                                                            int64_t count, int64_t stride, int parts) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    O v = Y[q];
    for (int p = 0; p < parts; ++p) v += ws[p * stride + q];
    Y[q] = v;
}

// ---- narrow blocks: each wave streams R rows of T once and keeps up to NC columns of X in registers.

__device__ inline void unpack(const u32x4& v, float (&f)[4]) {
    f[0] = __uint_as_float(v.x); f[1] = __uint_as_float(v.y); f[2] = __uint_as_float(v.z); f[3] = __uint_as_float(v.w);
}
__device__ inline void unpack(const u32x4& v, double (&f)[2]) {
    f[0] = __hiloint2double(v.y, v.x); f[1] = __hiloint2double(v.w, v.z);
}
__device__ inline void unpack(const u32x4& v, float (&f)[8]) {
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[2 * q] = __uint_as_float(w[q] << 16);
        f[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
    }
}

template <int P>
struct SkinnyVec;
template <>
struct SkinnyVec<WFQ_PREC_FP64> { static constexpr int E = 2; };
template <>
struct SkinnyVec<WFQ_PREC_FP32> { static constexpr int E = 4; };
template <>
struct SkinnyVec<WFQ_PREC_BF16> { static constexpr int E = 8; };

template <int P, int NC, int R>
__global__ void __launch_bounds__(256) tx_skinny_kernel(const typename Prec<P>::elem* __restrict__ X,
                                                        const typename Prec<P>::elem* __restrict__ T,
                                                        typename Prec<P>::out* __restrict__ Y, int64_t ld, int ncol) {
    using elem = typename Prec<P>::elem;
    using S = typename Prec<P>::sacc;
    constexpr int E = SkinnyVec<P>::E;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * R;
    S acc[R][NC];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = 0;
    for (int64_t k = (int64_t)lane * E; k < ld; k += 64 * E) {
        S xv[NC][E];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            u32x4 v = *reinterpret_cast<const u32x4*>(X + c * ld + k);
            unpack(v, xv[c]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            S tv[E];
            unpack(*reinterpret_cast<const u32x4*>(T + (row0 + r) * ld + k), tv);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int e = 0; e < E; ++e) acc[r][c] += tv[e] * xv[c][e];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            S v = acc[r][c];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
            acc[r][c] = v;
        }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < ncol)
#pragma unroll
                for (int r = 0; r < R; ++r) Y[c * ld + row0 + r] = acc[r][c];
    }
}

// ---- variant registry: every kernel shape that can compute a block product, per precision.

struct Variant {
    const char* name;
    int bm, bn;        // output tile (m = columns of Y, n = atoms); bm = 0 for the narrow kernel
    int max_ncol;      // largest ncol the variant accepts (narrow kernels hold columns in registers)
    void (*launch)(const Structure& s, const void* X, const void* T, void* Y, int64_t ld, int ncol, hipStream_t st);
};

// Number of k parts for a grid of `tiles` work-groups over nk k-steps when `slots` work-groups fit
// on the chip at once: the time is taken as proportional to (rounds of work-groups) x (k-steps per
// part), plus two k-steps per extra part for writing and adding the partial tiles. A split must
// win by 3 % and keep parts >= 8 k-steps and the partial tiles within the work-space cap.
int choose_split(int64_t tiles, int nk, int64_t slots, uint64_t part_bytes, uint64_t cap) {
    auto cost = [&](int sp) { return (double)((tiles * sp + slots - 1) / slots) * ((nk + sp - 1) / sp) + 2.0 * (sp - 1); };
    int best = 1;
    double best_cost = cost(1);
    for (int sp = 2; sp <= 8; ++sp) {
        if (nk / sp < 8 || (uint64_t)(sp - 1) * part_bytes > cap) break;
        const double c = cost(sp);
        if (c < 0.97 * best_cost) {
            best = sp;
            best_cost = c;
        }
    }
    return best;
}


template <int P, int WM, int WN, int WAVES_M, int WAVES_N, int KB, int OCC, int ILV = 0>
void launch_mfma(const Structure& s, const void* X, const void* T, void* Y, int64_t ld, int ncol, hipStream_t st) {
    constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
    constexpr int NT = 64 * WAVES_M * WAVES_N;
    using elem = typename Prec<P>::elem;
    using out = typename Prec<P>::out;
    auto kern = tx_mfma_kernel<P, WM, WN, WAVES_M, WAVES_N, KB, OCC, ILV>;
    static const int per_cu = [&] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kern), NT, 0) !=
                hipSuccess || nb < 1)
            nb = 1;
        return nb;
    }();
    const int mtc = (ncol + BM - 1) / BM, ntc = (int)(ld / BN);
    const int nk = (int)(ld * (int64_t)sizeof(elem) / KB);
    const uint64_t part_bytes = (uint64_t)mtc * BM * ld * sizeof(out);
    const uint64_t cap = s.split_fixed ? s.split_fixed_bytes : kSplitWsCap;
    const int split = choose_split((int64_t)mtc * ntc, nk, (int64_t)per_cu * device_cus(s.device), part_bytes, cap);
    out* ws = split > 1 ? static_cast<out*>(split_workspace(s, (split - 1) * part_bytes)) : nullptr;
    hipLaunchKernelGGL(kern, dim3(mtc * ntc * split), dim3(NT), 0, st, static_cast<const elem*>(X),
                       static_cast<const elem*>(T), static_cast<out*>(Y), ld, ncol, mtc, ntc, split, ws);
    if (split > 1) {
        const int64_t count = (int64_t)ncol * ld;
        hipLaunchKernelGGL(split_reduce_kernel<out>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                           static_cast<out*>(Y), ws, count, (int64_t)mtc * BM * ld, split - 1);
    }
}

template <int P, int NC, int R = 4>
void launch_skinny(const Structure&, const void* X, const void* T, void* Y, int64_t ld, int ncol, hipStream_t st) {
    using elem = typename Prec<P>::elem;
    using out = typename Prec<P>::out;
    hipLaunchKernelGGL((tx_skinny_kernel<P, NC, R>), dim3((unsigned)(ld / (4 * R))), dim3(256), 0, st,
                       static_cast<const elem*>(X), static_cast<const elem*>(T), static_cast<out*>(Y), ld, ncol);
}

template <int P>
const std::vector<Variant>& variants() {
    constexpr int OCC2 = P == WFQ_PREC_FP64 ? 1 : 2;
    static const std::vector<Variant> v = {
        {"skinny2", 0, 4, 2, launch_skinny<P, 2>},
        {"skinny4", 0, 4, 4, launch_skinny<P, 4>},
        {"skinny8", 0, 4, 8, launch_skinny<P, 8>},
        {"skinny2r8", 0, 8, 2, launch_skinny<P, 2, 8>},
        {"skinny4r8", 0, 8, 4, launch_skinny<P, 4, 8>},
        {"m32n128", 32, 128, 1 << 30, launch_mfma<P, 2, 2, 1, 4, 128, 2>},
        {"m64n128", 64, 128, 1 << 30, launch_mfma<P, 4, 2, 1, 4, 128, 2>},
        {"m128n128", 128, 128, 1 << 30, launch_mfma<P, 4, 4, 2, 2, 128, OCC2>},
        {"m128n64", 128, 64, 1 << 30, launch_mfma<P, 4, 2, 2, 2, 128, 2>},
        {"m64n256", 64, 256, 1 << 30, launch_mfma<P, 4, 4, 1, 4, 128, 1>},
        {"m128n256w8", 128, 256, 1 << 30, launch_mfma<P, 4, 4, 2, 4, 128, 1>},
        {"m256n128w8", 256, 128, 1 << 30, launch_mfma<P, 4, 4, 4, 2, 128, 1>},
        {"m128n128k256", 128, 128, 1 << 30, launch_mfma<P, 4, 4, 2, 2, 256, 1>},
        {"m64n128k256", 64, 128, 1 << 30, launch_mfma<P, 4, 2, 1, 4, 256, 1>},
        {"m128n256w8i", 128, 256, 1 << 30, launch_mfma<P, 4, 4, 2, 4, 128, 1, 1>},
        {"m256n128w8i", 256, 128, 1 << 30, launch_mfma<P, 4, 4, 4, 2, 128, 1, 1>},
        {"m64n128i", 64, 128, 1 << 30, launch_mfma<P, 4, 2, 1, 4, 128, 2, 1>},
        {"m128n64i", 128, 64, 1 << 30, launch_mfma<P, 4, 2, 2, 2, 128, 2, 1>},
        {"m64n128k256i", 64, 128, 1 << 30, launch_mfma<P, 4, 2, 1, 4, 256, 1, 1>},
    };
    return v;
}

// Wider column tiles for FP32 and BF16 (their accumulators are half the size of FP64 ones), so
// that column counts between the powers of two are not padded up to the next multiple of 128.
// the narrow matrix-free product as a block-product variant (FP64 only; T is recomputed, the stored
// copy is not read)
// (NC is the largest column count of the registry entry; the kernel is chosen by ncol)
template <int NC>
void launch_otfn(const Structure& s, const void* X, const void*, void* Y, int64_t ld, int ncol, hipStream_t st) {
    static_assert(NC == 2 || NC == 4, "narrow matrix-free registry entries take 2 or 4 columns");
    otf_narrow_f64(s, static_cast<const double*>(X), static_cast<double*>(Y), ld, ncol, device_cus(s.device), st);
}

template <int P>
const std::vector<Variant>& variants_all() {
    static const std::vector<Variant> v = [] {
        std::vector<Variant> r = variants<P>();
        if constexpr (P == WFQ_PREC_FP64) {
            r.push_back({"otfn2", 0, 4, 2, launch_otfn<2>});
            r.push_back({"otfn4", 0, 4, 4, launch_otfn<4>});
        }
        if constexpr (P != WFQ_PREC_FP64) {
            r.push_back({"m96n256w8", 96, 256, 1 << 30, launch_mfma<P, 3, 4, 2, 4, 128, 1>});
            r.push_back({"m160n256w8", 160, 256, 1 << 30, launch_mfma<P, 5, 4, 2, 4, 128, 1>});
            r.push_back({"m192n256w8", 192, 256, 1 << 30, launch_mfma<P, 6, 4, 2, 4, 128, 1>});
            r.push_back({"m192n128w8", 192, 128, 1 << 30, launch_mfma<P, 3, 4, 4, 2, 128, 1>});
            r.push_back({"m224n256w8", 224, 256, 1 << 30, launch_mfma<P, 7, 4, 2, 4, 128, 1>});
            r.push_back({"m224n128w8", 224, 128, 1 << 30, launch_mfma<P, 7, 2, 2, 4, 128, 1>});
            // 64-byte k stages: half the LDS, so two work-groups share a CU and one's matrix-core
            // work covers the other's barrier
            r.push_back({"m128n256w8k64", 128, 256, 1 << 30, launch_mfma<P, 4, 4, 2, 4, 64, 2>});
        }
        return r;
    }();
    return v;
}

const std::vector<Variant>& variants_of(int prec) {
    return prec == WFQ_PREC_FP64 ? variants_all<WFQ_PREC_FP64>()
           : prec == WFQ_PREC_FP32 ? variants_all<WFQ_PREC_FP32>() : variants_all<WFQ_PREC_BF16>();
}

int find_variant(int prec, const char* name) {
    const auto& v = variants_of(prec);
    for (size_t k = 0; k < v.size(); ++k)
        if (std::strcmp(v[k].name, name) == 0) return (int)k;
    return -1;
}

// Built-in choice when no tuning result covers ncol: the fastest shapes measured on MI355X for a
// 20 000-atom T, per precision and column count.
int default_variant(int prec, int ncol) {
    struct Pick { int upto; const char* name; };
    static const Pick f64[] = {{2, "skinny2"}, {4, "skinny4"}, {8, "skinny8"}, {32, "m32n128"}, {64, "m64n128i"},
                               {96, "m128n256w8i"}, {128, "m128n256w8"}, {192, "m64n128i"}, {256, "m128n256w8i"},
                               {320, "m64n128"}, {1 << 30, "m128n256w8i"}};
    static const Pick f32[] = {{2, "skinny2"}, {4, "skinny4r8"}, {32, "m32n128"}, {64, "m64n128k256i"},
                               {96, "m96n256w8"}, {128, "m128n256w8k64"}, {160, "m160n256w8"}, {192, "m96n256w8"},
                               {224, "m224n128w8"}, {256, "m128n256w8k64"}, {288, "m96n256w8"}, {320, "m160n256w8"},
                               {1 << 30, "m128n256w8k64"}};
    // BF16 T is 2 bytes per element: even one column streams it faster through the matrix cores
    static const Pick b16[] = {{64, "m64n128i"}, {128, "m128n128"}, {192, "m192n256w8"}, {256, "m256n128w8i"},
                               {320, "m160n256w8"}, {1 << 30, "m192n256w8"}};
    const Pick* t = prec == WFQ_PREC_FP64 ? f64 : prec == WFQ_PREC_FP32 ? f32 : b16;
    while (ncol > t->upto) ++t;
    const int k = find_variant(prec, t->name);
    return k >= 0 ? k : find_variant(prec, "m128n256w8");   // present for every precision
}

// padded size from which untuned narrow FP64 products are recomputed rather than streamed
constexpr int64_t kOtfNarrowFrom = 16384;
// matrix-free FP64 products of up to this many 4-column chunks use the narrow kernel
constexpr int kOtfNarrowChunks = 3;

int pick_variant(const Structure& s, int prec, int ncol) {
    const auto& tuned = s.tuned[prec];
    // the tuned entry with the smallest ncol >= this one (or the largest tuned one), used only when
    // it was tuned for a comparable width (within a factor of two)
    auto it = tuned.lower_bound(ncol);
    if (it == tuned.end() && !tuned.empty()) it = std::prev(tuned.end());
    if (it != tuned.end() && it->first <= 2 * ncol && ncol <= 2 * it->first) {
        const Variant& v = variants_of(prec)[it->second];
        if (ncol <= v.max_ncol) return it->second;
    }
    // narrow FP64 products of large structures: recomputing the elements on the vector ALUs
    // (about 16 FP64 operations per pair) beats streaming 8 bytes per pair of the stored copy
    if (prec == WFQ_PREC_FP64 && ncol <= 4 && s.npad >= kOtfNarrowFrom)
        return find_variant(prec, ncol <= 2 ? "otfn2" : "otfn4");
    return default_variant(prec, ncol);
}

void run_variant(const Structure& s, int prec, int var, const void* X, void* Y, int ncol, hipStream_t st) {
    const void* T = prec == WFQ_PREC_FP64 ? (const void*)s.T64 : prec == WFQ_PREC_FP32 ? (const void*)s.T32
                                                                                       : (const void*)s.T16;
    if (T == nullptr) throw Error{WFQ_EINVAL, "the stored copy of T for this precision was not built"};
    const Variant& v = variants_of(prec)[var];
    if (ncol > v.max_ncol) throw Error{WFQ_EINVAL, "kernel variant cannot take that many columns"};
    v.launch(s, X, T, Y, s.npad, ncol, st);
    WFQ_CHECK_LAUNCH();
}

template <typename E>
__global__ void convert_kernel(const double* __restrict__ src, E* __restrict__ dst, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) dst[i] = cast_from_double<E>(src[i]);
}

}  // namespace

int device_cus(int device) {
    int cus = 0;
    WFQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    return cus > 0 ? cus : 1;
}

void* split_workspace(const Structure& s, uint64_t bytes) {
    if (s.split_fixed) {
        // a caller-provided region (the allocation-free entry point): never allocate
        if (bytes > s.split_fixed_bytes) throw Error{WFQ_ENOMEM, "split-k partial tiles exceed the fixed work space"};
        return s.split_fixed;
    }
    if (bytes > s.split_ws_bytes) {
        if (s.split_ws) {
            WFQ_HIP(hipFree(s.split_ws));
            s.split_ws = nullptr;
            s.split_ws_bytes = 0;
        }
        ++s.epoch;
        hipError_t e = hipMalloc(&s.split_ws, bytes);
        if (e != hipSuccess) throw Error{WFQ_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
        s.split_ws_bytes = bytes;
    }
    return s.split_ws;
}

void convert_from_f64(int prec, const double* src, void* dst, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    dim3 grd((unsigned)((count + 255) / 256));
    if (prec == WFQ_PREC_FP64)
        WFQ_HIP(hipMemcpyAsync(dst, src, count * 8, hipMemcpyDeviceToDevice, st));
    else if (prec == WFQ_PREC_FP32)
        hipLaunchKernelGGL(convert_kernel<float>, grd, dim3(256), 0, st, src, static_cast<float*>(dst), count);
    else
        hipLaunchKernelGGL(convert_kernel<uint16_t>, grd, dim3(256), 0, st, src, static_cast<uint16_t*>(dst), count);
    WFQ_CHECK_LAUNCH();
}

void tx_f64(const Structure& s, const double* X, double* Y, int ncol, hipStream_t st) {
    if (ncol > 0) run_variant(s, WFQ_PREC_FP64, pick_variant(s, WFQ_PREC_FP64, ncol), X, Y, ncol, st);
}
void tx_f32(const Structure& s, const float* X, float* Y, int ncol, hipStream_t st) {
    if (ncol > 0) run_variant(s, WFQ_PREC_FP32, pick_variant(s, WFQ_PREC_FP32, ncol), X, Y, ncol, st);
}
void tx_bf16(const Structure& s, const uint16_t* X, float* Y, int ncol, hipStream_t st) {
    if (ncol > 0) run_variant(s, WFQ_PREC_BF16, pick_variant(s, WFQ_PREC_BF16, ncol), X, Y, ncol, st);
}

void tx_any(const Structure& s, int prec, const void* X, void* Y, int ncol, hipStream_t st) {
    if (s.t_mode == WFQ_TMODE_OTF) {
        if (prec == WFQ_PREC_FP32)
            otf_tx_f32(s, static_cast<const float*>(X), static_cast<float*>(Y), ncol, st);
        else if (prec == WFQ_PREC_FP64 && ncol <= kOtfNarrowChunks * 4)
            // up to 16 columns: narrow recomputed products of at most 4 columns each (each such product
            // costs about what one 32-column matrix-core pass costs for 12 or more columns)
            for (int c0 = 0; c0 < ncol; c0 += 4)
                otf_narrow_f64(s, static_cast<const double*>(X) + (int64_t)c0 * s.npad,
                               static_cast<double*>(Y) + (int64_t)c0 * s.npad, s.npad, std::min(4, ncol - c0),
                               device_cus(s.device), st);
        else if (prec == WFQ_PREC_FP64)
            otf_tx_f64(s, static_cast<const double*>(X), static_cast<double*>(Y), ncol, st);
        else
            throw Error{WFQ_EINVAL, "matrix-free T runs in FP32 or FP64"};
        return;
    }
    if (prec == WFQ_PREC_FP64)
        tx_f64(s, static_cast<const double*>(X), static_cast<double*>(Y), ncol, st);
    else if (prec == WFQ_PREC_FP32)
        tx_f32(s, static_cast<const float*>(X), static_cast<float*>(Y), ncol, st);
    else
        tx_bf16(s, static_cast<const uint16_t*>(X), static_cast<float*>(Y), ncol, st);
}

void tx_variant_run(const Structure& s, int prec, int var, const void* X, void* Y, int ncol, hipStream_t st) {
    if (ncol > 0) run_variant(s, prec, var, X, Y, ncol, st);
}

bool tx_is_otf_narrow(const Structure& s, int prec, int ncol) {
    if (prec != WFQ_PREC_FP64) return false;
    if (s.t_mode == WFQ_TMODE_OTF) return ncol <= kOtfNarrowChunks * 4;
    if (ncol > 4) return false;
    return std::strncmp(variants_of(prec)[pick_variant(s, prec, ncol)].name, "otfn", 4) == 0;
}

const char* tx_variant(int precision, int ncol) {
    return variants_of(precision)[default_variant(precision, ncol)].name;
}

int tx_variant_count(int precision) { return (int)variants_of(precision).size(); }
const char* tx_variant_name(int precision, int k) { return variants_of(precision)[k].name; }
int tx_variant_max_ncol(int precision, int k) { return variants_of(precision)[k].max_ncol; }

// Time every variant that accepts ncol (reps launches each, after one warm-up launch) on random
// device data and keep the fastest for this ncol in s.tuned. ms[k] = average time of variant k
// (negative when the variant does not apply).
void tune_tx(Structure& s, int prec, int ncol, int reps, double* ms, hipStream_t st) {
    const int64_t rows = round_up(ncol, kColPad);
    const int es = prec == WFQ_PREC_FP64 ? 8 : prec == WFQ_PREC_FP32 ? 4 : 2;
    const int os = prec == WFQ_PREC_FP64 ? 8 : 4;
    void *X = nullptr, *Y = nullptr;
    double* X64 = nullptr;
    WFQ_HIP(hipMalloc(&X, rows * s.npad * es));
    WFQ_HIP(hipMalloc(&Y, rows * s.npad * os));
    WFQ_HIP(hipMalloc(&X64, rows * s.npad * 8));
    {
        std::vector<double> h(rows * s.npad, 0.0);
        uint64_t state = 0x9E3779B97F4A7C15ull * (uint64_t)(ncol + 1);
        for (int64_t c = 0; c < ncol; ++c)
            for (int64_t i = 0; i < s.n; ++i) {
                state = state * 6364136223846793005ull + 1442695040888963407ull;
                h[c * s.npad + i] = (double)(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
            }
        h2d_sync(s, X64, h.data(), h.size() * 8, st);
        WFQ_HIP(hipStreamSynchronize(st));
    }
    convert_from_f64(prec, X64, X, rows * s.npad, st);
    hipEvent_t a, b;
    WFQ_HIP(hipEventCreate(&a));
    WFQ_HIP(hipEventCreate(&b));
    const auto& vs = variants_of(prec);
    double best = 1e300;
    int best_k = -1;
    for (size_t k = 0; k < vs.size(); ++k) {
        ms[k] = -1.0;
        if (ncol > vs[k].max_ncol || (vs[k].bm == 0 && ncol > vs[k].max_ncol)) continue;
        run_variant(s, prec, (int)k, X, Y, ncol, st);
        WFQ_HIP(hipEventRecord(a, st));
        for (int r = 0; r < reps; ++r) run_variant(s, prec, (int)k, X, Y, ncol, st);
        WFQ_HIP(hipEventRecord(b, st));
        WFQ_HIP(hipEventSynchronize(b));
        float t = 0.f;
        WFQ_HIP(hipEventElapsedTime(&t, a, b));
        ms[k] = t / reps;
        if (ms[k] < best) {
            best = ms[k];
            best_k = (int)k;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(X);
    (void)hipFree(Y);
    (void)hipFree(X64);
    if (best_k >= 0) s.tuned[prec][ncol] = best_k;
    ++s.epoch;
}

}  // namespace wfq
