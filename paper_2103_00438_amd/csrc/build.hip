// Structure set-up on the device: atom ordering, the sparse Drude Laplacian L and the dense
// damped Coulomb matrix T (arXiv 2103.00438, Section "Theoretical Model").
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.h"
#include "device_util.h"

namespace wfq {

namespace {

constexpr double kBohrA = 0.529177210903;  // Angstrom per bohr
constexpr double kCoincidentA = 1e-6;      // atoms closer than this are rejected

// Spread the low 21 bits of v so that bit b moves to bit 3b (Morton interleave helper).
uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

struct CellGrid {
    double lo[3];
    double h;       // cell edge (>= cutoff radius)
    int dim[3];
};

// ----------------------------------------------------------------------- device kernels

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

struct GridArgs {
    double lo0, lo1, lo2, inv_h;
    int d0, d1, d2;
};

__device__ inline void cell_of(const GridArgs& g, double x, double y, double z, int& cx, int& cy, int& cz) {
    cx = clampi((int)floor((x - g.lo0) * g.inv_h), 0, g.d0 - 1);
    cy = clampi((int)floor((y - g.lo1) * g.inv_h), 0, g.d1 - 1);
    cz = clampi((int)floor((z - g.lo2) * g.inv_h), 0, g.d2 - 1);
}

// 1 - f(r) of Eq. (fermi), divided by r: the off-diagonal Kbar_ij of Eq. (k-tot-factor).
__device__ inline double kbar_of(double r, double inv_sr0, double d) {
    double x = d * (r * inv_sr0 - 1.0);
    return 1.0 / ((1.0 + exp(x)) * r);
}

// Pass 1 (count=true): number of neighbours within rc per atom; pass 2: write the CSR row of
// L = P - Kbar with the diagonal first, then -Kbar_ij in cell traversal order (deterministic).
// The pair (i, j) uses r0_ij = (r0_i + r0_j) / 2 (species of the two atoms) and its own cutoff
// r_c,ij = s r0_ij cfac, cfac = 1 + ln(1/eps - 1) / d.
template <bool kCount>
__global__ void neighbour_kernel(int64_t n, const double* __restrict__ pos, int64_t npad, GridArgs g,
                                 const int32_t* __restrict__ cell_start, const int32_t* __restrict__ cell_count,
                                 const double* __restrict__ r0a, double fs, double cfac, double fd, double close2,
                                 int32_t* __restrict__ counts, const int32_t* __restrict__ rowptr,
                                 int32_t* __restrict__ col, double* __restrict__ val, int32_t* __restrict__ flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* px = pos;
    const double* py = pos + npad;
    const double* pz = pos + 2 * npad;
    double xi = px[i], yi = py[i], zi = pz[i];
    const double r0i = r0a[i];
    int cx, cy, cz;
    cell_of(g, xi, yi, zi, cx, cy, cz);
    int cnt = 0;
    double diag = 0.0;
    int64_t base = kCount ? 0 : rowptr[i];
    int out = 1;
    for (int dz = -1; dz <= 1; ++dz) {
        int z = cz + dz;
        if (z < 0 || z >= g.d2) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int y = cy + dy;
            if (y < 0 || y >= g.d1) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                int x = cx + dx;
                if (x < 0 || x >= g.d0) continue;
                int64_t c = ((int64_t)z * g.d1 + y) * g.d0 + x;
                int s0 = cell_start[c], sc = cell_count[c];
                for (int jj = 0; jj < sc; ++jj) {
                    int j = s0 + jj;
                    if (j == i) continue;
                    double ddx = xi - px[j], ddy = yi - py[j], ddz = zi - pz[j];
                    double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    if (r2 < close2) flag[0] = 1;
                    const double sr0 = fs * 0.5 * (r0i + r0a[j]);
                    const double rc = sr0 * cfac;
                    if (r2 < rc * rc) {
                        if (kCount) {
                            ++cnt;
                        } else {
                            double k = kbar_of(sqrt(r2), 1.0 / sr0, fd);
                            diag += k;
                            col[base + out] = j;
                            val[base + out] = -k;
                            ++out;
                        }
                    }
                }
            }
        }
    }
    if (kCount) {
        counts[i] = cnt + 1;  // + diagonal
    } else {
        col[base] = (int32_t)i;
        val[base] = diag;
    }
}

// Near-field correction of the far-field element: C_ij = T_ij - 1 / r_ij for 0 < r_ij < rfar (where
// erf(r_ij / sqrt(d_i^2 + d_j^2)) is not yet 1 in FP64), C_ii = eta_i; T = 1/r (off the diagonal) + C.
// Pass 1 (kCount) writes the entries per row; pass 2 fills the transposed ELL layout [w][npad]
// (diagonal first, then the neighbours in cell traversal order; padding entries: column i, value 0).
// The search visits the cells within R = ceil(rfar / h) of the atom's cell.
template <bool kCount>
__global__ void near_kernel(int64_t n, const double* __restrict__ pos, const double* __restrict__ width,
                            const double* __restrict__ eta, int64_t npad, GridArgs g, int R,
                            const int32_t* __restrict__ cell_start, const int32_t* __restrict__ cell_count,
                            double rfar2, int32_t* __restrict__ counts, int w, int32_t* __restrict__ ecol,
                            double* __restrict__ eval) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i >= n) {
        if (!kCount)
            for (int t = 0; t < w; ++t) {
                ecol[(int64_t)t * npad + i] = 0;
                eval[(int64_t)t * npad + i] = 0.0;
            }
        return;
    }
    const double* px = pos;
    const double* py = pos + npad;
    const double* pz = pos + 2 * npad;
    const double xi = px[i], yi = py[i], zi = pz[i], di2 = width[i] * width[i];
    int cx, cy, cz;
    cell_of(g, xi, yi, zi, cx, cy, cz);
    int out = 1;
    if (!kCount) {
        ecol[i] = (int32_t)i;
        eval[i] = eta[i];
    }
    for (int dz = -R; dz <= R; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= g.d2) continue;
        for (int dy = -R; dy <= R; ++dy) {
            const int y = cy + dy;
            if (y < 0 || y >= g.d1) continue;
            for (int dx = -R; dx <= R; ++dx) {
                const int x = cx + dx;
                if (x < 0 || x >= g.d0) continue;
                const int64_t c = ((int64_t)z * g.d1 + y) * g.d0 + x;
                const int s0 = cell_start[c], sc = cell_count[c];
                for (int jj = 0; jj < sc; ++jj) {
                    const int j = s0 + jj;
                    if (j == i) continue;
                    const double ddx = xi - px[j], ddy = yi - py[j], ddz = zi - pz[j];
                    const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    if (r2 < rfar2) {
                        if (!kCount && out < w) {
                            const double r = sqrt(r2);
                            // erf(x) / r - 1 / r = -erfc(x) / r
                            ecol[(int64_t)out * npad + i] = j;
                            eval[(int64_t)out * npad + i] = -erfc(r / sqrt(di2 + width[j] * width[j])) / r;
                        }
                        ++out;
                    }
                }
            }
        }
    }
    if (kCount) {
        counts[i] = out;
    } else {
        for (int t = out; t < w; ++t) {
            ecol[(int64_t)t * npad + i] = (int32_t)i;
            eval[(int64_t)t * npad + i] = 0.0;
        }
    }
}

// largest of n counts (one block; set-up only)
__global__ void max_kernel(int64_t n, const int32_t* __restrict__ counts, int32_t* __restrict__ out) {
    __shared__ int32_t part[1024];
    int32_t m = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) m = max(m, counts[i]);
    part[threadIdx.x] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 1024; ++k) m = max(m, part[k]);
        out[0] = m;
    }
}

// Exclusive scan of n counts into rowptr[0..n] by one block (set-up only, n up to a few million).
__global__ void scan_kernel(int64_t n, const int32_t* __restrict__ counts, int32_t* __restrict__ rowptr) {
    __shared__ int64_t part[1024];
    int t = threadIdx.x;
    int64_t per = (n + 1023) / 1024;
    int64_t b = t * per, e = min(n, b + per);
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += counts[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < 1024; ++k) {
            int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        rowptr[n] = (int32_t)acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t i = b; i < e; ++i) {
        rowptr[i] = (int32_t)acc;
        acc += counts[i];
    }
}

// Dense T of Eq. (d-matrix) in FP64, stored in any of FP64 / FP32 / BF16 (row-major, ld = npad).
// Each block fills a 32 x 256 tile; padding rows/columns are written as zero.
__global__ void __launch_bounds__(256) build_T_kernel(int64_t n, int64_t npad, const double* __restrict__ pos,
                                                      const double* __restrict__ eta, const double* __restrict__ width,
                                                      double* __restrict__ T64, float* __restrict__ T32,
                                                      uint16_t* __restrict__ T16) {
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i0 = (int64_t)blockIdx.y * 32;
    const double* px = pos;
    const double* py = pos + npad;
    const double* pz = pos + 2 * npad;
    bool jin = j < n;
    double xj = jin ? px[j] : 0.0, yj = jin ? py[j] : 0.0, zj = jin ? pz[j] : 0.0;
    double dj2 = jin ? width[j] * width[j] : 0.0;
    for (int r = 0; r < 32; ++r) {
        int64_t i = i0 + r;
        double v = 0.0;
        if (i < n && jin) {
            if (i == j) {
                v = eta[i];
            } else {
                double dx = px[i] - xj, dy = py[i] - yj, dz = pz[i] - zj;
                double rr = sqrt(dx * dx + dy * dy + dz * dz);
                double di = width[i];
                v = erf(rr / sqrt(di * di + dj2)) / rr;
            }
        }
        int64_t o = i * npad + j;
        if (T64) T64[o] = v;
        if (T32) T32[o] = (float)v;
        if (T16) T16[o] = bf16_rne(v);
    }
}

// Transposed ELL copy of the CSR rows: entry t of row i at [t][i], so that consecutive rows
// (consecutive lanes) read consecutive addresses. Short rows are padded with (i, 0).
__global__ void ell_kernel(int64_t n, int64_t npad, int w, const int32_t* __restrict__ rowptr,
                           const int32_t* __restrict__ col, const double* __restrict__ val,
                           int32_t* __restrict__ ecol, double* __restrict__ eval) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    int p0 = i < n ? rowptr[i] : 0, len = i < n ? rowptr[i + 1] - p0 : 0;
    for (int t = 0; t < w; ++t) {
        ecol[(int64_t)t * npad + i] = t < len ? col[p0 + t] : (int32_t)(i < n ? i : 0);
        eval[(int64_t)t * npad + i] = t < len ? val[p0 + t] : 0.0;
    }
}

// x[i] = 1 for the atoms, 0 for the padding
__global__ void ones_kernel(int64_t n, int64_t npad, double* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npad) x[i] = i < n ? 1.0 : 0.0;
}

// b[d][i] = E0 sum_j L_ij (r_j . k_d): minus R of Eq. (r-vector-def) with V of Eq. (potential).
__global__ void rhs_kernel(int64_t n, int64_t npad, const double* __restrict__ pos, const int32_t* __restrict__ rowptr,
                           const int32_t* __restrict__ col, const double* __restrict__ val,
                           const double* __restrict__ dirs, int n_dir, double E0, double* __restrict__ out,
                           int64_t ld) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int d = blockIdx.y;
    if (i >= npad || d >= n_dir) return;
    double acc = 0.0;
    if (i < n) {
        double kx = dirs[3 * d], ky = dirs[3 * d + 1], kz = dirs[3 * d + 2];
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = col[p];
            acc += val[p] * (pos[j] * kx + pos[npad + j] * ky + pos[2 * npad + j] * kz);
        }
        acc *= E0;
    }
    out[d * ld + i] = acc;
}

template <typename T>
T* dev_alloc(Structure& s, size_t count) {
    size_t bytes = count * sizeof(T);
    if (s.budget && s.bytes + bytes > s.budget)
        throw Error{WFQ_ENOMEM, "device budget exceeded while building the structure (" +
                                    std::to_string((s.bytes + bytes) >> 20) + " MiB needed)"};
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw Error{WFQ_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    s.bytes += bytes;
    return static_cast<T*>(p);
}

}  // namespace

void free_structure(Structure& s) {
    free_solve_cache(s);
    void* ptrs[] = {s.pos, s.eta, s.width, s.rowptr, s.col, s.val, s.T64, s.T32, s.T16, s.dperm, s.ell_col, s.ell_val,
                    s.sphere, s.near_col, s.near_val, s.r0a};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    s.pos = s.eta = s.width = s.val = s.T64 = s.sphere = nullptr;
    s.rowptr = s.col = s.dperm = s.ell_col = nullptr;
    s.ell_val = nullptr;
    s.near_col = nullptr;
    s.near_val = nullptr;
    s.r0a = nullptr;
    s.T32 = nullptr;
    s.T16 = nullptr;
    if (s.split_ws) (void)hipFree(s.split_ws);
    s.split_ws = nullptr;
    s.split_ws_bytes = 0;
    if (s.pin_stage) (void)hipHostFree(s.pin_stage);
    s.pin_stage = nullptr;
    s.pin_stage_bytes = 0;
    s.bytes = 0;
}

namespace {

// Device scratch of one build step: every buffer taken is freed by release() or, on an exception,
// by the destructor (after the device work that may still use it has finished).
struct ScratchDev {
    std::vector<void*> bufs;
    template <typename T>
    T* take(int64_t count) {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, std::max<int64_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) throw Error{WFQ_ENOMEM, std::string("hipMalloc of build scratch failed: ") + hipGetErrorString(e)};
        bufs.push_back(p);
        return static_cast<T*>(p);
    }
    void release() {
        for (void* p : bufs) (void)hipFree(p);
        bufs.clear();
    }
    ScratchDev() = default;
    ScratchDev(const ScratchDev&) = delete;
    ScratchDev& operator=(const ScratchDev&) = delete;
    ~ScratchDev() {
        if (!bufs.empty()) (void)hipDeviceSynchronize();
        release();
    }
};

// the structure's pinned staging buffer, at least min(bytes, 32 MiB) long; returns its length
size_t pin_stage(const Structure& s, size_t bytes, hipStream_t st) {
    constexpr size_t kChunk = 32u << 20;
    const size_t cap = std::min(bytes, kChunk);
    if (s.pin_stage_bytes < cap) {
        if (s.pin_stage) {
            WFQ_HIP(hipStreamSynchronize(st));
            WFQ_HIP(hipHostFree(s.pin_stage));
            s.pin_stage = nullptr;
            s.pin_stage_bytes = 0;
        }
        WFQ_HIP(hipHostMalloc(&s.pin_stage, cap, hipHostMallocDefault));
        s.pin_stage_bytes = cap;
    }
    return cap;
}

}  // namespace

void d2h_sync(const Structure& s, void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) {
        WFQ_HIP(hipStreamSynchronize(st));
        return;
    }
    const size_t cap = pin_stage(s, bytes, st);
    for (size_t off = 0; off < bytes; off += cap) {
        const size_t len = std::min(cap, bytes - off);
        WFQ_HIP(hipMemcpyAsync(s.pin_stage, static_cast<const char*>(src) + off, len, hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipStreamSynchronize(st));
        std::memcpy(static_cast<char*>(dst) + off, s.pin_stage, len);
    }
}

void h2d_sync(const Structure& s, void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return;
    const size_t cap = pin_stage(s, bytes, st);
    // the staging buffer may still be the source of an earlier copy on this stream
    WFQ_HIP(hipStreamSynchronize(st));
    for (size_t off = 0; off < bytes; off += cap) {
        const size_t len = std::min(cap, bytes - off);
        std::memcpy(s.pin_stage, static_cast<const char*>(src) + off, len);
        WFQ_HIP(hipMemcpyAsync(static_cast<char*>(dst) + off, s.pin_stage, len, hipMemcpyHostToDevice, st));
        WFQ_HIP(hipStreamSynchronize(st));
    }
}

void build_structure(Structure& s, const wfq_geometry* g, const wfq_params* p, const double* eta_atom,
                     const double* r0_atom, double W, hipStream_t st) {
    const int64_t n = g->n;
    s.n = n;
    s.npad = round_up(n, kPad);
    double r0max = 0.0;
    for (int64_t i = 0; i < n; ++i) r0max = std::max(r0max, r0_atom[i]);
    s.r0 = r0max / kBohrA;   // the largest pair cutoff sets the cell grid
    s.fd = p->fermi_d;
    s.fs = p->fermi_s;
    s.cfac = 1.0 + std::log(1.0 / p->cutoff_eps - 1.0) / s.fd;
    s.rc = s.fs * s.r0 * s.cfac;
    s.W = W;
    s.tau = p->tau;

    // ---- a0: units and ordering. Atoms are grouped by cell (edge >= rc) and the cells are ordered
    // along a Morton curve, so that neighbours in space are near in memory.
    std::vector<double> xyz(3 * n);
    for (int64_t i = 0; i < 3 * n; ++i) xyz[i] = g->xyz[i] / kBohrA;
    CellGrid grid;
    double hi[3];
    for (int a = 0; a < 3; ++a) {
        grid.lo[a] = hi[a] = xyz[a];
        for (int64_t i = 1; i < n; ++i) {
            grid.lo[a] = std::min(grid.lo[a], xyz[3 * i + a]);
            hi[a] = std::max(hi[a], xyz[3 * i + a]);
        }
    }
    grid.h = s.rc * (1.0 + 1e-9);
    for (;;) {
        int64_t total = 1;
        for (int a = 0; a < 3; ++a) {
            grid.dim[a] = std::max(1, (int)std::floor((hi[a] - grid.lo[a]) / grid.h) + 1);
            total *= grid.dim[a];
        }
        if (total <= (int64_t)1 << 24 && grid.dim[0] < (1 << 21) && grid.dim[1] < (1 << 21) && grid.dim[2] < (1 << 21))
            break;
        grid.h *= 1.5;
    }
    std::vector<int64_t> cell(n);
    std::vector<uint64_t> code(n);
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        for (int a = 0; a < 3; ++a)
            c[a] = std::min(grid.dim[a] - 1, std::max(0, (int)std::floor((xyz[3 * i + a] - grid.lo[a]) / grid.h)));
        cell[i] = ((int64_t)c[2] * grid.dim[1] + c[1]) * grid.dim[0] + c[0];
        code[i] = spread3(c[0]) | spread3(c[1]) << 1 | spread3(c[2]) << 2;
    }
    s.perm.resize(n);
    std::iota(s.perm.begin(), s.perm.end(), 0);
    std::stable_sort(s.perm.begin(), s.perm.end(), [&](int64_t a, int64_t b) { return code[a] < code[b]; });
    s.iperm.resize(n);
    for (int64_t k = 0; k < n; ++k) s.iperm[s.perm[k]] = k;

    const int64_t ncell = (int64_t)grid.dim[0] * grid.dim[1] * grid.dim[2];
    std::vector<int32_t> cell_start(ncell, 0), cell_count(ncell, 0);
    for (int64_t k = n - 1; k >= 0; --k) {
        int64_t c = cell[s.perm[k]];
        cell_count[c] += 1;
        cell_start[c] = (int32_t)k;   // the atoms of one cell are contiguous in the new order
    }

    std::vector<double> pos_h(3 * s.npad, 0.0), eta_h(s.npad, 0.0), width_h(s.npad, 0.0), r0_h(s.npad, 0.0);
    s.pos_host.assign(3 * n, 0.0);
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = s.perm[k];
        for (int a = 0; a < 3; ++a) {
            pos_h[a * s.npad + k] = xyz[3 * i + a];
            s.pos_host[a * n + k] = xyz[3 * i + a];
        }
        double e = eta_atom[i];
        eta_h[k] = e;
        r0_h[k] = r0_atom[i] / kBohrA;
        width_h[k] = std::sqrt(2.0 / M_PI) / e;   // d_i = sqrt(2/pi) / eta_i (width-from-hardness)
    }

    std::vector<int32_t> perm32(s.perm.begin(), s.perm.end());
    s.dperm = dev_alloc<int32_t>(s, n);
    h2d_sync(s, s.dperm, perm32.data(), n * 4, st);
    s.pos = dev_alloc<double>(s, 3 * s.npad);
    s.eta = dev_alloc<double>(s, s.npad);
    s.width = dev_alloc<double>(s, s.npad);
    h2d_sync(s, s.pos, pos_h.data(), pos_h.size() * 8, st);
    h2d_sync(s, s.eta, eta_h.data(), eta_h.size() * 8, st);
    h2d_sync(s, s.width, width_h.data(), width_h.size() * 8, st);
    s.r0a = dev_alloc<double>(s, s.npad);
    h2d_sync(s, s.r0a, r0_h.data(), r0_h.size() * 8, st);
    // bounding spheres of consecutive 64-atom blocks (internal order; padding atoms excluded, an
    // empty block gets radius 0), used by the matrix-free products to find far-apart tile pairs
    // (the host copy lives until the stream is synchronised at the end of the build)
    std::vector<double> sph((size_t)(s.npad / 64) * 4, 0.0);
    {
        const int64_t nb = s.npad / 64;
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t k0 = b * 64, k1 = std::min<int64_t>(n, k0 + 64);
            if (k1 <= k0) continue;
            double lo[3], hi[3];
            for (int a = 0; a < 3; ++a) lo[a] = hi[a] = s.pos_host[a * n + k0];
            for (int64_t k = k0; k < k1; ++k)
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], s.pos_host[a * n + k]);
                    hi[a] = std::max(hi[a], s.pos_host[a * n + k]);
                }
            double c[3], r2 = 0.0;
            for (int a = 0; a < 3; ++a) c[a] = 0.5 * (lo[a] + hi[a]);
            for (int64_t k = k0; k < k1; ++k) {
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) d2 += (s.pos_host[a * n + k] - c[a]) * (s.pos_host[a * n + k] - c[a]);
                r2 = std::max(r2, d2);
            }
            for (int a = 0; a < 3; ++a) sph[b * 4 + a] = c[a];
            sph[b * 4 + 3] = std::sqrt(r2);
        }
        s.sphere = dev_alloc<double>(s, sph.size());
        h2d_sync(s, s.sphere, sph.data(), sph.size() * 8, st);
        s.width_max = 0.0;
        for (int64_t k = 0; k < n; ++k) s.width_max = std::max(s.width_max, width_h[k]);
    }

    // ---- a1: neighbour search and CSR of L = P - Kbar
    // scratch of the search (cell table, per-row counts, the coincident-atom flag): freed on every
    // path out of this block, the error paths included
    ScratchDev scratch;
    int32_t* d_start = scratch.take<int32_t>(ncell);
    int32_t* d_count = scratch.take<int32_t>(ncell);
    int32_t* d_counts = scratch.take<int32_t>(n);
    int32_t* d_flag = scratch.take<int32_t>(1);
    h2d_sync(s, d_start, cell_start.data(), ncell * 4, st);
    h2d_sync(s, d_count, cell_count.data(), ncell * 4, st);
    WFQ_HIP(hipMemsetAsync(d_flag, 0, 4, st));
    GridArgs ga{grid.lo[0], grid.lo[1], grid.lo[2], 1.0 / grid.h, grid.dim[0], grid.dim[1], grid.dim[2]};
    const double close = kCoincidentA / kBohrA;
    s.rowptr = dev_alloc<int32_t>(s, n + 1);
    dim3 blk(256), grd((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(neighbour_kernel<true>, grd, blk, 0, st, n, s.pos, s.npad, ga, d_start, d_count, s.r0a, s.fs,
                       s.cfac, s.fd, close * close, d_counts, nullptr, nullptr, nullptr, d_flag);
    WFQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, n, d_counts, s.rowptr);
    WFQ_CHECK_LAUNCH();
    // both scalars come back through the structure's pinned staging buffer (never a copy into
    // pageable memory such as this thread's stack)
    int32_t nnz32 = 0, flag = 0;
    d2h_sync(s, &nnz32, s.rowptr + n, 4, st);
    d2h_sync(s, &flag, d_flag, 4, st);
    if (flag) throw Error{WFQ_EINVAL, "two atoms are closer than 1e-6 Angstrom"};
    s.nnz = nnz32;
    s.col = dev_alloc<int32_t>(s, s.nnz);
    s.val = dev_alloc<double>(s, s.nnz);
    hipLaunchKernelGGL(neighbour_kernel<false>, grd, blk, 0, st, n, s.pos, s.npad, ga, d_start, d_count, s.r0a, s.fs,
                       s.cfac, s.fd, close * close, nullptr, s.rowptr, s.col, s.val, d_flag);
    WFQ_CHECK_LAUNCH();

    // connectivity of the Kbar graph (breadth-first search on the host)
    {
        std::vector<int32_t> rp(n + 1), cl(s.nnz);
        d2h_sync(s, rp.data(), s.rowptr, (n + 1) * 4, st);
        d2h_sync(s, cl.data(), s.col, s.nnz * 4, st);
        std::vector<char> seen(n, 0);
        std::vector<int32_t> stack{0};
        seen[0] = 1;
        int64_t reached = 1;
        while (!stack.empty()) {
            int32_t i = stack.back();
            stack.pop_back();
            for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
                if (!seen[cl[q]]) {
                    seen[cl[q]] = 1;
                    ++reached;
                    stack.push_back(cl[q]);
                }
        }
        s.connected = reached == n;
        int w = 0;
        for (int64_t i = 0; i < n; ++i) w = std::max(w, rp[i + 1] - rp[i]);
        s.ell_w = w;
    }
    s.ell_col = dev_alloc<int32_t>(s, (size_t)s.ell_w * s.npad);
    s.ell_val = dev_alloc<double>(s, (size_t)s.ell_w * s.npad);
    hipLaunchKernelGGL(ell_kernel, dim3((unsigned)(s.npad / 256)), dim3(256), 0, st, n, s.npad, s.ell_w, s.rowptr,
                       s.col, s.val, s.ell_col, s.ell_val);
    WFQ_CHECK_LAUNCH();
    // ---- near-field correction of the far-field element (used by the narrow matrix-free products)
    {
        s.rfar = 6.0 * std::sqrt(2.0) * s.width_max;   // erfc(6) = 2e-17: beyond it T_ij = 1 / r_ij in FP64
        const int R = std::max(1, (int)std::ceil(s.rfar / grid.h));
        hipLaunchKernelGGL(near_kernel<true>, dim3((unsigned)(s.npad / 256)), dim3(256), 0, st, n, s.pos, s.width,
                           s.eta, s.npad, ga, R, d_start, d_count, s.rfar * s.rfar, d_counts, 0, nullptr, nullptr);
        WFQ_CHECK_LAUNCH();
        hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, st, n, d_counts, d_flag);
        WFQ_CHECK_LAUNCH();
        int32_t wmax = 0;
        d2h_sync(s, &wmax, d_flag, 4, st);
        s.near_w = std::max(1, (int)wmax);
        s.near_col = dev_alloc<int32_t>(s, (size_t)s.near_w * s.npad);
        s.near_val = dev_alloc<double>(s, (size_t)s.near_w * s.npad);
        hipLaunchKernelGGL(near_kernel<false>, dim3((unsigned)(s.npad / 256)), dim3(256), 0, st, n, s.pos, s.width,
                           s.eta, s.npad, ga, R, d_start, d_count, s.rfar * s.rfar, nullptr, s.near_w, s.near_col,
                           s.near_val);
        WFQ_CHECK_LAUNCH();
    }
    WFQ_HIP(hipStreamSynchronize(st));
    scratch.release();

    // ---- a2: stored T copies
    uint32_t mask = p->store_mask ? p->store_mask : (WFQ_STORE_FP64 | WFQ_STORE_FP32);
    s.t_mode = p->t_mode;
    if (s.t_mode == WFQ_TMODE_AUTO) {
        uint64_t need = 0;
        if (mask & WFQ_STORE_FP64) need += (uint64_t)s.npad * s.npad * 8;
        if (mask & WFQ_STORE_FP32) need += (uint64_t)s.npad * s.npad * 4;
        if (mask & WFQ_STORE_BF16) need += (uint64_t)s.npad * s.npad * 2;
        // leave at least a third of the budget for the Krylov work space
        s.t_mode = (s.budget == 0 || s.bytes + need <= s.budget / 3 * 2) ? WFQ_TMODE_STORED : WFQ_TMODE_OTF;
    }
    if (s.t_mode == WFQ_TMODE_STORED) {
        const size_t nn = (size_t)s.npad * s.npad;
        if (mask & WFQ_STORE_FP64) s.T64 = dev_alloc<double>(s, nn);
        if (mask & WFQ_STORE_FP32) s.T32 = dev_alloc<float>(s, nn);
        if (mask & WFQ_STORE_BF16) s.T16 = dev_alloc<uint16_t>(s, nn);
        dim3 tg((unsigned)(s.npad / 256), (unsigned)(s.npad / 32));
        hipLaunchKernelGGL(build_T_kernel, tg, dim3(256), 0, st, n, s.npad, s.pos, s.eta, s.width, s.T64, s.T32,
                           s.T16);
        WFQ_CHECK_LAUNCH();
    }
    // ---- a3: rho_T >= lambda_max(T) for the solvers' error bound (Gershgorin: the entries of T are
    // positive, so the largest row sum bounds the spectrum). One recomputed FP64 product with the
    // vector of ones; the sum of n positive terms is exact to n u relative, covered by the 1e-9 margin.
    {
        ScratchDev sc;
        double* ones = sc.take<double>(s.npad);
        double* rows = sc.take<double>(s.npad);
        hipLaunchKernelGGL(ones_kernel, dim3((unsigned)(s.npad / 256)), dim3(256), 0, st, n, s.npad, ones);
        WFQ_CHECK_LAUNCH();
        otf_narrow_f64(s, ones, rows, s.npad, 1, device_cus(s.device), st);
        std::vector<double> h((size_t)n);
        d2h_sync(s, h.data(), rows, (size_t)n * sizeof(double), st);
        s.t_rowsum = *std::max_element(h.begin(), h.end()) * (1.0 + 1e-9);
        sc.release();
    }
    WFQ_HIP(hipStreamSynchronize(st));
}

void build_rhs(const Structure& s, const double* dirs_dev, int n_dir, double E0, double* out, int64_t ld,
               hipStream_t st) {
    dim3 grd((unsigned)((s.npad + 255) / 256), (unsigned)n_dir);
    hipLaunchKernelGGL(rhs_kernel, grd, dim3(256), 0, st, s.n, s.npad, s.pos, s.rowptr, s.col, s.val, dirs_dev,
                       n_dir, E0, out, ld);
    WFQ_CHECK_LAUNCH();
}

}  // namespace wfq
