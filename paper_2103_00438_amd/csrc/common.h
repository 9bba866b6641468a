// Internal declarations shared by the HIP translation units of libwfq.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/wfq.h"

namespace wfq {

// Every dense vector / matrix dimension is padded to a multiple of this, so the block-product
// kernels never need bounds checks (padding entries are kept at exactly zero).
constexpr int kPad = 256;
// Rows of the packed right-hand-side block are padded to this: the largest m-tile of any
// block-product variant, so no variant reads or writes past the allocated rows.
constexpr int kColPad = 256;
constexpr uint64_t kSplitWsCap = 512ull << 20;   // work space of split-k block products
constexpr uint64_t kSymWsCap = 32ull << 30;      // per-block sums of the symmetric narrow products

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 16 bytes, kept in registers

struct Error {
    int code;
    std::string msg;
};

void set_error(int code, const std::string& msg);

#define WFQ_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::wfq::Error{WFQ_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define WFQ_CHECK_LAUNCH() WFQ_HIP(hipGetLastError())

// ------------------------------------------------------------------ device-resident structure

struct SolveCache;   // the solver's work space and captured graphs, kept between solves

struct Structure {
    int device = 0;
    int64_t n = 0;       // atoms
    int64_t npad = 0;    // n rounded up to kPad
    std::vector<int64_t> perm;   // internal index -> caller index
    std::vector<int64_t> iperm;  // caller index -> internal index
    std::vector<double> pos_host;  // [3][n] internal order, bohr
    int32_t* dperm = nullptr;    // device [n], internal index -> caller index
    double* pos = nullptr;       // device [3][npad] SoA, bohr (padding: zeros)
    double* eta = nullptr;       // device [npad]
    double* width = nullptr;     // device [npad], d_i
    double* sphere = nullptr;    // device [npad / 64][4]: centre and radius of each 64-atom block (bohr)
    double width_max = 0.0;      // largest d_i
    int64_t nnz = 0;
    int32_t* rowptr = nullptr;   // device [n + 1]
    int32_t* col = nullptr;      // device [nnz]
    double* val = nullptr;       // device [nnz]
    int ell_w = 0;               // ELL width: longest row of L (diagonal included)
    int32_t* ell_col = nullptr;  // device [ell_w][npad], column of entry t of row i (padding: i)
    double* ell_val = nullptr;   // device [ell_w][npad], value (padding: 0)
    // near-field correction C = T - 1/r over pairs closer than rfar (eta on the diagonal), transposed
    // ELL [near_w][npad]: T X = (1/r) X (far-field formula for every pair) + C X
    double rfar = 0.0;           // bohr
    int near_w = 0;
    int32_t* near_col = nullptr;
    double* near_val = nullptr;
    double* T64 = nullptr;       // device [npad][npad]
    float* T32 = nullptr;
    uint16_t* T16 = nullptr;     // bf16 bit patterns
    int t_mode = WFQ_TMODE_STORED;
    double r0 = 0, fd = 0, fs = 0, rc = 0, W = 0, tau = 0;   // r0: largest of the atoms' r0 (bohr)
    double cfac = 0;             // r_c = s r0 cfac, cfac = 1 + ln(1/eps - 1) / d
    double* r0a = nullptr;       // device [npad], r0 of each atom's species (bohr)
    double t_rowsum = 0;         // >= lambda_max(T): the largest row sum of T (its entries are positive)
    uint64_t budget = 0;
    uint64_t bytes = 0;          // device bytes held by this structure
    bool connected = true;
    std::map<int, int> tuned[3];   // per precision: ncol -> block-product variant chosen by tune_tx
    // partial tiles of split-k block products (grown on demand, at most kSplitWsCap bytes)
    mutable void* split_ws = nullptr;
    mutable uint64_t split_ws_bytes = 0;
    // bytes of that work space a solve has reserved in its budget for the per-block sums of the
    // symmetric narrow products (0: at most kSplitWsCap)
    mutable uint64_t sym_ws_allowed = 0;
    // when set, the partial tiles go to this region (at most split_fixed_bytes) and nothing is
    // allocated: the block products then choose only splits whose partial tiles fit
    mutable void* split_fixed = nullptr;
    mutable uint64_t split_fixed_bytes = 0;
    // bumped whenever a block-product choice (tuning) or the partial-tile buffer changes: captured
    // launch sequences that refer to either are then stale
    mutable uint64_t epoch = 0;
    // pinned host staging of device-to-host copies (d2h_sync)
    mutable void* pin_stage = nullptr;
    mutable size_t pin_stage_bytes = 0;
    SolveCache* cache = nullptr;
};

// frees the solver's cached work space and graphs (the structure's device must be current)
void free_solve_cache(Structure& s);

// Device-to-host copy into ordinary (pageable) host memory, staged in chunks through the
// structure's pinned staging buffer (allocated on first use, freed with the structure): the copy
// engines write only memory the library owns, never the caller's pages. The stream's earlier work
// is finished and dst holds the data on return.
void d2h_sync(const Structure& s, void* dst, const void* src, size_t bytes, hipStream_t st);
// Host-to-device copy from ordinary host memory through the same pinned staging buffer (the copy
// engines read only memory the library owns); the copy is complete on return.
void h2d_sync(const Structure& s, void* dst, const void* src, size_t bytes, hipStream_t st);

struct KernelStat {
    const char* name;
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
};

enum KernelClass {
    KC_GEMM_F64 = 0, KC_GEMM_F32, KC_GEMM_BF16, KC_SKINNY, KC_OTF, KC_OTF_F64,
    KC_SPMM, KC_DOT, KC_UPDATE, KC_GIVENS, KC_PACK, KC_XUPDATE, KC_RESID, KC_QMR, KC_PRECOND, KC_OTHER,
    KC_SKINNY_F32, KC_SKINNY_BF16, KC_OTF_NARROW, KC_RECYCLE,
    KC_COUNT
};

// ------------------------------------------------------------------ per-kernel timing

// Times kernel launches with HIP events recorded on the launching stream (enabled per solve).
class Timer {
  public:
    explicit Timer(bool on) : on_(on) {}
    ~Timer();
    void begin(hipStream_t st);
    void end(hipStream_t st, int kclass, double flops, double bytes);
    // wait for the recorded events and add them to stats
    void collect(KernelStat* stats);
    bool on() const { return on_; }

  private:
    struct Rec {
        hipEvent_t a, b;
        int kc;
        double flops, bytes;
    };
    bool on_;
    std::vector<Rec> recs_;
    std::vector<hipEvent_t> pool_;
    hipEvent_t pending_ = nullptr;
    hipEvent_t get();
};

// ------------------------------------------------------------------ builders (build.hip)
// eta_atom, r0_atom: [n] per-atom hardness (Hartree) and r0 (Angstrom) in the caller's order; W the
// resolved Drude prefactor
void build_structure(Structure& s, const wfq_geometry* g, const wfq_params* p, const double* eta_atom,
                     const double* r0_atom, double W, hipStream_t st);
void free_structure(Structure& s);
void build_rhs(const Structure& s, const double* dirs_dev, int n_dir, double E0, double* out, int64_t ld,
               hipStream_t st);

// ------------------------------------------------------------------ products (gemm.hip)
// Y[c][i] = sum_k T[i][k] X[c][k] for c < ncol, i < npad; X, Y row-major with leading dimension ld.
// X must hold round_up(ncol, kColPad) rows (rows >= ncol zero). Y likewise.
void tx_f64(const Structure& s, const double* X, double* Y, int ncol, hipStream_t st);
void tx_f32(const Structure& s, const float* X, float* Y, int ncol, hipStream_t st);
void tx_bf16(const Structure& s, const uint16_t* X, float* Y, int ncol, hipStream_t st);
const char* tx_variant(int precision, int ncol);
// true when a product of ncol columns in `prec` recomputes the elements with the narrow kernel
bool tx_is_otf_narrow(const Structure& s, int prec, int ncol);
// T X with the stored copy of T in `prec`, or recomputed on the fly when the structure is matrix-free
void tx_any(const Structure& s, int prec, const void* X, void* Y, int ncol, hipStream_t st);
// one registered block-product variant (index as listed by tx_variant_name), stored T only
void tx_variant_run(const Structure& s, int prec, int var, const void* X, void* Y, int ncol, hipStream_t st);
int tx_variant_count(int precision);
const char* tx_variant_name(int precision, int k);
int tx_variant_max_ncol(int precision, int k);
void tune_tx(Structure& s, int prec, int ncol, int reps, double* ms, hipStream_t st);
// dst[i] = cast(src[i]) for i < count (round to nearest even)
void convert_from_f64(int prec, const double* src, void* dst, int64_t count, hipStream_t st);
void otf_tx_f32(const Structure& s, const float* X, float* Y, int ncol, hipStream_t st);
// Y = T X for at most 4 real FP64 columns with every element recomputed (no stored T needed), on
// the vector ALUs; `cus` = compute units of the device (sets the split of the source range). With
// Yi != NULL also Yi[i][c] = Y[c][i] with rows of 4 doubles (columns >= ncol zero; Yi 32-byte aligned,
// npad rows), so that a gather of row j reads every column at once.
void otf_narrow_f64(const Structure& s, const double* X, double* Y, int64_t ld, int ncol, int cus, hipStream_t st,
                    double* Yi = nullptr);
// compute units of a device
int device_cus(int device);
// true when narrow recomputed products of ncol <= 4 columns take the symmetric form (each element
// evaluated once for both of its rows: n >= 65 536 and the per-block sums fit the work space)
bool otf_sym_fits(const Structure& s, int ncol);
// work space of the symmetric form for ncol columns (0 below 65 536 atoms, where it is not used)
uint64_t otf_sym_bytes(const Structure& s, int ncol);
// partial-tile work space of the block products (grown on demand, or the fixed region when set)
void* split_workspace(const Structure& s, uint64_t bytes);
void otf_tx_f64(const Structure& s, const double* X, double* Y, int ncol, hipStream_t st);

}  // namespace wfq
