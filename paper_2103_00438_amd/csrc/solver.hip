// Host drivers of the batched solves (arXiv 2103.00438, Section "Solution strategies").
//
// All (frequency, field) systems of one structure share T, so each Krylov step applies T to the
// current basis vectors of every active system at once: one block product T X with 2 real columns
// per complex system. Restarted GMRES(m) runs its inner cycles with T in the requested precision
// (FP64, FP32, or BF16 with FP32 accumulation); every restart is an FP64 refinement point where the
// true residual b - (L T + z I) x is recomputed with the FP64 copy of T, and the next cycle starts
// from it. Systems leave the active set when their estimate reaches the target (the block shrinks),
// and a system whose FP64 residual stalls while its inner estimate fell is moved to a higher
// precision (its inner operator was not accurate enough).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <tuple>

#include "krylov.h"
#include "solver.h"

namespace wfq {

// ------------------------------------------------------------------ Timer

Timer::~Timer() {
    for (auto& r : recs_) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : pool_) (void)hipEventDestroy(e);
    if (pending_) (void)hipEventDestroy(pending_);
}

hipEvent_t Timer::get() {
    if (!pool_.empty()) {
        hipEvent_t e = pool_.back();
        pool_.pop_back();
        return e;
    }
    hipEvent_t e;
    WFQ_HIP(hipEventCreate(&e));
    return e;
}

void Timer::begin(hipStream_t st) {
    if (!on_) return;
    pending_ = get();
    WFQ_HIP(hipEventRecord(pending_, st));
}

void Timer::end(hipStream_t st, int kclass, double flops, double bytes) {
    if (!on_ || !pending_) return;
    hipEvent_t b = get();
    WFQ_HIP(hipEventRecord(b, st));
    recs_.push_back({pending_, b, kclass, flops, bytes});
    pending_ = nullptr;
}

void Timer::collect(KernelStat* stats) {
    for (auto& r : recs_) {
        WFQ_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        WFQ_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        if (stats) {
            stats[r.kc].launches += 1;
            stats[r.kc].ms += ms;
            stats[r.kc].flops += r.flops;
            stats[r.kc].bytes += r.bytes;
        }
        pool_.push_back(r.a);
        pool_.push_back(r.b);
    }
    recs_.clear();
}

namespace {

// A typed slice of one of the solver's two allocations (device memory and pinned host memory).
template <typename T>
struct Buf {
    T* p = nullptr;
    size_t count = 0;
};

// Lays the solver's arrays out back to back (256-byte aligned) in one region; with base == nullptr
// it only measures the region's size.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    void take(Buf<T>& b, size_t count) {
        off = (off + 255) & ~size_t(255);
        b.count = count;
        b.p = (base && count) ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
    }
};

int elem_size(int prec) { return prec == WFQ_PREC_FP64 ? 8 : prec == WFQ_PREC_FP32 ? 4 : 2; }
int out_size(int prec) { return prec == WFQ_PREC_FP64 ? 8 : 4; }

bool have_copy(const Structure& S, int prec) {
    if (S.t_mode == WFQ_TMODE_OTF) return prec != WFQ_PREC_BF16;   // recomputed in FP32 or FP64
    return prec == WFQ_PREC_FP64 ? S.T64 != nullptr : prec == WFQ_PREC_FP32 ? S.T32 != nullptr : S.T16 != nullptr;
}

// next precision up that has a stored copy (FP64 always last)
int escalate_prec(const Structure& S, int prec) {
    if (prec == WFQ_PREC_BF16 && have_copy(S, WFQ_PREC_FP32)) return WFQ_PREC_FP32;
    return WFQ_PREC_FP64;
}

// A refinement cycle at reduced precision failed when the FP64 residual grew (a restarted Krylov
// cycle with the exact operator never increases it), or when it fell by less than 2x although the
// inner estimate claimed more than 10x.
bool needs_escalation(double beta, double beta_prev, double est_end) {
    if (!(beta <= beta_prev)) return true;
    return beta > 0.5 * beta_prev && beta > 10.0 * est_end;
}

enum Slot { SLOT_G0 = 0, SLOT_G1 = 1, SLOT_G2 = 2, SLOT_STEP = 3, SLOT_ACT = 4, NSLOT = 5 };

// structures above this padded size interleave the products' planes before the SpMM (an extra pass
// over Y that pays where the sparse product is bound by its gathers, not by launch latency)
constexpr int64_t kPairsFrom = 8192;

// What a solve's work space depends on: a solve with the same shape reuses it.
struct WorkShape {
    int B = 0, m = 0, n_dir = 0, prec = 0, ms_m = 0;   // ms_m: shared-basis dimension (0: no multi-shift)
    bool qmr = false;
    bool bj = false;   // block-Jacobi preconditioning
    int rk = 0;        // recycle space dimension (0: no recycling)
    bool operator==(const WorkShape& o) const {
        return B == o.B && m == o.m && n_dir == o.n_dir && prec == o.prec && ms_m == o.ms_m && qmr == o.qmr &&
               bj == o.bj && rk == o.rk;
    }
};

// arrays of the multi-shift phase (one real basis per direction, one shifted recurrence per system)
struct MsWork {
    Buf<double> V, H, part, h1, h2, nrm, inv_h, cs, est, tol_abs;
    Buf<double> TV;   // FP64 solves: T u_j of every vector that entered a product, kept for the closing residual
    Buf<double> Sm;   // with TV: U = Q S, S upper triangular, columns in the layout of H
    Buf<double> dots, hp, gam, irho, nu;   // one-reduction Arnoldi: [d][2 (m + 1)], [d][m + 1], [d] x 3
    Buf<double> Yi;   // FP64 narrow products: the product interleaved, [npad][4], for the SpMM's gathers
    Buf<int> pos;     // system -> packed column of the closing residual's products
    int ngrp = 0;     // groups of ms_xupdate in the last phase
    Buf<double2> sn, g, R, y, z;
    Buf<int> dirs, sdir, sys, flags, ksteps, grp_sys, grp_dir, run;
    Buf<int> h_dirs, h_sys, h_k;   // pinned
    Buf<double> h_nrm;             // pinned
};

struct Work {
    WorkShape shape;
    void* dev = nullptr;    // the one device allocation every device array lives in
    void* host = nullptr;   // the one pinned host allocation
    size_t dev_bytes = 0, host_bytes = 0;
    int B = 0, mdim = 0, n_dir = 0;
    int64_t n = 0, npad = 0, nwc = 0, nblk = 0, mpad = 0;
    bool need32 = false, need16 = false;
    bool ms_tv_ready = false;   // the multi-shift phase left T x of its iterates computable from ms.TV
    Buf<double> V, X, b, X64, Y64, cs, est, inv_h, inv_beta, beta, norm2, tol_abs;
    Buf<double> qT, qtq;   // |x|_T = sqrt(x^H T x) at the last FP64 residual, and its block partials
    Buf<float> X32, Y32, Y16, Yp32;   // Yp*: the products' planes interleaved for the SpMM (large N)
    Buf<double> Yp64;
    Buf<uint16_t> X16;
    Buf<double2> partial, h1, h2, R, Hu, sn, g, y, z, alpha, gam;
    Buf<double> nu, irho;
    // QMR scalars and partials
    Buf<double2> rho_a, rho_b, sigma, part_sig, part_nrm;
    Buf<double> tau2, eta, snorm, tpb;
    Buf<int> first;
    Buf<int> flags, ksteps, dir, run, sys[NSLOT];
    Buf<double> d_dirs, stage_re, stage_im;
    Buf<int> warm_sys, warm_a, warm_b;   // warm starts: target and the two solved neighbours
    Buf<double2> warm_t;                 // interpolation weight in z
    // block-Jacobi: C_b (FP64, [npad/64][64][64]), the inverted blocks of every system
    // ([B][npad/64][64 x 64] complex FP32, column-major) and the preconditioned vector u of every system
    Buf<double> bj_C, bj_U;
    Buf<float2> bj_P;
    // subspace recycling: C and U' of every system, the per-system counts, partial dots, coefficients,
    // B of the cycle, the neighbours of the targets and per-system scale factors
    Buf<double> rc_C, rc_U, rc_inv, h_rc_inv;
    Buf<int> rc_kk, rc_nbr, h_rc_kk, h_rc_nbr;
    Buf<double2> rc_part, rc_coef, rc_B;
    RecycleSpace rc;
    bool rc_active = false;   // the current pass projects onto the recycle spaces
    MsWork ms;
    // pinned host mirrors
    Buf<double> h_snorm, h_est, h_beta, h_invb, h_qT;
    // est (B doubles), flags and ksteps (B ints each) side by side on the device and in the pinned
    // mirror, so that the per-step read-back is one copy
    Buf<double> step_dev, step_host;
    Buf<int> h_sys[NSLOT], h_flags, h_ksteps, h_run;
    Buf<double2> h_g, h_alpha;
    Basis Vb, Xb, Ub;

    Work() = default;
    Work(const Work&) = delete;
    Work& operator=(const Work&) = delete;
    ~Work() {
        if (dev) (void)hipFree(dev);
        if (host) (void)hipHostFree(host);
    }
};

int ms_dim(const wfq_solve_opts& o, int64_t n);

void layout_work(Work& w, const Structure& S, Arena& d, Arena& h) {
    const WorkShape& sh = w.shape;
    const int B = sh.B, m = sh.m, n_dir = sh.n_dir, prec = sh.prec;
    w.B = B;
    w.mdim = m + 1;
    w.n_dir = n_dir;
    w.n = S.n;
    w.npad = S.npad;
    w.nwc = wave_chunks(S.n);
    w.nblk = resid_blocks(S.n);
    w.mpad = round_up(2 * (int64_t)B, kColPad);
    w.need16 = prec == WFQ_PREC_BF16;
    w.need32 = prec == WFQ_PREC_FP32 || (prec == WFQ_PREC_BF16 && have_copy(S, WFQ_PREC_FP32));
    const int64_t np = S.npad;
    d.take(w.V, (size_t)B * w.mdim * 2 * np);
    d.take(w.X, (size_t)B * 2 * np);
    d.take(w.b, (size_t)n_dir * np);
    d.take(w.X64, (size_t)w.mpad * np);
    d.take(w.Y64, (size_t)w.mpad * np);
    d.take(w.X32, w.need32 ? (size_t)w.mpad * np : 0);
    d.take(w.Y32, w.need32 ? (size_t)w.mpad * np : 0);
    d.take(w.X16, w.need16 ? (size_t)w.mpad * np : 0);
    d.take(w.Y16, w.need16 ? (size_t)w.mpad * np : 0);
    const bool pairs = np > kPairsFrom;
    d.take(w.Yp64, pairs ? (size_t)w.mpad * np : 0);
    d.take(w.Yp32, pairs && (w.need32 || w.need16) ? (size_t)w.mpad * np : 0);
    d.take(w.partial, (size_t)B * 2 * w.mdim * w.nwc);   // fused dots: two entries per basis vector
    d.take(w.h1, (size_t)B * 2 * w.mdim);
    d.take(w.h2, (size_t)B * w.mdim);
    d.take(w.R, (size_t)B * w.mdim * w.mdim);
    d.take(w.Hu, sh.qmr ? 0 : (size_t)B * w.mdim * w.mdim);
    d.take(w.gam, B);
    d.take(w.nu, B);
    d.take(w.irho, B);
    d.take(w.cs, (size_t)B * w.mdim);
    d.take(w.sn, (size_t)B * w.mdim);
    d.take(w.g, (size_t)B * (w.mdim + 1));
    d.take(w.y, (size_t)B * w.mdim);
    d.take(w.z, B);
    d.take(w.alpha, (size_t)B * 3);
    d.take(w.step_dev, (size_t)2 * B);
    w.est = Buf<double>{w.step_dev.p, (size_t)B};
    d.take(w.inv_h, B);
    d.take(w.inv_beta, B);
    d.take(w.beta, B);
    d.take(w.norm2, (size_t)B * std::max(w.nwc, w.nblk));
    d.take(w.tol_abs, B);
    d.take(w.qT, B);
    d.take(w.qtq, (size_t)B * w.nblk);
    w.flags = Buf<int>{w.step_dev.p ? reinterpret_cast<int*>(w.step_dev.p + B) : nullptr, (size_t)B};
    w.ksteps = Buf<int>{w.step_dev.p ? reinterpret_cast<int*>(w.step_dev.p + B) + B : nullptr, (size_t)B};
    d.take(w.run, B);
    d.take(w.dir, B);
    for (int k = 0; k < NSLOT; ++k) {
        d.take(w.sys[k], B);
        h.take(w.h_sys[k], B);
    }
    d.take(w.rho_a, B);
    d.take(w.rho_b, B);
    d.take(w.sigma, B);
    d.take(w.part_sig, (size_t)B * w.nblk);
    d.take(w.part_nrm, (size_t)B * w.nblk);
    d.take(w.tau2, B);
    d.take(w.eta, B);
    d.take(w.snorm, B);
    d.take(w.first, B);
    d.take(w.tpb, sh.qmr ? (size_t)B * 2 * np : 0);   // QMR: compact T p, rows by system id
    d.take(w.d_dirs, (size_t)3 * n_dir);
    d.take(w.warm_sys, B);
    d.take(w.warm_a, B);
    d.take(w.warm_b, B);
    d.take(w.warm_t, B);
    d.take(w.bj_C, sh.bj ? (size_t)np * 64 : 0);
    d.take(w.bj_P, sh.bj ? (size_t)B * np * 64 : 0);
    d.take(w.bj_U, sh.bj ? (size_t)B * 2 * np : 0);
    {
        const size_t rk = (size_t)sh.rk;
        d.take(w.rc_C, (size_t)B * rk * 2 * np);
        d.take(w.rc_U, (size_t)B * rk * 2 * np);
        d.take(w.rc_inv, rk ? (size_t)B : 0);
        d.take(w.rc_kk, rk ? (size_t)B : 0);
        d.take(w.rc_nbr, (size_t)B * rk);
        d.take(w.rc_part, (size_t)B * rk * wave_chunks(S.n));
        d.take(w.rc_coef, (size_t)B * rk);
        d.take(w.rc_B, (size_t)B * rk * (m + 1));
        h.take(w.h_rc_inv, rk ? (size_t)B : 0);
        h.take(w.h_rc_kk, rk ? (size_t)B : 0);
        h.take(w.h_rc_nbr, (size_t)B * rk);
    }
    d.take(w.stage_re, (size_t)B * S.n);   // host outputs are staged through these
    d.take(w.stage_im, (size_t)B * S.n);
    h.take(w.step_host, (size_t)2 * B);
    w.h_est = Buf<double>{w.step_host.p, (size_t)B};
    w.h_flags = Buf<int>{w.step_host.p ? reinterpret_cast<int*>(w.step_host.p + B) : nullptr, (size_t)B};
    w.h_ksteps = Buf<int>{w.step_host.p ? reinterpret_cast<int*>(w.step_host.p + B) + B : nullptr, (size_t)B};
    h.take(w.h_run, B);
    h.take(w.h_beta, B);
    h.take(w.h_qT, B);
    h.take(w.h_invb, B);
    h.take(w.h_snorm, B);
    h.take(w.h_g, (size_t)B * (w.mdim + 1));
    h.take(w.h_alpha, (size_t)B * 3);
    if (sh.ms_m > 0) {
        MsWork& q = w.ms;
        const int64_t mm = sh.ms_m, mdim1 = mm + 1, pslots = mm + 2;
        d.take(q.V, (size_t)n_dir * mdim1 * np);
        if (sh.prec == WFQ_PREC_FP64) d.take(q.TV, (size_t)n_dir * mdim1 * np);
        d.take(q.pos, B);
        d.take(q.H, (size_t)n_dir * mm * (mm + 1));
        d.take(q.part, (size_t)n_dir * 2 * mdim1 * w.nwc);   // >= pslots: also the fused dots' partials
        if (sh.prec == WFQ_PREC_FP64) d.take(q.Sm, (size_t)n_dir * mm * (mm + 1));
        d.take(q.dots, (size_t)n_dir * 2 * mdim1);
        d.take(q.hp, (size_t)n_dir * mdim1);
        d.take(q.gam, n_dir);
        d.take(q.irho, n_dir);
        d.take(q.nu, n_dir);
        d.take(q.Yi, (size_t)np * 4);
        d.take(q.h1, (size_t)n_dir * pslots);
        d.take(q.h2, (size_t)n_dir * pslots);
        d.take(q.nrm, (size_t)n_dir * (np / 64));
        d.take(q.inv_h, n_dir);
        d.take(q.cs, (size_t)B * mm);
        d.take(q.sn, (size_t)B * mm);
        d.take(q.g, (size_t)B * (mm + 1));
        d.take(q.R, (size_t)B * (mm * (mm + 1) / 2));
        d.take(q.y, (size_t)B * mm);
        d.take(q.z, B);
        d.take(q.est, B);
        d.take(q.tol_abs, B);
        d.take(q.dirs, n_dir);
        d.take(q.sdir, B);
        d.take(q.sys, B);
        d.take(q.flags, B);
        d.take(q.ksteps, B);
        d.take(q.run, B);
        // groups of up to kMsGroup systems of one direction: at most B + (kMsGroup - 1) n_dir slots
        d.take(q.grp_sys, (size_t)B + (size_t)(kMsGroup - 1) * n_dir);
        d.take(q.grp_dir, (size_t)B + n_dir);
        h.take(q.h_dirs, n_dir);
        h.take(q.h_sys, B);
        h.take(q.h_k, B);
        h.take(q.h_nrm, (size_t)n_dir * pslots);
    }
    w.Vb = Basis{w.V.p, (int64_t)w.mdim * 2 * np, 2 * np, np};
    w.Xb = sh.qmr ? Basis{w.V.p + 5 * 2 * np, (int64_t)w.mdim * 2 * np, 2 * np, np}   // the QMR iterate
                  : Basis{w.X.p, 2 * np, 2 * np, np};
    w.Ub = Basis{w.bj_U.p, 2 * np, 0, np};   // one vector per system: every slot index names it
    w.rc.C = Basis{w.rc_C.p, (int64_t)sh.rk * 2 * np, 2 * np, np};
    w.rc.U = Basis{w.rc_U.p, (int64_t)sh.rk * 2 * np, 2 * np, np};
    w.rc.kmax = sh.rk;
    w.rc.kk = w.rc_kk.p;
    w.rc.part = w.rc_part.p;
    w.rc.coef = w.rc_coef.p;
    w.rc.Bm = w.rc_B.p;
}

// Allocates the work space of one shape: one device and one pinned host allocation.
void make_work(Work& w, const Structure& S, const WorkShape& sh) {
    w.shape = sh;
    Arena d, h;
    layout_work(w, S, d, h);
    w.dev_bytes = std::max<size_t>(d.off, 256);
    w.host_bytes = std::max<size_t>(h.off, 256);
    hipError_t e = hipMalloc(&w.dev, w.dev_bytes);
    if (e != hipSuccess) {
        w.dev = nullptr;
        throw Error{WFQ_ENOMEM, std::string("hipMalloc of the Krylov work space failed: ") + hipGetErrorString(e)};
    }
    WFQ_HIP(hipHostMalloc(&w.host, w.host_bytes, hipHostMallocDefault));
    Arena d2{static_cast<char*>(w.dev), 0}, h2{static_cast<char*>(w.host), 0};
    layout_work(w, S, d2, h2);
}

// Every solve starts from a zeroed work space (a reused one holds the previous solve's data).
void clear_work(Work& w, hipStream_t st) {
    WFQ_HIP(hipMemsetAsync(w.dev, 0, w.dev_bytes, st));
    std::memset(w.host, 0, w.host_bytes);
}

// ---- HIP graphs of inner-iteration chunks
//
// For small structures the inner iterations are bound by launch latency (a step is ~10 launches of a
// few microseconds each). A chunk of steps between two host synchronisations is the same launch
// sequence whenever its first step, length and list sizes repeat (the lists' contents live in device
// buffers, and convergence inside a chunk is handled by the device-side run mask), so it is captured
// once as a HIP graph and replayed. A chunk runs eagerly the first time its key is seen and is
// captured the second time, so one-off shapes never pay for a capture, and every buffer a graph
// refers to (the work space, the split-k partial tiles) exists before it is captured.

struct GraphKey {
    int kind, j0, c, ns, g0, g1, g2;
    bool operator<(const GraphKey& o) const {
        return std::tie(kind, j0, c, ns, g0, g1, g2) < std::tie(o.kind, o.j0, o.c, o.ns, o.g0, o.g1, o.g2);
    }
};

constexpr size_t kMaxGraphs = 1024;

struct GraphCache {
    std::map<GraphKey, hipGraphExec_t> exec;
    std::set<GraphKey> seen;
    uint64_t epoch = 0;   // Structure::epoch when the graphs were captured
    void clear() {
        for (auto& e : exec) (void)hipGraphExecDestroy(e.second);
        exec.clear();
        seen.clear();
    }
    ~GraphCache() { clear(); }
};

// Runs `body` (kernel launches on st only) eagerly, or as a captured graph, or replays the graph.
template <typename F>
void run_chunk(GraphCache* gc, const Structure& S, const GraphKey& k, hipStream_t st, F&& body) {
    if (!gc) {
        body();
        return;
    }
    if (gc->epoch != S.epoch) {   // a block-product choice or a buffer it uses changed
        gc->clear();
        gc->epoch = S.epoch;
    }
    auto it = gc->exec.find(k);
    if (it != gc->exec.end()) {
        WFQ_HIP(hipGraphLaunch(it->second, st));
        return;
    }
    if (gc->seen.insert(k).second || gc->exec.size() >= kMaxGraphs) {
        body();
        return;
    }
    hipGraph_t g = nullptr;
    WFQ_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    try {
        body();
    } catch (...) {
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    WFQ_HIP(hipStreamEndCapture(st, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (r != hipSuccess) throw Error{WFQ_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(r)};
    gc->exec.emplace(k, e);
    WFQ_HIP(hipGraphLaunch(e, st));
}

}  // namespace

// The handle's solve work space and its graphs, kept between solves of the same shape when small.
struct SolveCache {
    std::unique_ptr<Work> work;
    GraphCache graphs;
};

void free_solve_cache(Structure& S) {
    delete S.cache;   // graphs first, then the work space
    S.cache = nullptr;
}

namespace {

// The work space for a solve of shape sh: the handle's cached one when the shape matches, else a
// new one, which the handle keeps (the previous one is freed first). Repeated solves of one shape
// then allocate nothing: freeing and allocating a work space of tens of GB costs seconds.
Work& solve_work(Structure& S, const WorkShape& sh, GraphCache*& graphs, std::unique_ptr<Work>& own) {
    (void)own;
    graphs = nullptr;
    if (!(S.cache && S.cache->work && S.cache->work->shape == sh)) {
        free_solve_cache(S);
        auto w = std::make_unique<Work>();
        make_work(*w, S, sh);
        S.cache = new SolveCache;
        S.cache->work = std::move(w);
    }
    graphs = &S.cache->graphs;
    return *S.cache->work;
}

// view of one vector slot of a basis as a one-slot basis
Basis slot_view(const Basis& V, int j) { return Basis{V.base + (int64_t)j * V.vec_stride, V.sys_stride, V.vec_stride, V.npad}; }

void upload(Work& w, int slot, const std::vector<int>& v, hipStream_t st) {
    std::memcpy(w.h_sys[slot].p, v.data(), v.size() * sizeof(int));
    if (!v.empty())
        WFQ_HIP(hipMemcpyAsync(w.sys[slot].p, w.h_sys[slot].p, v.size() * sizeof(int), hipMemcpyHostToDevice, st));
}

struct SysState {
    double omega = 0;   // Hartree
    int dir = 0;
    double2 z{0, 0};
    int prec = WFQ_PREC_FP64;
    int status = WFQ_OK;
    int iters = 0, cycles = 0;
    double bnorm = 0, beta = 0, relres = 1, est_end = 0;
    double qT = 0;      // |q|_T at the last FP64 residual
    double t_done = 0;
    bool done = false;
};

// Bound on |q - q*|_T / |q*|_T, |v|_T = sqrt(v^H T v). With T symmetric positive definite and L
// symmetric positive semi-definite, L T is self-adjoint in the T inner product with real eigenvalues
// lambda >= 0, so |(L T + z I)^-1|_T = 1 / min |lambda + z| <= 1 / |Im z|. Hence
// |q - q*|_T <= |r|_T / |Im z| <= sqrt(rho_T) |r|_2 / |Im z|, rho_T >= lambda_max(T) the largest row
// sum of T (Gershgorin), and eps = that / |q|_T gives |q - q*|_T / |q*|_T <= eps / (1 - eps).
constexpr double kLightAU = 137.035999084;   // speed of light in atomic units (CODATA 2018)

double error_bound(const Structure& S, const SysState& q) {
    if (!(q.beta > 0.0)) return q.beta == 0.0 ? 0.0 : q.beta;   // exact, or NaN passed on
    const double eps = std::sqrt(S.t_rowsum) * q.beta / (std::fabs(q.z.y) * q.qT);
    return eps < 1.0 ? eps / (1.0 - eps) : INFINITY;
}

void* x_block(Work& w, int prec) {
    return prec == WFQ_PREC_FP64 ? (void*)w.X64.p : prec == WFQ_PREC_FP32 ? (void*)w.X32.p : (void*)w.X16.p;
}
const void* y_block(Work& w, int prec) {
    return prec == WFQ_PREC_FP64 ? (const void*)w.Y64.p : prec == WFQ_PREC_FP32 ? (const void*)w.Y32.p
                                                                                 : (const void*)w.Y16.p;
}

// One T X block product for the columns of one precision group (X already packed).
// Y = T X on the solve's product block. With Yi (a narrow FP64 product of at most 4 columns) the
// product is also written interleaved into Yi (rows of 4 doubles) for the multi-shift SpMM's gathers.
void block_product(const Structure& S, Work& w, int prec, int ncol, Timer& tm, hipStream_t st,
                   double* Yi = nullptr) {
    const double n = (double)S.n;
    tm.begin(st);
    if (Yi) {
        if (prec != WFQ_PREC_FP64 || ncol > 4 || !tx_is_otf_narrow(S, prec, ncol))
            throw Error{WFQ_EINVAL, "block_product: the interleaved copy needs a narrow FP64 product"};
        otf_narrow_f64(S, w.X64.p, w.Y64.p, S.npad, ncol, device_cus(S.device), st, Yi);
    } else {
        tx_any(S, prec, x_block(w, prec), const_cast<void*>(y_block(w, prec)), ncol, st);
    }
    if (tx_is_otf_narrow(S, prec, ncol)) {
        // work: per element 3 differences, 3 operations for r^2, the reciprocal square root and 4 for
        // its Newton step, and one multiply-add per column and row (the near-field correction is a
        // sparse extra); the symmetric form evaluates each element once for both rows, so n^2 / 2
        // elements; bytes: positions and X read once per source part, Y written
        const double chunks = (ncol + 3) / 4;   // products of up to 4 columns
        const double elems = otf_sym_fits(S, std::min(ncol, 4)) ? 0.5 * n * n : n * n;
        tm.end(st, KC_OTF_NARROW, elems * 11.0 * chunks + n * n * ncol, n * (24.0 * chunks + 8.0 * ncol) + n * 8.0 * ncol);
        return;
    }
    if (S.t_mode == WFQ_TMODE_OTF) {
        // flops: the MFMA accumulation; the element evaluations are counted by launches x n^2 pairs
        tm.end(st, prec == WFQ_PREC_FP64 ? KC_OTF_F64 : KC_OTF, 2.0 * n * n * ncol, ncol * n * 2.0 * elem_size(prec));
        return;
    }
    const int kc = ncol <= 8 ? (prec == WFQ_PREC_FP64 ? KC_SKINNY : prec == WFQ_PREC_FP32 ? KC_SKINNY_F32 : KC_SKINNY_BF16)
                             : (prec == WFQ_PREC_FP64 ? KC_GEMM_F64 : prec == WFQ_PREC_FP32 ? KC_GEMM_F32 : KC_GEMM_BF16);
    tm.end(st, kc, 2.0 * n * n * ncol, elem_size(prec) * n * n + ncol * n * (elem_size(prec) + out_size(prec)));
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void progress_line(const wfq_solve_opts& o, const char* what, int cycle, int step, size_t active, double worst,
                   std::chrono::steady_clock::time_point t0) {
    if (!o.progress) return;
    std::fprintf(stderr, "[wfq] %s cycle %d step %d: %zu active, worst relres %.3e, %.1f s\n", what, cycle, step,
                 active, worst, ms_since(t0) / 1e3);
    std::fflush(stderr);
}

// FP64 refinement residual of the systems in `act`: V(s,0) = b - (L T + z I) x, beta = ||V(s,0)||,
// qT = |x|_T (from the same product T x). With from_ms, x is the multi-shift phase's iterate V y and
// T x is formed as TV y from the kept FP64 products T v_j instead of a new product.
void fp64_residual(const Structure& S, Work& w, const std::vector<int>& act, Timer& tm, hipStream_t st,
                   bool from_ms = false) {
    const int na = (int)act.size();
    const double n = (double)S.n;
    if (from_ms) {
        MsWork& q = w.ms;
        const int m = w.shape.ms_m;
        std::vector<int> pos(w.B, -1);
        for (int k = 0; k < na; ++k) pos[act[k]] = k;
        h2d_sync(S, q.pos.p, pos.data(), w.B * sizeof(int), st);
        tm.begin(st);
        ms_txupdate(q.TV.p, S.n, S.npad, m + 1, q.grp_sys.p, q.grp_dir.p, q.ngrp, q.ksteps.p, q.y.p, m, q.pos.p,
                    w.Y64.p, S.npad, st);
        tm.end(st, KC_XUPDATE, 0, 0);
    } else {
        tm.begin(st);
        pack_columns(WFQ_PREC_FP64, w.Xb, w.sys[SLOT_ACT].p, na, 0, nullptr, false, w.X64.p, w.npad, st);
        tm.end(st, KC_PACK, 0, 32.0 * n * na);
        block_product(S, w, WFQ_PREC_FP64, 2 * na, tm, st);
    }
    tm.begin(st);
    residual(S, w.Y64.p, w.npad, w.sys[SLOT_ACT].p, na, w.z.p, w.Xb, w.b.p, w.dir.p, w.Vb, w.norm2.p, (int)w.nblk,
             w.qtq.p, st);
    sumsq(w.sys[SLOT_ACT].p, na, w.norm2.p, (int)w.nblk, w.beta.p, st);
    sumsq(w.sys[SLOT_ACT].p, na, w.qtq.p, (int)w.nblk, w.qT.p, st);
    tm.end(st, KC_RESID, 4.0 * S.nnz * na + 8 * n * na, 12.0 * S.nnz + na * n * (16 + 16 + 16 + 8));
}

// Restarted GMRES(m) with FP64 refinement at every restart, for the systems of one batch.
// `only` (if not NULL) restricts the solve to those systems of the batch; the others are untouched.
void gmres_batch(const Structure& S, Work& w, std::vector<SysState>& ss, double tol, const wfq_solve_opts& o,
                 Timer& tm, hipStream_t st, std::chrono::steady_clock::time_point t0, GraphCache* graphs,
                 bool warm = false, const std::vector<int>* only = nullptr) {
    const int B = (int)ss.size();
    const int m = w.mdim - 1;
    const double n = (double)S.n;
    // per-system constants
    {
        std::vector<double2> zh(B);
        std::vector<int> dh(B);
        for (int s = 0; s < B; ++s) {
            zh[s] = ss[s].z;
            dh[s] = ss[s].dir;
        }
        h2d_sync(S, w.z.p, zh.data(), B * sizeof(double2), st);
        h2d_sync(S, w.dir.p, dh.data(), B * sizeof(int), st);
        if (!warm && !only) {
            WFQ_HIP(hipMemsetAsync(w.X.p, 0, w.X.count * sizeof(double), st));
        } else if (!warm) {
            // x0 = 0 for the listed systems only (the others may hold solutions of an earlier pass)
            for (int s : *only)
                WFQ_HIP(hipMemsetAsync(w.Xb.base + (size_t)s * w.Xb.sys_stride, 0, 2 * S.npad * sizeof(double), st));
        }
        WFQ_HIP(hipStreamSynchronize(st));
    }
    std::vector<int> all;
    if (only) {
        all = *only;
    } else {
        all.resize(B);
        for (int s = 0; s < B; ++s) all[s] = s;
    }
    if (all.empty()) return;
    upload(w, SLOT_ACT, all, st);
    const bool bj = w.shape.bj;
    if (bj) {
        // the inverted diagonal blocks of every system of the solve
        tm.begin(st);
        bj_setup(S, w.sys[SLOT_ACT].p, (int)all.size(), w.z.p, w.bj_C.p, w.bj_P.p, st);
        tm.end(st, KC_PRECOND, 8.0 * S.nnz * 64 + (double)all.size() * (S.npad / 64) * 64.0 * 63 * 128 * 8,
               S.npad * 64.0 * 8 * (1.0 + all.size()));
    }
    // x0 = 0, r0 = b
    copy_rhs(S, w.sys[SLOT_ACT].p, (int)all.size(), w.b.p, w.dir.p, w.Vb, w.norm2.p, (int)w.nblk, st);
    sumsq(w.sys[SLOT_ACT].p, (int)all.size(), w.norm2.p, (int)w.nblk, w.beta.p, st);
    WFQ_HIP(hipMemcpyAsync(w.h_beta.p, w.beta.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
    WFQ_HIP(hipStreamSynchronize(st));
    std::vector<int> active;
    {
        std::vector<double> tol_h(B);
        for (int s : all) {
            ss[s].bnorm = ss[s].beta = w.h_beta.p[s];
            tol_h[s] = 0.5 * tol * ss[s].bnorm;   // inner target: half the outer one
            if (ss[s].bnorm == 0.0) {
                ss[s].relres = 0.0;
                ss[s].done = true;
                ss[s].t_done = ms_since(t0);
            } else if (!std::isfinite(ss[s].bnorm)) {
                ss[s].status = WFQ_ENUMERIC;
                ss[s].done = true;
            } else {
                active.push_back(s);
            }
        }
        h2d_sync(S, w.tol_abs.p, tol_h.data(), B * sizeof(double), st);
        WFQ_HIP(hipStreamSynchronize(st));
    }
    if (warm && !active.empty()) {
        // start from the given x: r = b - (L T + z I) x in FP64
        upload(w, SLOT_ACT, active, st);
        fp64_residual(S, w, active, tm, st, w.ms_tv_ready && !only);
        WFQ_HIP(hipMemcpyAsync(w.h_beta.p, w.beta.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipMemcpyAsync(w.h_qT.p, w.qT.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipStreamSynchronize(st));
        std::vector<int> still;
        for (int s : active) {
            ss[s].beta = w.h_beta.p[s];
            ss[s].qT = w.h_qT.p[s];
            ss[s].relres = ss[s].beta / ss[s].bnorm;
            if (ss[s].relres <= tol) {
                ss[s].done = true;
                ss[s].t_done = ms_since(t0);
            } else {
                still.push_back(s);
            }
        }
        active.swap(still);
        if (o.progress) {
            double worst = 0.0;
            for (int s : all) worst = std::max(worst, ss[s].relres);
            progress_line(o, "gmres from the given start", 0, 0, active.size(), worst, t0);
        }
    }
    w.ms_tv_ready = false;   // later residuals are of other iterates

    while (!active.empty()) {
        if (w.rc_active) {
            // recycling: x += U' C^H r, r -= C C^H r, and the norm of the projected residual
            upload(w, SLOT_ACT, active, st);
            tm.begin(st);
            rc_project(w.rc, w.Vb, 0, &w.Xb, w.sys[SLOT_ACT].p, (int)active.size(), nullptr, S.n, w.norm2.p,
                       (int)w.nblk, st);
            sumsq(w.sys[SLOT_ACT].p, (int)active.size(), w.norm2.p, (int)w.nblk, w.beta.p, st);
            tm.end(st, KC_RECYCLE, 0, 0);
            WFQ_HIP(hipMemcpyAsync(w.h_beta.p, w.beta.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
            WFQ_HIP(hipStreamSynchronize(st));
            std::vector<int> still;
            for (int s : active) {
                ss[s].beta = w.h_beta.p[s];
                if (ss[s].beta > 0.0) {
                    still.push_back(s);
                } else {   // the solution lies in the recycle space
                    ss[s].relres = 0.0;
                    ss[s].done = true;
                    ss[s].t_done = ms_since(t0);
                }
            }
            active.swap(still);
            if (active.empty()) break;
        }
        // cycle start: g = beta e1, v0 = r / beta
        std::memset(w.h_g.p, 0, (size_t)B * (w.mdim + 1) * sizeof(double2));
        for (int s : active) {
            w.h_g.p[(size_t)s * (w.mdim + 1)] = make_double2(ss[s].beta, 0.0);
            w.h_invb.p[s] = 1.0 / ss[s].beta;
            w.h_ksteps.p[s] = 0;
            ss[s].cycles += 1;
        }
        WFQ_HIP(hipMemcpyAsync(w.g.p, w.h_g.p, (size_t)B * (w.mdim + 1) * sizeof(double2), hipMemcpyHostToDevice, st));
        WFQ_HIP(hipMemcpyAsync(w.inv_beta.p, w.h_invb.p, B * sizeof(double), hipMemcpyHostToDevice, st));
        std::vector<int> stepping;
        for (int s : active)
            if (ss[s].iters < o.max_iter) stepping.push_back(s);
        // Convergence is tracked on the device (the column step records the completed columns and
        // clears run[s] when a flag is raised; every step kernel skips stopped systems). The host reads the
        // flags and compacts the lists every `chunk` steps: after every step for large problems, whose
        // block products shrink as systems drop out, and every 8 steps for small ones, where the
        // round trip would cost more than the steps.
        const int chunk = (S.npad <= 8192) ? 8 : 1;
        WFQ_HIP(hipMemcpyAsync(w.ksteps.p, w.h_ksteps.p, B * sizeof(int), hipMemcpyHostToDevice, st));
        std::vector<int> grp[3];
        auto lists = [&]() {   // upload the group lists, the step list and run = 1 for them
            for (int p = 0; p < 3; ++p) grp[p].clear();
            for (int s : stepping) grp[ss[s].prec].push_back(s);
            for (int p = 0; p < 3; ++p)
                if (!grp[p].empty()) upload(w, p, grp[p], st);
            upload(w, SLOT_STEP, stepping, st);
            std::fill(w.h_run.p, w.h_run.p + B, 0);
            for (int s : stepping) w.h_run.p[s] = 1;
            WFQ_HIP(hipMemcpyAsync(w.run.p, w.h_run.p, B * sizeof(int), hipMemcpyHostToDevice, st));
            WFQ_HIP(hipStreamSynchronize(st));   // the pinned lists are rewritten by the next call
        };
        lists();
        std::vector<int> it0(B, 0);
        for (int s : active) it0[s] = ss[s].iters;
        const DcgsArgs da{w.h1.p, w.h2.p, w.Hu.p, w.R.p, w.cs.p, w.sn.p, w.g.p, w.est.p, w.tol_abs.p, w.flags.p,
                          w.ksteps.p, w.run.p, w.nu.p, w.inv_h.p, w.gam.p, w.irho.p, w.norm2.p};
        // graphs only where steps are chunked and no per-launch events are recorded
        GraphCache* gc = (chunk > 1 && !tm.on()) ? graphs : nullptr;
        // steps k = 0 .. m: step k forms the product of the newest direction (k < m) and completes
        // column k - 1 (k >= 1); the last step only completes column m - 1
        for (int k0 = 0; k0 <= m && !stepping.empty();) {
            const int ns = (int)stepping.size();
            // steps until the next read-back: the chunk, the end of the cycle, or the first system
            // that could pass max_iter (a step completes at most one column)
            int c = std::min(chunk, m + 1 - k0);
            for (int s : stepping) c = std::min(c, o.max_iter - ss[s].iters);
            auto step = [&](int k) {
                const bool with_z = k < m;
                if (with_z) {
                    // the operator on the newest direction, one block product per precision group
                    for (int p = 0; p < 3; ++p) {
                        if (grp[p].empty()) continue;
                        const int ng = (int)grp[p].size();
                        const double* scale = k == 0 ? w.inv_beta.p : w.inv_h.p;
                        tm.begin(st);
                        if (bj) {
                            // u = M^-1 v: the product is taken of u, and u is the shifted term
                            bj_pack(p, w.Vb, k, w.sys[p].p, ng, scale, w.bj_P.p, w.npad, w.Ub, x_block(w, p), w.npad,
                                    w.run.p, st);
                            tm.end(st, KC_PRECOND, 8.0 * 64 * n * ng, ng * n * (512.0 + 48 + 2 * elem_size(p)));
                        } else {
                            pack_columns(p, w.Vb, w.sys[p].p, ng, k, scale, true, x_block(w, p), w.npad, st,
                                         w.run.p);
                            tm.end(st, KC_PACK, 0, ng * n * (32.0 + 2 * elem_size(p)));
                        }
                        block_product(S, w, p, 2 * ng, tm, st);
                        tm.begin(st);
                        if (w.Yp64.p)
                            spmm_shift_pairs(S, p == WFQ_PREC_FP64, y_block(w, p), w.npad,
                                             p == WFQ_PREC_FP64 ? (void*)w.Yp64.p : (void*)w.Yp32.p, w.sys[p].p,
                                             ng, w.z.p, w.Vb, bj ? 0 : k, k + 1, st, bj ? &w.Ub : nullptr);
                        else
                            spmm_shift(S, p == WFQ_PREC_FP64, y_block(w, p), w.npad, w.sys[p].p, ng, w.z.p, w.Vb,
                                       bj ? 0 : k, k + 1, st, false, bj ? &w.Ub : nullptr);
                        tm.end(st, KC_SPMM, 4.0 * S.nnz * ng + 8 * n * ng,
                               12.0 * S.nnz + ng * n * (2.0 * out_size(p) + 16 + 16));
                    }
                    if (w.rc_active) {
                        // keep the new direction orthogonal to C; C^H A u is kept for B
                        tm.begin(st);
                        rc_project(w.rc, w.Vb, k + 1, nullptr, w.sys[SLOT_STEP].p, ns, w.run.p, S.n, nullptr, 0, st);
                        tm.end(st, KC_RECYCLE, 8.0 * n * ns * w.rc.kmax, 32.0 * n * ns * (w.rc.kmax + 1));
                    }
                }
                // one fused sweep of dots, the Hessenberg column and its rotation, one update sweep
                const int* sl = w.sys[SLOT_STEP].p;
                tm.begin(st);
                dcgs_dots(w.Vb, S.n, sl, ns, k, with_z, w.partial.p, w.mdim, w.run.p, st);
                reduce_dots(S.n, sl, ns, with_z ? 2 * k + 1 : k, w.partial.p, 2 * w.mdim, w.h1.p, st, w.run.p);
                tm.end(st, KC_DOT, 16.0 * n * ns * (k + 1), 16.0 * n * ns * (k + 2));
                tm.begin(st);
                dcgs_coeff(sl, ns, k, with_z, w.mdim, da, st);
                tm.end(st, KC_GIVENS, 0, 0);
                if (with_z && w.rc_active) rc_bcol(w.rc, sl, ns, w.run.p, k, w.mdim, w.h1.p, w.irho.p, st);
                if (with_z) {
                    tm.begin(st);
                    dcgs_update(w.Vb, S.n, sl, ns, k, w.mdim, da, st);
                    tm.end(st, KC_UPDATE, 16.0 * n * ns * k, 16.0 * n * ns * (k + 4));
                }
            };
            const GraphKey key{w.rc_active ? 2 : 0, k0, c, ns, (int)grp[0].size(), (int)grp[1].size(),
                               (int)grp[2].size()};
            run_chunk(gc, S, key, st, [&] {
                for (int k = k0; k < k0 + c; ++k) step(k);
            });
            k0 += c;
            // est, flags and ksteps: the whole region, laid out for the work space's batch size (a
            // batch may hold fewer systems than that)
            WFQ_HIP(hipMemcpyAsync(w.step_host.p, w.step_dev.p, w.step_dev.count * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
            WFQ_HIP(hipStreamSynchronize(st));
            std::vector<int> next;
            for (int s : stepping) {
                ss[s].iters = it0[s] + w.h_ksteps.p[s];   // columns completed in this cycle
                ss[s].est_end = w.h_est.p[s];
                const int f = w.h_flags.p[s];
                if (f & 4) {
                    ss[s].status = WFQ_ENUMERIC;
                    continue;
                }
                if (f == 0 && ss[s].iters < o.max_iter) next.push_back(s);
            }
            const bool changed = next.size() != stepping.size();
            stepping.swap(next);
            if (changed && !stepping.empty()) lists();
            if (k0 % 10 == 0) progress_line(o, "gmres", ss[active[0]].cycles, k0, stepping.size(), -1.0, t0);
        }
        // drop systems that hit NaN
        std::vector<int> act2;
        for (int s : active) {
            if (ss[s].status == WFQ_ENUMERIC) {
                ss[s].done = true;
                ss[s].t_done = ms_since(t0);
            } else {
                act2.push_back(s);
            }
        }
        active.swap(act2);
        if (active.empty()) break;
        // x += V y, then the FP64 refinement residual
        const int na = (int)active.size();
        upload(w, SLOT_ACT, active, st);
        WFQ_HIP(hipMemcpyAsync(w.ksteps.p, w.h_ksteps.p, B * sizeof(int), hipMemcpyHostToDevice, st));
        tm.begin(st);
        tri_solve(w.sys[SLOT_ACT].p, na, w.ksteps.p, w.mdim, w.R.p, w.g.p, w.y.p, st);
        if (bj) {
            // x += M^-1 (V y)
            WFQ_HIP(hipMemsetAsync(w.bj_U.p, 0, w.bj_U.count * sizeof(double), st));
            x_update(w.Vb, w.Ub, S.n, w.sys[SLOT_ACT].p, na, w.ksteps.p, w.y.p, w.mdim, st);
            tm.end(st, KC_XUPDATE, 0, 16.0 * n * na * (m + 2));
            tm.begin(st);
            bj_add(w.sys[SLOT_ACT].p, na, w.bj_P.p, w.npad, w.Ub, w.Xb, st);
            tm.end(st, KC_PRECOND, 8.0 * 64 * n * na, na * n * (512.0 + 48));
        } else {
            x_update(w.Vb, w.Xb, S.n, w.sys[SLOT_ACT].p, na, w.ksteps.p, w.y.p, w.mdim, st);
            if (w.rc_active) rc_xfix(w.rc, w.Xb, w.sys[SLOT_ACT].p, na, w.ksteps.p, w.y.p, w.mdim, S.n, st);
            tm.end(st, KC_XUPDATE, 0, 16.0 * n * na * (m + 2));
        }
        fp64_residual(S, w, active, tm, st);
        WFQ_HIP(hipMemcpyAsync(w.h_beta.p, w.beta.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipMemcpyAsync(w.h_qT.p, w.qT.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipStreamSynchronize(st));
        std::vector<int> still;
        const double now = ms_since(t0);
        for (int s : active) {
            const double beta_prev = ss[s].beta;
            ss[s].beta = w.h_beta.p[s];
            ss[s].relres = ss[s].beta / ss[s].bnorm;
            ss[s].qT = w.h_qT.p[s];
            if (!std::isfinite(ss[s].beta)) {
                ss[s].status = WFQ_ENUMERIC;
                ss[s].done = true;
                ss[s].t_done = now;
            } else if (ss[s].relres <= tol) {
                ss[s].done = true;
                ss[s].t_done = now;
            } else if (ss[s].iters >= o.max_iter) {
                ss[s].status = WFQ_ENOCONV;
                ss[s].done = true;
                ss[s].t_done = now;
            } else {
                if (o.escalate && ss[s].prec != WFQ_PREC_FP64 && needs_escalation(ss[s].beta, beta_prev, ss[s].est_end))
                    ss[s].prec = escalate_prec(S, ss[s].prec);
                still.push_back(s);
            }
        }
        if (o.progress) {
            double worst = 0.0;
            for (int s : active) worst = std::max(worst, ss[s].relres);
            progress_line(o, "gmres refinement", ss[active[0]].cycles, 0, still.size(), worst, t0);
        }
        active.swap(still);
    }
}

// ---- multi-shift GMRES: one real Arnoldi basis of L T per direction for all frequencies

int ms_dim(const wfq_solve_opts& o, int64_t n) {
    const int64_t m = o.shift_dim > 0 ? o.shift_dim : 400;
    return (int)std::max<int64_t>(1, std::min<int64_t>(m, std::min<int64_t>(n, o.max_iter)));
}

uint64_t ms_bytes(const Structure& S, const wfq_solve_opts& o, int B, int n_dir) {
    const uint64_t m = ms_dim(o, S.n), np = S.npad, nwc = wave_chunks(S.n);
    uint64_t b = (uint64_t)n_dir * (m + 1) * np * 8;            // bases
    if (o.precision == WFQ_PREC_FP64) b *= 2;                    // and their products T u_j
    b += (uint64_t)n_dir * m * (m + 1) * 8 * (o.precision == WFQ_PREC_FP64 ? 2 : 1);   // Hessenberg (and S)
    b += (uint64_t)n_dir * (2 * (m + 1) * nwc * 8 + nwc * 8 + (m + 2) * 16);   // partials, h1, h2
    b += (uint64_t)n_dir * (3 * (m + 1) + 3) * 8;                // dots, hp, gamma, 1 / rho, nu
    b += np * 32;                                                // the interleaved product
    b += (uint64_t)B * (m * (m + 1) / 2) * 16;                   // R, packed
    b += (uint64_t)B * (m * 40 + (m + 1) * 16 + 64);             // cs, sn, y, g, scalars
    return b + (1u << 20);
}

// the all-reduced-precision residual floor is taken as this many times the relative error of one product
constexpr double kRelaxFloor = 100.0;

// Relative error of the first shared-basis product in `prec` against FP64, max over directions:
// ||L (T_prec - T) v0|| / ||L T v0|| with v0 = b / ||b||. Leaves slot 0 of every direction normalised
// and inv_h = 1 (so the first step of the phase packs v0 as it is); uses slots 1 and 2 as scratch.
double ms_product_error(const Structure& S, Work& w, int prec, const std::vector<double>& beta, hipStream_t st) {
    MsWork& q = w.ms;
    const int nd = w.n_dir;
    const int m = w.shape.ms_m, mdim1 = m + 1, pslots = m + 2;
    const int64_t n = S.n, np = S.npad;
    // v0 and L T v0 with FP64 T (slot 2), then L T_prec v0 (slot 1)
    ms_pack(WFQ_PREC_FP64, q.V.p, np, mdim1, 0, q.dirs.p, nd, q.inv_h.p, w.X64.p, np, st);
    tx_any(S, WFQ_PREC_FP64, w.X64.p, w.Y64.p, nd, st);
    ms_spmm(S, true, w.Y64.p, np, q.dirs.p, nd, q.V.p, mdim1, 2, nullptr, st);
    std::vector<double> ones(nd, 1.0);
    h2d_sync(S, q.inv_h.p, ones.data(), nd * sizeof(double), st);
    ms_pack(prec, q.V.p, np, mdim1, 0, q.dirs.p, nd, q.inv_h.p, x_block(w, prec), np, st);
    tx_any(S, prec, x_block(w, prec), const_cast<void*>(y_block(w, prec)), nd, st);
    ms_spmm(S, prec == WFQ_PREC_FP64, y_block(w, prec), np, q.dirs.p, nd, q.V.p, mdim1, 1, nullptr, st);
    // ||slot 2||^2, then slot 2 -= slot 1 with the squared norm of the difference per 64-row block
    ms_dot(q.V.p, n, np, mdim1, 0, 2, q.dirs.p, nd, q.part.p, pslots, true, st);
    ms_reduce(q.dirs.p, nd, q.part.p, pslots, n, 1, q.h1.p, st);
    std::vector<double> coef((size_t)nd * pslots, 0.0);
    for (int d = 0; d < nd; ++d) coef[(size_t)d * pslots + 1] = 1.0;
    h2d_sync(S, q.h2.p, coef.data(), coef.size() * sizeof(double), st);
    ms_update(q.V.p, n, np, mdim1, 2, 2, q.dirs.p, nd, q.h2.p, pslots, q.nrm.p, st);
    std::vector<double> h1((size_t)nd * pslots), nrm((size_t)nd * (np / 64));
    d2h_sync(S, h1.data(), q.h1.p, h1.size() * sizeof(double), st);
    d2h_sync(S, nrm.data(), q.nrm.p, nrm.size() * sizeof(double), st);
    double delta = 0.0;
    for (int d = 0; d < nd; ++d) {
        if (!(beta[d] > 0.0)) continue;
        double e2 = 0.0;
        for (int64_t b = 0; b < np / 64; ++b) e2 += nrm[(size_t)d * (np / 64) + b];
        const double r2 = h1[(size_t)d * pslots];
        if (r2 > 0.0) delta = std::max(delta, std::sqrt(e2 / r2));
    }
    return delta;
}

// Runs the shared-basis phase for the systems of one batch and leaves each system's iterate in
// w.Xb (zero where the phase could not help); ss[s].iters = steps of the shared basis it used.
void msgmres_phase(const Structure& S, Work& w, std::vector<SysState>& ss, double tol, const wfq_solve_opts& o,
                   Timer& tm, hipStream_t st, std::chrono::steady_clock::time_point t0, GraphCache* graphs) {
    const int B = (int)ss.size();
    const int nd = w.n_dir;
    const int m = ms_dim(o, S.n);
    const int mdim1 = m + 1, pslots = m + 2;
    const int64_t n = S.n, np = S.npad, nwc = wave_chunks(S.n);
    const int prec = o.precision;
    const double dn = (double)n;
    MsWork& q = w.ms;
    if (w.shape.ms_m != m) throw Error{WFQ_EDEVICE, "multi-shift work space of the wrong dimension"};
    w.ms_tv_ready = false;
    // with every product of the basis in FP64 the products are kept, and T x of each iterate is then
    // the same combination of them as x is of the basis
    bool keep_tv = q.TV.p != nullptr;
    double *V = q.V.p, *H = q.H.p, *part = q.part.p, *h1 = q.h1.p, *h2 = q.h2.p, *nrm = q.nrm.p, *inv_h = q.inv_h.p;
    double *cs = q.cs.p, *est = q.est.p, *tol_abs = q.tol_abs.p;
    double2 *sn = q.sn.p, *g = q.g.p, *R = q.R.p, *y = q.y.p, *z = q.z.p;
    int *dirs = q.dirs.p, *sdir = q.sdir.p, *sys = q.sys.p, *flags = q.flags.p, *ksteps = q.ksteps.p;
    int *grp_sys = q.grp_sys.p, *grp_dir = q.grp_dir.p, *run = q.run.p;
    int *h_dirs = q.h_dirs.p, *h_sys = q.h_sys.p, *h_k = q.h_k.p;
    double* h_nrm = q.h_nrm.p;

    // v_0 of direction d is b_d / ||b_d||
    for (int d = 0; d < nd; ++d) {
        WFQ_HIP(hipMemcpyAsync(V + (size_t)d * mdim1 * np, w.b.p + (size_t)d * np, np * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
        h_dirs[d] = d;
    }
    WFQ_HIP(hipMemcpyAsync(dirs, h_dirs, nd * sizeof(int), hipMemcpyHostToDevice, st));
    ms_dot(V, n, np, mdim1, 0, 0, dirs, nd, part, pslots, true, st);
    ms_reduce(dirs, nd, part, pslots, n, 1, h1, st);
    WFQ_HIP(hipMemcpyAsync(h_nrm, h1, (size_t)nd * pslots * sizeof(double), hipMemcpyDeviceToHost, st));
    WFQ_HIP(hipStreamSynchronize(st));
    std::vector<double> beta(nd), invb(nd);
    for (int d = 0; d < nd; ++d) {
        beta[d] = std::sqrt(h_nrm[(size_t)d * pslots]);
        invb[d] = beta[d] > 0.0 ? 1.0 / beta[d] : 0.0;
    }
    {
        // g = beta e_1 (system-minor: entry 0 of every system first)
        std::vector<double2> gh((size_t)B * (m + 1), make_double2(0.0, 0.0)), zh(B);
        std::vector<double> th(B);
        std::vector<int> dh(B);
        for (int s = 0; s < B; ++s) {
            gh[(size_t)s] = make_double2(beta[ss[s].dir], 0.0);
            th[s] = tol * beta[ss[s].dir];
            dh[s] = ss[s].dir;
            zh[s] = ss[s].z;
        }
        h2d_sync(S, g, gh.data(), gh.size() * sizeof(double2), st);
        h2d_sync(S, tol_abs, th.data(), B * sizeof(double), st);
        h2d_sync(S, sdir, dh.data(), B * sizeof(int), st);
        h2d_sync(S, z, zh.data(), B * sizeof(double2), st);
        h2d_sync(S, inv_h, invb.data(), nd * sizeof(double), st);
        WFQ_HIP(hipStreamSynchronize(st));
    }
    // Precision of the shared basis's products. With relaxation (ms_relax != 0 and a reduced
    // `precision`) the first steps run with FP64 T and the rest in `precision` once every unconverged
    // frequency's residual estimate is below the switch level: in an inexact Arnoldi process the error
    // of the product at step j reaches the final residual scaled by the residual of step j (Simoncini &
    // Szyld 2003; Bouras & Fraysse 2005), so the late steps tolerate the larger error.
    int cur = prec;
    double switch_at = 0.0;
    const bool relax = o.ms_relax != 0.0 && prec != WFQ_PREC_FP64 && have_copy(S, WFQ_PREC_FP64) && m >= 3;
    if (relax) {
        cur = WFQ_PREC_FP64;
        if (o.ms_relax > 0.0) {
            switch_at = o.ms_relax;
        } else {
            const double delta = ms_product_error(S, w, prec, beta, st);
            // the residual floor of a basis built entirely in `precision` is taken as kRelaxFloor times the
            // relative error of one product; switching at level s adds about s times that floor
            switch_at = delta > 0.0 ? std::min(1.0, std::max(tol, 0.5 * tol / (kRelaxFloor * delta))) : 1.0;
        }
        if (o.progress) {
            std::fprintf(stderr, "[wfq] multi-shift: FP64 products until every estimate is below %.3e (%.1f s)\n",
                         switch_at, ms_since(t0) / 1e3);
            std::fflush(stderr);
        }
    }
    std::vector<int> stepping;
    for (int s = 0; s < B; ++s) {
        h_k[s] = 0;
        if (!ss[s].done && beta[ss[s].dir] > 0.0) stepping.push_back(s);
    }
    // Convergence is tracked on the device (the Givens step records each system's step count and
    // clears run[s] when a flag is raised); the host compacts the lists every 8 steps. A direction
    // whose systems all stopped inside a chunk keeps stepping to the chunk's end: its extra basis
    // vectors are never used.
    constexpr int kChunk = 8;
    int na = 0, ns = 0;
    auto lists = [&]() {
        std::vector<char> used(nd, 0);
        for (int s : stepping) used[ss[s].dir] = 1;
        na = 0;
        for (int d = 0; d < nd; ++d)
            if (used[d]) h_dirs[na++] = d;
        ns = (int)stepping.size();
        std::memcpy(h_sys, stepping.data(), ns * sizeof(int));
        std::fill(w.h_run.p, w.h_run.p + B, 0);
        for (int s : stepping) w.h_run.p[s] = 1;
        WFQ_HIP(hipMemcpyAsync(dirs, h_dirs, na * sizeof(int), hipMemcpyHostToDevice, st));
        WFQ_HIP(hipMemcpyAsync(sys, h_sys, ns * sizeof(int), hipMemcpyHostToDevice, st));
        WFQ_HIP(hipMemcpyAsync(run, w.h_run.p, B * sizeof(int), hipMemcpyHostToDevice, st));
        WFQ_HIP(hipStreamSynchronize(st));   // the pinned lists are rewritten by the next call
    };
    if (!stepping.empty()) lists();
    // Steps 0 .. m: step j forms the product of u_j (j < m), finalises q_j and completes column j - 1
    // of Hbar (one-reduction Gram-Schmidt), then takes that column's Givens step for every system.
    const int ps2 = 2 * mdim1;
    double *dots = q.dots.p, *hp = q.hp.p, *gam = q.gam.p, *irho = q.irho.p, *nu = q.nu.p;
    GraphCache* gc = tm.on() ? nullptr : graphs;
    // chunk length: kChunk steps, fewer when the slowest frequency's estimate, extrapolated at the
    // rate of the last chunk, reaches the tolerance sooner (fewer products after it converges)
    int next_c = kChunk;
    double worst_prev = 0.0;
    for (int j0 = 0; j0 <= m && !stepping.empty();) {
        const int c = std::min(next_c, m + 1 - j0);
        keep_tv = keep_tv && cur == WFQ_PREC_FP64;
        auto step = [&](int j) {
            const bool wz = j < m;
            if (wz) {
                // z = L T u_j (one real column per direction) into slot j + 1
                tm.begin(st);
                ms_pack(cur, V, np, mdim1, j, dirs, na, inv_h, x_block(w, cur), np, st);
                tm.end(st, KC_PACK, 0, na * dn * (16.0 + elem_size(cur)));
                double* yi = cur == WFQ_PREC_FP64 && na <= 4 && tx_is_otf_narrow(S, cur, na) ? q.Yi.p : nullptr;
                block_product(S, w, cur, na, tm, st, yi);
                tm.begin(st);
                double* tv = keep_tv ? q.TV.p : nullptr;
                ms_spmm(S, cur == WFQ_PREC_FP64, y_block(w, cur), np, dirs, na, V, mdim1, j + 1, tv, st, yi);
                // L is read once for all directions (up to four per pass)
                tm.end(st, KC_SPMM, 2.0 * S.nnz * na,
                       12.0 * S.nnz * ((na + 3) / 4) + na * dn * (out_size(cur) + 8 + (tv ? 8 : 0)));
            }
            // one sweep of dots against q_0 .. q_{j-1} and u, one update sweep
            tm.begin(st);
            ms_dcgs_dot(V, n, np, mdim1, j, wz, dirs, na, part, ps2, st);
            ms_reduce(dirs, na, part, ps2, n, wz ? 2 * j + 2 : j + 1, dots, st);
            tm.end(st, KC_DOT, (wz ? 4.0 : 2.0) * dn * na * (j + 1), 8.0 * dn * na * (j + (wz ? 2 : 1)));
            tm.begin(st);
            ms_dcgs_coeff(dirs, na, j, wz, m, dots, ps2, hp, H, keep_tv ? q.Sm.p : nullptr, nu, inv_h, gam, irho, st);
            if (wz)
                ms_dcgs_update(V, n, np, mdim1, j, dirs, na, dots, ps2, gam, irho, nrm, nu, inv_h, st);
            tm.end(st, KC_UPDATE, wz ? 4.0 * dn * na * j : 0.0, wz ? 8.0 * dn * na * (j + 4) : 0.0);
            // every unconverged frequency of those directions: one Givens step on column j - 1 of
            // Hbar + z Ibar
            if (j >= 1) {
                tm.begin(st);
                ms_givens(sys, ns, j - 1, m, sdir, z, H, cs, sn, g, R, B, est, tol_abs, flags, run, ksteps, st);
                tm.end(st, KC_GIVENS, 0, 0);
            }
        };
        run_chunk(gc, S, GraphKey{1, j0, c, ns, na, cur, keep_tv ? 1 : 0}, st, [&] {
            for (int j = j0; j < j0 + c; ++j) step(j);
        });
        j0 += c;
        WFQ_HIP(hipMemcpyAsync(w.h_flags.p, flags, B * sizeof(int), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipMemcpyAsync(w.h_est.p, est, B * sizeof(double), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipMemcpyAsync(w.h_ksteps.p, ksteps, B * sizeof(int), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipStreamSynchronize(st));
        std::vector<int> next;
        double worst = 0.0;
        for (int s : stepping) {
            const int f = w.h_flags.p[s];
            h_k[s] = (f & 4) ? 0 : w.h_ksteps.p[s];   // NaN: leave the system to batched GMRES from x = 0
            ss[s].est_end = w.h_est.p[s];
            if (f == 0) {
                next.push_back(s);
                worst = std::max(worst, w.h_est.p[s] / beta[ss[s].dir]);
            }
        }
        if (relax && cur != prec && worst <= switch_at) {
            cur = prec;
            if (o.progress) {
                std::fprintf(stderr, "[wfq] multi-shift: products in the reduced precision from step %d\n", j0);
                std::fflush(stderr);
            }
        }
        next_c = kChunk;
        if (worst > 0.0 && worst_prev > 0.0 && worst < worst_prev) {
            const double rate = std::pow(worst / worst_prev, 1.0 / c);   // per step
            const double left = std::log(tol / worst) / std::log(rate);   // steps to the tolerance
            if (left < kChunk - 1) next_c = std::max(1, (int)std::ceil(left) + 1);   // + the Givens lag
        }
        worst_prev = worst;
        const bool changed = next.size() != stepping.size();
        stepping.swap(next);
        if (changed && !stepping.empty()) lists();
        progress_line(o, "multi-shift", 0, j0, stepping.size(), worst, t0);
    }
    // iterates: y = R^-1 g, x = V y (groups of systems of one direction share the basis reads)
    std::vector<int> withk;
    for (int s = 0; s < B; ++s)
        if (h_k[s] > 0) withk.push_back(s);
    WFQ_HIP(hipMemcpyAsync(ksteps, h_k, B * sizeof(int), hipMemcpyHostToDevice, st));
    std::vector<int> gs, gd;
    for (int d = 0; d < nd; ++d) {
        std::vector<int> mem;
        for (int s = 0; s < B; ++s)
            if (ss[s].dir == d) mem.push_back(s);
        for (size_t q = 0; q < mem.size(); q += kMsGroup) {
            for (int t = 0; t < kMsGroup; ++t) gs.push_back(q + t < mem.size() ? mem[q + t] : -1);
            gd.push_back(d);
        }
    }
    const int ngrp = (int)gd.size();
    if (gs.size() > q.grp_sys.count || gd.size() > q.grp_dir.count)
        throw Error{WFQ_EDEVICE, "multi-shift system groups exceed their work space"};
    h2d_sync(S, grp_sys, gs.data(), gs.size() * sizeof(int), st);
    h2d_sync(S, grp_dir, gd.data(), gd.size() * sizeof(int), st);
    tm.begin(st);
    if (!withk.empty()) {
        std::memcpy(h_sys, withk.data(), withk.size() * sizeof(int));
        WFQ_HIP(hipMemcpyAsync(sys, h_sys, withk.size() * sizeof(int), hipMemcpyHostToDevice, st));
        ms_solve(sys, (int)withk.size(), ksteps, m, R, B, g, y, st);
    }
    ms_xupdate(V, n, np, mdim1, grp_sys, grp_dir, ngrp, ksteps, y, m, w.Xb, st);
    // the kept products are of u_0 .. u_{k-1} = Q S: T x = T U (S^-1 y), so y becomes S^-1 y
    if (keep_tv && !withk.empty()) ms_sinv(sys, (int)withk.size(), ksteps, m, q.Sm.p, sdir, y, st);
    tm.end(st, KC_XUPDATE, 0, 0);
    WFQ_HIP(hipStreamSynchronize(st));
    q.ngrp = ngrp;
    w.ms_tv_ready = keep_tv;
    for (int s = 0; s < B; ++s) ss[s].iters += h_k[s];
    if (o.progress) progress_line(o, "multi-shift done", 0, 0, stepping.size(), -1.0, t0);
}

// J-symmetric QMR from BCG (J = T) with FP64 refinement every o.restart steps; systems whose Lanczos
// process breaks down are returned in `broken` (their QMR iterate stays in slot 5) for a GMRES
// fallback.
void qmr_batch(const Structure& S, Work& w, std::vector<SysState>& ss, double tol, const wfq_solve_opts& o,
               Timer& tm, hipStream_t st, std::chrono::steady_clock::time_point t0, std::vector<int>& broken) {
    const int B = (int)ss.size();
    const double n = (double)S.n;
    const Basis Q = w.Vb;
    const Basis XQ = slot_view(Q, 5);
    {
        std::vector<double2> zh(B);
        std::vector<int> dh(B);
        for (int s = 0; s < B; ++s) {
            zh[s] = ss[s].z;
            dh[s] = ss[s].dir;
        }
        h2d_sync(S, w.z.p, zh.data(), B * sizeof(double2), st);
        h2d_sync(S, w.dir.p, dh.data(), B * sizeof(int), st);
        WFQ_HIP(hipMemsetAsync(w.V.p, 0, w.V.count * sizeof(double), st));
    }
    std::vector<int> all(B);
    for (int s = 0; s < B; ++s) all[s] = s;
    upload(w, SLOT_ACT, all, st);
    copy_rhs(S, w.sys[SLOT_ACT].p, B, w.b.p, w.dir.p, Q, w.norm2.p, (int)w.nblk, st);   // r = b (x0 = 0)
    sumsq(w.sys[SLOT_ACT].p, B, w.norm2.p, (int)w.nblk, w.beta.p, st);
    WFQ_HIP(hipMemcpyAsync(w.h_beta.p, w.beta.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
    WFQ_HIP(hipStreamSynchronize(st));
    std::vector<int> active;
    for (int s = 0; s < B; ++s) {
        ss[s].bnorm = ss[s].beta = w.h_beta.p[s];
        if (ss[s].bnorm == 0.0) {
            ss[s].relres = 0.0;
            ss[s].done = true;
            ss[s].t_done = ms_since(t0);
        } else if (!std::isfinite(ss[s].bnorm)) {
            ss[s].status = WFQ_ENUMERIC;
            ss[s].done = true;
        } else {
            active.push_back(s);
        }
    }
    const int nblk = (int)w.nblk;
    while (!active.empty()) {
        // cycle start: x = xq, p = T p = 0, s = r, tau = ||r||
        const int na = (int)active.size();
        upload(w, SLOT_ACT, active, st);
        std::vector<double> t2(B, 0.0);
        std::vector<int> fh(B, 1);
        for (int s : active) {
            t2[s] = ss[s].beta * ss[s].beta;
            ss[s].cycles += 1;
        }
        h2d_sync(S, w.tau2.p, t2.data(), B * sizeof(double), st);
        h2d_sync(S, w.first.p, fh.data(), B * sizeof(int), st);
        qmr_restart(w.sys[SLOT_ACT].p, na, Q, st);
        WFQ_HIP(hipStreamSynchronize(st));
        double2* rho_new = w.rho_a.p;
        double2* rho_old = w.rho_b.p;
        std::vector<int> stepping;
        for (int s : active)
            if (ss[s].iters < o.max_iter) stepping.push_back(s);
        for (int k = 0; k < o.restart && !stepping.empty(); ++k) {
            const int ns = (int)stepping.size();
            std::vector<int> grp[3];
            for (int s : stepping) grp[ss[s].prec].push_back(s);
            for (int p = 0; p < 3; ++p) {
                if (grp[p].empty()) continue;
                const int ng = (int)grp[p].size();
                upload(w, p, grp[p], st);
                tm.begin(st);
                pack_columns(p, Q, w.sys[p].p, ng, 0, nullptr, false, x_block(w, p), w.npad, st);
                tm.end(st, KC_PACK, 0, ng * n * (16.0 + 2 * elem_size(p)));
                block_product(S, w, p, 2 * ng, tm, st);
                tm.begin(st);
                qmr_rho(p == WFQ_PREC_FP64, y_block(w, p), w.npad, w.sys[p].p, ng, Q, S.n, w.part_sig.p, nblk, st);
                reduce_complex(w.sys[p].p, ng, w.part_sig.p, nblk, rho_new, st);
                qmr_dirs(p == WFQ_PREC_FP64, y_block(w, p), w.npad, w.sys[p].p, ng, Q, S.n, rho_new, rho_old,
                         w.first.p, w.tpb.p, st);
                tm.end(st, KC_QMR, 0, ng * n * (16.0 * 5 + 4 * out_size(p)));
            }
            upload(w, SLOT_STEP, stepping, st);
            const int* sl = w.sys[SLOT_STEP].p;
            tm.begin(st);
            qmr_q(S, sl, ns, Q, w.z.p, w.tpb.p, w.part_sig.p, w.part_nrm.p, nblk, st);
            tm.end(st, KC_SPMM, 4.0 * S.nnz * ns, 12.0 * S.nnz + ns * n * 48.0);
            tm.begin(st);
            qmr_sigma(sl, ns, w.part_sig.p, w.part_nrm.p, nblk, rho_new, w.sigma.p, w.flags.p,
                      o.qmr_breakdown > 0.0 ? o.qmr_breakdown : 1e-14, st);
            qmr_xr(sl, ns, Q, S.n, rho_new, w.sigma.p, w.norm2.p, nblk, st);
            qmr_weights(sl, ns, w.norm2.p, nblk, w.tau2.p, w.eta.p, w.first.p, st);
            qmr_smooth(sl, ns, Q, S.n, w.eta.p, w.norm2.p, nblk, st);
            sumsq(sl, ns, w.norm2.p, nblk, w.snorm.p, st);
            tm.end(st, KC_QMR, 0, ns * n * 16.0 * 12);
            WFQ_HIP(hipMemcpyAsync(w.h_flags.p, w.flags.p, B * sizeof(int), hipMemcpyDeviceToHost, st));
            WFQ_HIP(hipMemcpyAsync(w.h_snorm.p, w.snorm.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
            WFQ_HIP(hipStreamSynchronize(st));
            std::swap(rho_new, rho_old);
            std::vector<int> next;
            for (int s : stepping) {
                ss[s].iters += 1;
                ss[s].est_end = w.h_snorm.p[s];
                const int f = w.h_flags.p[s];
                if (f & 4) {
                    ss[s].status = WFQ_ENUMERIC;
                    continue;
                }
                if (f & 8) {
                    ss[s].status = WFQ_EBREAKDOWN;
                    continue;
                }
                if (w.h_snorm.p[s] > 0.5 * tol * ss[s].bnorm && ss[s].iters < o.max_iter) next.push_back(s);
            }
            stepping.swap(next);
            if ((k + 1) % 10 == 0) progress_line(o, "qmr", ss[active[0]].cycles, k + 1, stepping.size(), -1.0, t0);
        }
        // systems that broke down leave for the GMRES fallback; NaN ends a system
        std::vector<int> act2;
        for (int s : active) {
            if (ss[s].status == WFQ_ENUMERIC) {
                ss[s].done = true;
                ss[s].t_done = ms_since(t0);
            } else if (ss[s].status == WFQ_EBREAKDOWN) {
                broken.push_back(s);
            } else {
                act2.push_back(s);
            }
        }
        active.swap(act2);
        if (active.empty()) break;
        // FP64 refinement point: r = b - (L T + z I) xq into slot 0
        upload(w, SLOT_ACT, active, st);
        {
            const int na2 = (int)active.size();
            tm.begin(st);
            pack_columns(WFQ_PREC_FP64, XQ, w.sys[SLOT_ACT].p, na2, 0, nullptr, false, w.X64.p, w.npad, st);
            tm.end(st, KC_PACK, 0, 32.0 * n * na2);
            block_product(S, w, WFQ_PREC_FP64, 2 * na2, tm, st);
            tm.begin(st);
            residual(S, w.Y64.p, w.npad, w.sys[SLOT_ACT].p, na2, w.z.p, XQ, w.b.p, w.dir.p, Q, w.norm2.p, nblk,
                     w.qtq.p, st);
            sumsq(w.sys[SLOT_ACT].p, na2, w.norm2.p, nblk, w.beta.p, st);
            sumsq(w.sys[SLOT_ACT].p, na2, w.qtq.p, nblk, w.qT.p, st);
            tm.end(st, KC_RESID, 0, 12.0 * S.nnz + na2 * n * 56.0);
        }
        WFQ_HIP(hipMemcpyAsync(w.h_beta.p, w.beta.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipMemcpyAsync(w.h_qT.p, w.qT.p, B * sizeof(double), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipStreamSynchronize(st));
        std::vector<int> still;
        const double now = ms_since(t0);
        for (int s : active) {
            const double beta_prev = ss[s].beta;
            ss[s].beta = w.h_beta.p[s];
            ss[s].qT = w.h_qT.p[s];
            ss[s].relres = ss[s].beta / ss[s].bnorm;
            if (!std::isfinite(ss[s].beta)) {
                ss[s].status = WFQ_ENUMERIC;
                ss[s].done = true;
                ss[s].t_done = now;
            } else if (ss[s].relres <= tol) {
                ss[s].done = true;
                ss[s].t_done = now;
            } else if (ss[s].iters >= o.max_iter) {
                ss[s].status = WFQ_ENOCONV;
                ss[s].done = true;
                ss[s].t_done = now;
            } else {
                if (o.escalate && ss[s].prec != WFQ_PREC_FP64 && needs_escalation(ss[s].beta, beta_prev, ss[s].est_end))
                    ss[s].prec = escalate_prec(S, ss[s].prec);
                still.push_back(s);
            }
        }
        if (o.progress) {
            double worst = 0.0;
            for (int s : active) worst = std::max(worst, ss[s].relres);
            progress_line(o, "qmr refinement", ss[active[0]].cycles, 0, still.size(), worst, t0);
        }
        active.swap(still);
    }
}

// Warm starts across neighbouring frequencies (two passes): per direction, the systems of the batch
// sorted by frequency; every second one and the last are solved first from q0 = 0, and each of the
// others starts from the linear interpolation in z of its two solved neighbours (q depends on the
// frequency only through z). A neighbour that failed leaves the system at q0 = 0.
struct WarmPlan {
    std::vector<int> first, second, tgt, a, b;
    std::vector<double2> t;
};

WarmPlan warm_plan(const std::vector<SysState>& ss, int n_dir) {
    WarmPlan p;
    for (int d = 0; d < n_dir; ++d) {
        std::vector<int> mem;
        for (int s = 0; s < (int)ss.size(); ++s)
            if (ss[s].dir == d) mem.push_back(s);
        std::stable_sort(mem.begin(), mem.end(), [&](int x, int y) { return ss[x].omega < ss[y].omega; });
        const int c = (int)mem.size();
        for (int q = 0; q < c; ++q) {
            if (q % 2 == 0 || q == c - 1)
                p.first.push_back(mem[q]);
            else
                p.second.push_back(mem[q]);
        }
    }
    return p;
}

// Recycle spaces of the second-pass systems: the solutions of the k nearest solved systems of the
// same direction (by frequency), made into C = A U' with C^H C = I by two Gram-Schmidt passes per
// vector; a vector whose remainder is below 1e-12 ||b|| (the neighbours' solutions are nearly
// dependent) is dropped (set to zero).
void recycle_setup(const Structure& S, Work& w, const std::vector<SysState>& ss, const WarmPlan& p, hipStream_t st) {
    const int k = w.rc.kmax;
    const int nt = (int)p.second.size();
    if (nt == 0 || k == 0) return;
    std::fill(w.h_rc_kk.p, w.h_rc_kk.p + w.h_rc_kk.count, 0);
    std::vector<double> scale(nt, 0.0);
    for (int t = 0; t < nt; ++t) {
        const int s = p.second[t];
        std::vector<int> cand;
        for (int f : p.first)
            if (ss[f].dir == ss[s].dir && ss[f].status == WFQ_OK) cand.push_back(f);
        std::stable_sort(cand.begin(), cand.end(), [&](int x, int y) {
            return std::fabs(ss[x].omega - ss[s].omega) < std::fabs(ss[y].omega - ss[s].omega);
        });
        const int kc = std::min<int>(k, (int)cand.size());
        for (int i = 0; i < k; ++i) w.h_rc_nbr.p[(size_t)t * k + i] = i < kc ? cand[i] : -1;
        w.h_rc_kk.p[s] = kc;
        scale[t] = kc > 0 ? ss[cand[0]].bnorm : 0.0;
    }
    upload(w, SLOT_ACT, p.second, st);
    WFQ_HIP(hipMemcpyAsync(w.rc_kk.p, w.h_rc_kk.p, w.rc_kk.count * sizeof(int), hipMemcpyHostToDevice, st));
    WFQ_HIP(hipMemcpyAsync(w.rc_nbr.p, w.h_rc_nbr.p, (size_t)nt * k * sizeof(int), hipMemcpyHostToDevice, st));
    const int* sys = w.sys[SLOT_ACT].p;
    rc_init(w.rc, w.Vb, w.Xb, w.b.p, w.dir.p, w.z.p, sys, nt, w.rc_nbr.p, S.n, st);
    for (int i = 0; i < k; ++i) {
        rc_orth_step(w.rc, i, sys, nt, S.n, w.norm2.p, (int)w.nblk, st);
        rc_orth_step(w.rc, i, sys, nt, S.n, w.norm2.p, (int)w.nblk, st);
        sumsq(sys, nt, w.norm2.p, (int)w.nblk, w.rc_inv.p, st);
        WFQ_HIP(hipMemcpyAsync(w.h_rc_inv.p, w.rc_inv.p, w.rc_inv.count * sizeof(double), hipMemcpyDeviceToHost, st));
        WFQ_HIP(hipStreamSynchronize(st));
        for (int t = 0; t < nt; ++t) {
            const int s = p.second[t];
            const double nrm = w.h_rc_inv.p[s];
            w.h_rc_inv.p[s] = (i < w.h_rc_kk.p[s] && nrm > 1e-12 * scale[t] && std::isfinite(nrm)) ? 1.0 / nrm : 0.0;
        }
        WFQ_HIP(hipMemcpyAsync(w.rc_inv.p, w.h_rc_inv.p, w.rc_inv.count * sizeof(double), hipMemcpyHostToDevice, st));
        rc_scale(w.rc, i, sys, nt, w.rc_inv.p, st);
        WFQ_HIP(hipStreamSynchronize(st));   // the pinned mirror is rewritten by the next vector
    }
}

// the interpolation lists of the second pass, once the first pass is done
void warm_lists(WarmPlan& p, const std::vector<SysState>& ss) {
    for (int s : p.second) {
        // neighbours: the nearest solved systems of the same direction below and above in frequency
        int a = -1, b = -1;
        for (int f : p.first) {
            if (ss[f].dir != ss[s].dir) continue;
            if (ss[f].omega <= ss[s].omega && (a < 0 || ss[f].omega > ss[a].omega)) a = f;
            if (ss[f].omega >= ss[s].omega && (b < 0 || ss[f].omega < ss[b].omega)) b = f;
        }
        if (a < 0 || b < 0 || ss[a].status != WFQ_OK || ss[b].status != WFQ_OK) continue;
        const double2 za = ss[a].z, zb = ss[b].z, zs = ss[s].z;
        const double dr = zb.x - za.x, di = zb.y - za.y, den = dr * dr + di * di;
        const double nr = zs.x - za.x, ni = zs.y - za.y;
        const double2 t = den > 0.0 ? make_double2((nr * dr + ni * di) / den, (ni * dr - nr * di) / den)
                                    : make_double2(0.0, 0.0);
        p.tgt.push_back(s);
        p.a.push_back(a);
        p.b.push_back(b);
        p.t.push_back(t);
    }
}

}  // namespace

uint64_t batch_bytes(const Structure& S, const wfq_solve_opts& o, int B, int n_dir) {
    const uint64_t np = S.npad;
    const uint64_t mdim = o.algorithm == WFQ_QMR ? (uint64_t)kQmrSlots : (uint64_t)o.restart + 1;
    const uint64_t mpad = round_up(2 * (int64_t)B, kColPad);
    uint64_t b = 0;
    b += (uint64_t)B * mdim * 2 * np * 8;       // basis
    b += (uint64_t)B * 2 * np * 8;              // solution
    b += (uint64_t)n_dir * np * 8;              // right-hand sides
    b += mpad * np * 16;                        // FP64 block in/out
    if (o.precision == WFQ_PREC_FP32 || o.precision == WFQ_PREC_BF16) b += mpad * np * 8;
    if (o.precision == WFQ_PREC_BF16) b += mpad * np * 6;
    if ((int64_t)np > kPairsFrom) b += mpad * np * (o.precision == WFQ_PREC_FP64 ? 8 : 12);   // interleaved planes
    const uint64_t nwc = wave_chunks(S.n);
    b += (uint64_t)B * 2 * mdim * nwc * 16;     // fused dot partials (two entries per basis vector)
    b += (uint64_t)B * 2 * mdim * mdim * 16;    // R and the Hessenberg matrix before rotations
    b += (uint64_t)B * (mdim * 64 + 2 * np * 8 / 1);  // small arrays + output staging
    b += (uint64_t)B * (np / 256 + 1) * 8;             // block partials of x^H T x
    if (o.recycle > 0 && o.algorithm == WFQ_GMRES)      // recycle spaces (C and U'), dots, B
        b += (uint64_t)B * o.recycle * (2 * 2 * np * 8 + (wave_chunks(S.n) + mdim + 1) * 16 + 4) + B * 16;
    b += std::min<uint64_t>(kSplitWsCap, 7 * mpad * np * 8);   // split-k partial tiles
    if (o.algorithm == WFQ_MSGMRES) b += ms_bytes(S, o, B, n_dir);
    if (o.algorithm == WFQ_QMR) b += (uint64_t)B * 2 * np * 8;   // compact T p
    if (o.block_jacobi) b += np * 64 * 8 + (uint64_t)B * (np * 64 * 8 + 2 * np * 8);   // C, P, u
    return b;
}

int solve_all(Structure& S, const double* omegas_eV, int n_omega, const double* dirs, int n_dir, double tol,
              const wfq_solve_opts& o, const SolveOutputs& out, hipStream_t st, KernelStat* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    const double kHartreeEV = 27.211386245988;
    const int total = n_omega * n_dir;
    const double E0 = o.E0 != 0.0 ? o.E0 : 1.0;
    int prec = o.precision;
    if (!have_copy(S, prec))
        throw Error{WFQ_EINVAL, S.t_mode == WFQ_TMODE_OTF
                                    ? "matrix-free T runs in FP32 or FP64"
                                    : "the stored copy of T for the requested precision was not built (store_mask)"};
    if (!have_copy(S, WFQ_PREC_FP64))
        throw Error{WFQ_EINVAL, "FP64 refinement needs the FP64 copy of T (store_mask must include WFQ_STORE_FP64)"};
    if (o.block_jacobi && !S.T64)
        throw Error{WFQ_EINVAL, "block-Jacobi preconditioning needs the stored FP64 T (not matrix-free)"};

    // batch size: as many systems as fit the budget
    // (systems index the y/z dimension of several grids: at most 32768 per batch)
    int B = std::min(o.max_batch > 0 ? std::min(o.max_batch, total) : total, 32768);
    const uint64_t avail = S.budget > S.bytes ? S.budget - S.bytes : 0;
    while (B > 1 && S.budget && batch_bytes(S, o, B, n_dir) > avail) B = (B + 1) / 2;
    if (S.budget && batch_bytes(S, o, B, n_dir) > avail)
        throw Error{WFQ_ENOMEM, "not enough device memory for one system's Krylov work space"};
    // the symmetric narrow products (matrix-free FP64, up to 4 columns at a time) need one partial sum
    // per 1 024-atom block and row: reserved here when it exceeds the ordinary work-space cap and the
    // budget leaves room beside the batch; otherwise those products take the one-sided form
    {
        const uint64_t sym4 = otf_sym_bytes(S, 4);
        const bool reserve = sym4 > kSplitWsCap && sym4 <= kSymWsCap &&
                             (!S.budget || batch_bytes(S, o, B, n_dir) + sym4 <= avail);
        S.sym_ws_allowed = reserve ? sym4 : 0;
        if (S.split_ws && S.split_ws_bytes > std::max(kSplitWsCap, S.sym_ws_allowed)) {
            // a larger work space held from an earlier solve is not covered by this one's budget
            WFQ_HIP(hipFree(S.split_ws));
            S.split_ws = nullptr;
            S.split_ws_bytes = 0;
            ++S.epoch;
        }
    }

    const bool qmr = o.algorithm == WFQ_QMR;
    WorkShape sh;
    sh.B = B;
    sh.m = qmr ? kQmrSlots - 1 : o.restart;
    sh.n_dir = n_dir;
    sh.prec = prec;
    sh.ms_m = o.algorithm == WFQ_MSGMRES ? ms_dim(o, S.n) : 0;
    sh.qmr = qmr;
    sh.bj = o.block_jacobi && o.algorithm == WFQ_GMRES;
    sh.rk = (o.recycle > 0 && o.algorithm == WFQ_GMRES && n_omega >= 3) ? o.recycle : 0;
    GraphCache* graphs = nullptr;
    std::unique_ptr<Work> own;   // a work space too large to keep on the handle
    Work& w = solve_work(S, sh, graphs, own);
    clear_work(w, st);
    if (!o.graphs || !st) graphs = nullptr;
    // right-hand sides b_k = E0 L r_k (shared by every frequency)
    h2d_sync(S, w.d_dirs.p, dirs, 3 * n_dir * sizeof(double), st);
    build_rhs(S, w.d_dirs.p, n_dir, E0, w.b.p, S.npad, st);
    WFQ_HIP(hipStreamSynchronize(st));
    Timer tm(stats != nullptr);
    int worst = WFQ_OK;
    for (int s0 = 0; s0 < total; s0 += B) {
        const int nb = std::min(B, total - s0);
        std::vector<SysState> ss(nb);
        for (int s = 0; s < nb; ++s) {
            const int gid = s0 + s;
            ss[s].omega = omegas_eV[gid / n_dir] / kHartreeEV;
            ss[s].dir = gid % n_dir;
            const double om = ss[s].omega;
            ss[s].z = make_double2(-(om * om) / S.W, -(om / S.tau) / S.W);   // z = -(w^2 + i w / tau) / W
            ss[s].prec = prec;
        }
        if (o.algorithm == WFQ_MSGMRES) {
            // shared-basis phase, then batched GMRES from its iterates (FP64 residual first)
            msgmres_phase(S, w, ss, tol, o, tm, st, t0, graphs);
            gmres_batch(S, w, ss, tol, o, tm, st, t0, graphs, true);
        } else if (!qmr && sh.rk > 0) {
            // subspace recycling: every second frequency from zero, then the others by GMRES augmented
            // with the span of their nearest solved neighbours' solutions
            WarmPlan wp = warm_plan(ss, n_dir);
            gmres_batch(S, w, ss, tol, o, tm, st, t0, graphs, false, &wp.first);
            recycle_setup(S, w, ss, wp, st);
            w.rc_active = true;
            try {
                gmres_batch(S, w, ss, tol, o, tm, st, t0, graphs, false, &wp.second);
            } catch (...) {
                w.rc_active = false;
                throw;
            }
            w.rc_active = false;
        } else if (!qmr && o.warm_start && n_omega >= 3) {
            WarmPlan wp = warm_plan(ss, n_dir);
            gmres_batch(S, w, ss, tol, o, tm, st, t0, graphs, false, &wp.first);
            warm_lists(wp, ss);
            const int nt = (int)wp.tgt.size();
            if (nt > 0) {
                h2d_sync(S, w.warm_sys.p, wp.tgt.data(), nt * sizeof(int), st);
                h2d_sync(S, w.warm_a.p, wp.a.data(), nt * sizeof(int), st);
                h2d_sync(S, w.warm_b.p, wp.b.data(), nt * sizeof(int), st);
                h2d_sync(S, w.warm_t.p, wp.t.data(), nt * sizeof(double2), st);
                interp_start(w.warm_sys.p, nt, w.warm_a.p, w.warm_b.p, w.warm_t.p, w.Xb, S.n, st);
                WFQ_HIP(hipStreamSynchronize(st));
            }
            gmres_batch(S, w, ss, tol, o, tm, st, t0, graphs, true, &wp.second);
        } else if (!qmr) {
            gmres_batch(S, w, ss, tol, o, tm, st, t0, graphs);
        } else {
            std::vector<int> broken;
            qmr_batch(S, w, ss, tol, o, tm, st, t0, broken);
            if (!broken.empty()) {
                // GMRES fallback from the QMR iterate of each broken-down system, in groups whose
                // work space fits what the QMR work space leaves of the budget; a system for which
                // not even a one-system group fits keeps its QMR iterate and ends as WFQ_EBREAKDOWN
                wfq_solve_opts og = o;
                og.algorithm = WFQ_GMRES;
                og.restart = std::min(50, std::max(o.restart, 10));
                const uint64_t used = batch_bytes(S, o, B, n_dir);
                const uint64_t left = S.budget ? (avail > used ? avail - used : 0) : ~0ull;
                int G = (int)broken.size();
                while (G > 1 && batch_bytes(S, og, G, n_dir) > left) G = (G + 1) / 2;
                if (batch_bytes(S, og, G, n_dir) > left) {
                    for (int s : broken) ss[s].status = WFQ_EBREAKDOWN;
                    broken.clear();
                }
                for (size_t g0 = 0; g0 < broken.size(); g0 += G) {
                    const int nbk = (int)std::min<size_t>(G, broken.size() - g0);
                    Work wg;
                    WorkShape shg;
                    shg.B = nbk;
                    shg.m = og.restart;
                    shg.n_dir = n_dir;
                    shg.prec = prec;
                    make_work(wg, S, shg);
                    clear_work(wg, st);
                    WFQ_HIP(hipMemcpyAsync(wg.b.p, w.b.p, w.b.count * sizeof(double), hipMemcpyDeviceToDevice, st));
                    std::vector<SysState> sg(nbk);
                    for (int q = 0; q < nbk; ++q) {
                        const int s = broken[g0 + q];
                        sg[q] = ss[s];
                        sg[q].status = WFQ_OK;
                        sg[q].done = false;
                        WFQ_HIP(hipMemcpyAsync(wg.X.p + (size_t)q * 2 * S.npad, w.Xb.base + (size_t)s * w.Xb.sys_stride,
                                               2 * S.npad * sizeof(double), hipMemcpyDeviceToDevice, st));
                    }
                    gmres_batch(S, wg, sg, tol, og, tm, st, t0, nullptr, true);
                    for (int q = 0; q < nbk; ++q) {
                        const int s = broken[g0 + q];
                        const int iters_qmr = ss[s].iters, cycles_qmr = ss[s].cycles;
                        ss[s] = sg[q];
                        ss[s].iters += iters_qmr;
                        ss[s].cycles += cycles_qmr;
                        if (ss[s].status == WFQ_ENOCONV) ss[s].status = WFQ_EBREAKDOWN;
                        WFQ_HIP(hipMemcpyAsync(w.Xb.base + (size_t)s * w.Xb.sys_stride, wg.X.p + (size_t)q * 2 * S.npad,
                                               2 * S.npad * sizeof(double), hipMemcpyDeviceToDevice, st));
                    }
                    WFQ_HIP(hipStreamSynchronize(st));
                }
            }
        }
        // outputs of the batch
        std::vector<int> all(nb);
        for (int s = 0; s < nb; ++s) all[s] = s;
        upload(w, SLOT_ACT, all, st);
        observables(S, w.sys[SLOT_ACT].p, nb, w.Xb, E0, w.alpha.p, st);
        WFQ_HIP(hipMemcpyAsync(w.h_alpha.p, w.alpha.p, (size_t)nb * 3 * sizeof(double2), hipMemcpyDeviceToHost, st));
        if (out.on_device) {
            scatter_q(S, S.dperm, w.sys[SLOT_ACT].p, nb, w.Xb, out.q_re ? out.q_re + (size_t)s0 * S.n : nullptr,
                      out.q_im ? out.q_im + (size_t)s0 * S.n : nullptr, st);
        } else if (out.q_re || out.q_im) {
            scatter_q(S, S.dperm, w.sys[SLOT_ACT].p, nb, w.Xb, out.q_re ? w.stage_re.p : nullptr,
                      out.q_im ? w.stage_im.p : nullptr, st);
            if (out.q_re) d2h_sync(S, out.q_re + (size_t)s0 * S.n, w.stage_re.p, (size_t)nb * S.n * 8, st);
            if (out.q_im) d2h_sync(S, out.q_im + (size_t)s0 * S.n, w.stage_im.p, (size_t)nb * S.n * 8, st);
        }
        WFQ_HIP(hipStreamSynchronize(st));
        std::vector<double> are(nb * 3), aim(nb * 3);
        for (int s = 0; s < nb * 3; ++s) {
            are[s] = w.h_alpha.p[s].x;
            aim[s] = w.h_alpha.p[s].y;
        }
        if (out.alpha_re) {
            if (out.on_device)
                h2d_sync(S, out.alpha_re + (size_t)s0 * 3, are.data(), nb * 3 * 8, st);
            else
                std::memcpy(out.alpha_re + (size_t)s0 * 3, are.data(), nb * 3 * 8);
        }
        if (out.alpha_im) {
            if (out.on_device)
                h2d_sync(S, out.alpha_im + (size_t)s0 * 3, aim.data(), nb * 3 * 8, st);
            else
                std::memcpy(out.alpha_im + (size_t)s0 * 3, aim.data(), nb * 3 * 8);
        }
        if (out.on_device) WFQ_HIP(hipStreamSynchronize(st));   // are / aim are host temporaries
        for (int s = 0; s < nb; ++s) {
            const SysState& q = ss[s];
            if (out.info) {
                wfq_result& r = out.info[s0 + s];
                r.status = q.status;
                r.iters = q.iters;
                r.cycles = q.cycles;
                r.precision = q.prec;
                r.relres = q.relres;
                r.rmse = q.beta / std::sqrt((double)S.n);
                r.err_est = error_bound(S, q);
                r.t_done_ms = q.t_done;
                // Eq. (long-cross): sigma_k = (4 pi omega / c) Im(k . alpha), c in atomic units
                double ka = 0.0;
                for (int l = 0; l < 3; ++l) ka += dirs[3 * q.dir + l] * aim[(size_t)s * 3 + l];
                r.sigma = 4.0 * M_PI * q.omega / kLightAU * ka;
            }
            if (q.status != WFQ_OK && worst == WFQ_OK) worst = q.status;
            if (q.status == WFQ_ENUMERIC) worst = WFQ_ENUMERIC;
        }
    }
    tm.collect(stats);
    return worst;
}

}  // namespace wfq
