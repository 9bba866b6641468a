// Stand-ins for wfq_build / wfq_solve / wfq_destroy used by the request-loop harness: they keep the
// library's contracts (argument checks, outputs written in full, one handle per job) and account
// the device bytes that live handles reserve, so the harness can check admission by footprint.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <mutex>
#include <thread>

#include "solver.h"

namespace {
thread_local std::string g_err;
std::mutex g_mu;
uint64_t g_used = 0, g_peak = 0;
int g_live = 0, g_peak_live = 0;
}  // namespace

struct wfq_handle {
    int64_t n = 0;
    uint64_t bytes = 0;
};

namespace wfq {
uint64_t batch_bytes(const Structure& S, const wfq_solve_opts&, int B, int n_dir) {
    return (uint64_t)B * (uint64_t)S.npad * 4096 + (uint64_t)n_dir * 1024;
}
void set_error(int, const std::string& msg) { g_err = msg; }
}  // namespace wfq

// the value every stand-in solve writes for charge i of system (omega, dir)
double stub_charge(int64_t n, double omega, int dir, int64_t i, int part) {
    return std::sin(0.001 * (double)n + 1.7 * omega + 0.3 * dir + 1e-3 * (double)i + 0.5 * part);
}

extern "C" {

uint64_t stub_peak_bytes() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_peak;
}
int stub_peak_live() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_peak_live;
}
void stub_reset() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_used = g_peak = 0;
    g_live = g_peak_live = 0;
}

const char* wfq_last_error(void) { return g_err.c_str(); }

int wfq_build(const wfq_geometry* g, const wfq_params* p, wfq_handle** out) {
    if (out) *out = nullptr;
    if (!g || !p || !out || g->n < 2 || !g->xyz) {
        g_err = "bad arguments";
        return WFQ_EINVAL;
    }
    auto* h = new wfq_handle();
    h->n = g->n;
    h->bytes = p->device_budget;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_used += h->bytes;
        g_peak = std::max(g_peak, g_used);
        g_live += 1;
        g_peak_live = std::max(g_peak_live, g_live);
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(1 + g->n % 3));
    *out = h;
    return WFQ_OK;
}

void wfq_destroy(wfq_handle* h) {
    if (!h) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_used -= h->bytes;
        g_live -= 1;
    }
    delete h;
}

int wfq_solve(wfq_handle* h, const double* omegas_eV, int32_t n_omega, const double* dirs, int32_t n_dir, double tol,
              const wfq_solve_opts* o, double* q_re, double* q_im, double* alpha_re, double* alpha_im,
              wfq_result* info) {
    if (!h || !omegas_eV || !dirs || n_omega < 1 || n_dir < 1 || !o || !(tol > 0)) {
        g_err = "bad arguments";
        return WFQ_EINVAL;
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(2 + (h->n / 100) % 5));
    for (int k = 0; k < n_omega; ++k)
        for (int d = 0; d < n_dir; ++d) {
            const int64_t s = (int64_t)k * n_dir + d;
            for (int64_t i = 0; i < h->n; ++i) {
                if (q_re) q_re[s * h->n + i] = stub_charge(h->n, omegas_eV[k], d, i, 0);
                if (q_im) q_im[s * h->n + i] = stub_charge(h->n, omegas_eV[k], d, i, 1);
            }
            for (int l = 0; l < 3; ++l) {
                if (alpha_re) alpha_re[s * 3 + l] = omegas_eV[k] + l;
                if (alpha_im) alpha_im[s * 3 + l] = dirs[3 * d + l];
            }
            if (info) {
                info[s] = wfq_result{};
                info[s].relres = 0.5 * tol;
                info[s].iters = (int)(h->n % 17);
            }
        }
    return WFQ_OK;
}

}  // extern "C"
