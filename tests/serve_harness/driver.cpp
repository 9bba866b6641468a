// Request-loop harness: drives wfq_serve / wfq_submit / wfq_poll / wfq_wait / wfq_serve_stats /
// wfq_serve_stop (compiled from csrc/serve.hip) against the stand-ins of stub_lib.cpp, from several
// client threads at once. Prints one line per failed check and exits non-zero if any failed.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "wfq.h"

extern "C" {
uint64_t stub_peak_bytes();
int stub_peak_live();
void stub_reset();
}
double stub_charge(int64_t n, double omega, int dir, int64_t i, int part);

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                      \
            std::printf("\n");                             \
            ++g_fail;                                      \
        }                                                  \
    } while (0)

struct JobSpec {
    std::vector<double> xyz, om, dirs;
    int64_t n() const { return (int64_t)xyz.size() / 3; }
};

JobSpec make_job(int64_t n, int n_om, int n_dir, int seed) {
    JobSpec j;
    j.xyz.resize(3 * n);
    for (int64_t i = 0; i < 3 * n; ++i) j.xyz[i] = 1.42 * (double)i + 0.01 * seed;
    for (int k = 0; k < n_om; ++k) j.om.push_back(0.05 + 0.1 * k + 0.001 * seed);
    for (int d = 0; d < n_dir; ++d)
        for (int a = 0; a < 3; ++a) j.dirs.push_back(a == d ? 1.0 : 0.0);
    return j;
}

wfq_job as_job(const JobSpec& s) {
    wfq_job j{};
    j.geom.n = s.n();
    j.geom.xyz = s.xyz.data();
    j.geom.eta = nullptr;
    j.params.eta = 0.5;
    j.params.r0 = 1.42;
    j.params.fermi_d = 12;
    j.params.fermi_s = 1.1;
    j.params.cutoff_eps = 1e-12;
    j.params.W = 0.03;
    j.params.tau = 170;
    j.omegas_eV = s.om.data();
    j.n_omega = (int32_t)s.om.size();
    j.dirs = s.dirs.data();
    j.n_dir = (int32_t)s.dirs.size() / 3;
    return j;
}

wfq_serve_cfg config(uint64_t budget, int max_jobs, int max_queue) {
    wfq_serve_cfg c{};
    c.device_budget = budget;
    c.max_jobs = max_jobs;
    c.max_queue = max_queue;
    c.device = 0;
    c.opts.algorithm = WFQ_GMRES;
    c.opts.restart = 40;
    c.opts.max_iter = 1000;
    c.opts.precision = WFQ_PREC_FP32;
    c.tol = 1e-8;
    return c;
}

// every output of a finished job equals what the stand-in solve writes for it
void check_result(const JobSpec& s, int rc, const std::vector<double>& qr, const std::vector<double>& qi,
                  const wfq_job_timing& tm) {
    CHECK(rc == WFQ_OK, "status %d", rc);
    const int nd = (int)s.dirs.size() / 3;
    bool ok = true;
    for (size_t k = 0; k < s.om.size(); ++k)
        for (int d = 0; d < nd; ++d)
            for (int64_t i = 0; i < s.n(); ++i) {
                const size_t o = ((size_t)k * nd + d) * s.n() + i;
                ok = ok && qr[o] == stub_charge(s.n(), s.om[k], d, i, 0) && qi[o] == stub_charge(s.n(), s.om[k], d, i, 1);
            }
    CHECK(ok, "charges of a job of %lld atoms differ from the stand-in solve", (long long)s.n());
    CHECK(tm.t_done_ms >= tm.t_admit_ms && tm.t_admit_ms >= tm.t_submit_ms, "timing order");
    CHECK(tm.n_systems == (int)(s.om.size() * nd), "n_systems");
}

int wait_job(wfq_server* srv, uint64_t t, const JobSpec& s, bool poll_first, std::vector<double>* qr_out = nullptr) {
    const size_t S = s.om.size() * (s.dirs.size() / 3);
    std::vector<double> qr(S * s.n()), qi(S * s.n()), ar(S * 3), ai(S * 3);
    std::vector<wfq_result> info(S);
    wfq_job_timing tm{};
    int rc;
    if (poll_first) {
        while ((rc = wfq_poll(srv, t, qr.data(), qi.data(), ar.data(), ai.data(), info.data(), &tm)) == WFQ_EAGAIN)
            std::this_thread::yield();
    } else {
        rc = wfq_wait(srv, t, qr.data(), qi.data(), ar.data(), ai.data(), info.data(), &tm);
    }
    if (rc == WFQ_OK) check_result(s, rc, qr, qi, tm);
    if (qr_out) *qr_out = qr;
    return rc;
}

// many jobs from four client threads; results, overlap and the slot limit
void scenario_mix() {
    stub_reset();
    wfq_server* srv = nullptr;
    wfq_serve_cfg c = config(0, 3, 64);
    CHECK(wfq_serve(&c, &srv) == WFQ_OK, "serve");
    std::vector<std::thread> clients;
    for (int c = 0; c < 4; ++c)
        clients.emplace_back([srv, c] {
            for (int r = 0; r < 6; ++r) {
                JobSpec s = make_job(300 + 97 * r + 13 * c, 1 + (r + c) % 5, 1 + (r * c) % 3, 10 * c + r);
                wfq_job j = as_job(s);
                uint64_t t = 0;
                int rc = wfq_submit(srv, &j, &t);
                CHECK(rc == WFQ_OK, "submit %d", rc);
                if (rc == WFQ_OK) CHECK(wait_job(srv, t, s, r % 2 == 0) == WFQ_OK, "job failed");
            }
        });
    for (auto& t : clients) t.join();
    wfq_stats st{};
    CHECK(wfq_serve_stats(srv, &st) == WFQ_OK, "stats");
    CHECK(st.jobs_done == 24, "jobs_done %lld", (long long)st.jobs_done);
    CHECK(st.max_resident <= 3 && st.max_resident >= 2, "max_resident %d", st.max_resident);
    CHECK(stub_peak_live() <= 3, "more than max_jobs handles alive: %d", stub_peak_live());
    CHECK(st.p99_ms >= st.p50_ms && st.p50_ms > 0, "percentiles");
    wfq_serve_stop(srv);
}

// admission by footprint: the bytes reserved by resident jobs never exceed the budget
void scenario_budget() {
    stub_reset();
    const uint64_t budget = 160ull << 20;   // about two 512-atom jobs (64 MiB margin each + T + L)
    wfq_server* srv = nullptr;
    wfq_serve_cfg c = config(budget, 6, 64);
    CHECK(wfq_serve(&c, &srv) == WFQ_OK, "serve");
    std::vector<JobSpec> specs;
    std::vector<uint64_t> tickets;
    for (int k = 0; k < 10; ++k) {
        specs.push_back(make_job(400 + 10 * k, 2, 1, k));
        wfq_job j = as_job(specs.back());
        uint64_t t = 0;
        CHECK(wfq_submit(srv, &j, &t) == WFQ_OK, "submit");
        tickets.push_back(t);
    }
    for (int k = 0; k < 10; ++k) CHECK(wait_job(srv, tickets[k], specs[k], false) == WFQ_OK, "job %d", k);
    wfq_stats st{};
    wfq_serve_stats(srv, &st);
    CHECK(stub_peak_bytes() <= budget, "reserved %llu > budget %llu", (unsigned long long)stub_peak_bytes(),
          (unsigned long long)budget);
    CHECK(st.max_resident >= 2 && st.max_resident < 6, "budget should allow 2..5 resident, got %d", st.max_resident);
    wfq_serve_stop(srv);
}

// a job that can never fit ends with WFQ_ENOMEM and does not block the ones behind it
void scenario_never_fits() {
    stub_reset();
    wfq_server* srv = nullptr;
    wfq_serve_cfg c = config(160ull << 20, 2, 64);
    CHECK(wfq_serve(&c, &srv) == WFQ_OK, "serve");
    JobSpec big = make_job(4000, 1, 1, 1), small = make_job(500, 2, 2, 2);
    wfq_job jb = as_job(big), js = as_job(small);
    uint64_t tb = 0, ts = 0;
    CHECK(wfq_submit(srv, &jb, &tb) == WFQ_OK, "submit big");
    CHECK(wfq_submit(srv, &js, &ts) == WFQ_OK, "submit small");
    CHECK(wait_job(srv, tb, big, false) == WFQ_ENOMEM, "big job should fail with ENOMEM");
    CHECK(wait_job(srv, ts, small, false) == WFQ_OK, "small job");
    wfq_serve_stop(srv);
}

// bounded queue, unknown tickets, poll before completion, argument errors, stop with work pending
void scenario_queue_and_tickets() {
    stub_reset();
    wfq_server* srv = nullptr;
    wfq_serve_cfg c = config(0, 1, 2);
    CHECK(wfq_serve(&c, &srv) == WFQ_OK, "serve");
    JobSpec s = make_job(2000, 8, 3, 5);
    wfq_job j = as_job(s);
    std::vector<uint64_t> t;
    int eagain = 0;
    for (int k = 0; k < 8; ++k) {
        uint64_t tk = 0;
        const int rc = wfq_submit(srv, &j, &tk);
        if (rc == WFQ_OK) t.push_back(tk);
        else if (rc == WFQ_EAGAIN) ++eagain;
        else CHECK(false, "submit returned %d", rc);
    }
    CHECK(eagain > 0, "the queue limit was never reported");
    CHECK(wfq_poll(srv, 987654, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == WFQ_ENOTFOUND, "poll unknown");
    CHECK(wfq_wait(srv, 987654, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == WFQ_ENOTFOUND, "wait unknown");
    wfq_job bad = j;
    bad.n_omega = 0;
    uint64_t tb = 0;
    CHECK(wfq_submit(srv, &bad, &tb) == WFQ_EINVAL, "empty frequency list accepted");
    std::vector<double> om0{0.0};
    bad = j;
    bad.omegas_eV = om0.data();
    bad.n_omega = 1;
    CHECK(wfq_submit(srv, &bad, &tb) == WFQ_ESINGULAR, "omega = 0 accepted");
    for (uint64_t tk : t) CHECK(wait_job(srv, tk, s, false) == WFQ_OK, "queued job");
    for (uint64_t tk : t)
        CHECK(wfq_poll(srv, tk, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == WFQ_ENOTFOUND,
              "a retrieved ticket is still known");
    // leave two jobs queued and stop: they are drained before stop returns
    for (int k = 0; k < 2; ++k) {
        uint64_t tk = 0;
        CHECK(wfq_submit(srv, &j, &tk) == WFQ_OK, "submit before stop");
    }
    wfq_serve_stop(srv);
    CHECK(stub_peak_live() <= 1, "more than one job resident with max_jobs = 1");
    wfq_serve_cfg badc = config(0, 0, 2);
    wfq_server* s2 = nullptr;
    CHECK(wfq_serve(&badc, &s2) == WFQ_EINVAL && s2 == nullptr, "max_jobs = 0 accepted");
    badc = config(0, 65, 2);
    CHECK(wfq_serve(&badc, &s2) == WFQ_EINVAL && s2 == nullptr, "max_jobs = 65 accepted");
}

}  // namespace

int main(int argc, char** argv) {
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 3;
    for (int r = 0; r < rounds; ++r) {
        scenario_mix();
        scenario_budget();
        scenario_never_fits();
        scenario_queue_and_tickets();
    }
    std::printf("%s: %d failed checks\n", g_fail ? "FAIL" : "OK", g_fail);
    return g_fail ? 1 : 0;
}
