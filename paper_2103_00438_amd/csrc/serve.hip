// Request loop for spectrum jobs (one structure + frequency list + field directions each).
//
// Jobs wait in a FIFO queue. A fixed pool of max_jobs worker threads (started by wfq_serve, joined
// by wfq_serve_stop) takes them: a free worker admits the job at the head of the queue as soon as
// its estimated device footprint (stored T copies, L, Krylov work space) fits what the resident
// jobs leave of the budget, then runs it on its own HIP stream: set-up, batched solve, copy-out,
// release. Jobs that arrive while others run are admitted as soon as a worker and memory free up,
// so their work overlaps on the device. A job's arithmetic does not depend on what else is
// resident (no cross-job reductions, fixed kernel choice per shape), so its result is the same
// alone and in the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "solver.h"

using namespace wfq;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxWorkers = 64;   // upper limit of max_jobs (one worker thread per slot)

struct Job {
    uint64_t ticket = 0;
    std::vector<double> xyz, eta, omegas, dirs;
    std::vector<int32_t> species_idx;    // per-atom species (empty: none given)
    std::vector<wfq_species> species;    // the job's species table (params.species points here when run)
    wfq_params params{};
    int64_t n = 0;
    int n_omega = 0, n_dir = 0;
    uint64_t footprint = 0;
    // results
    std::vector<double> q_re, q_im, a_re, a_im;
    std::vector<wfq_result> info;
    int status = WFQ_OK;
    std::string error;
    bool done = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct wfq_server {
    wfq_serve_cfg cfg{};
    uint64_t budget = 0;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;       // worker wake-up (new job, freed memory, stop)
    std::condition_variable done_cv;  // job completion
    std::deque<std::shared_ptr<Job>> queue;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    std::vector<std::thread> workers;   // the pool: max_jobs threads for the server's lifetime
    uint64_t next_ticket = 1;
    uint64_t reserved = 0;
    int resident = 0;
    int max_resident = 0;
    bool stopping = false;
    // statistics
    std::vector<double> latencies;
    int64_t jobs_done = 0, systems_done = 0;
    double busy_ms = 0, busy_since = -1;

    double now_ms() { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
};

namespace {

uint64_t estimate_footprint(const Job& j, const wfq_serve_cfg& c) {
    const uint64_t np = (uint64_t)round_up(j.n, kPad);
    uint64_t t = 0;
    uint32_t mask = j.params.store_mask ? j.params.store_mask : (WFQ_STORE_FP64 | WFQ_STORE_FP32);
    if (mask & WFQ_STORE_FP64) t += np * np * 8;
    if (mask & WFQ_STORE_FP32) t += np * np * 4;
    if (mask & WFQ_STORE_BF16) t += np * np * 2;
    // L in CSR and ELL (up to 320 neighbours per atom for close-packed metals), the near-field
    // correction of the matrix-free products (up to ~600 entries per atom) and per-atom arrays
    t += np * 320 * 24 + np * 600 * 12 + np * 64;
    Structure probe;
    probe.n = j.n;
    probe.npad = (int64_t)np;
    t += batch_bytes(probe, c.opts, j.n_omega * j.n_dir, j.n_dir);
    return t + (64ull << 20);
}

// Runs one admitted job to completion. Never throws: any failure (including host allocation)
// becomes the job's status.
void run_job(wfq_server* srv, const std::shared_ptr<Job>& job) {
    int rc = WFQ_OK;
    std::string err;
    wfq_handle* h = nullptr;
    const int S = job->n_omega * job->n_dir;
    try {
        wfq_geometry g{job->n, job->xyz.data(), job->eta.empty() ? nullptr : job->eta.data(),
                       job->species_idx.empty() ? nullptr : job->species_idx.data()};
        wfq_params p = job->params;
        p.species = job->species.empty() ? nullptr : job->species.data();
        p.n_species = (int32_t)job->species.size();
        p.device = srv->cfg.device;
        p.device_budget = job->footprint;
        p.t_mode = WFQ_TMODE_STORED;
        rc = wfq_build(&g, &p, &h);
        if (rc == WFQ_EDISCONNECTED) rc = WFQ_OK;
        if (rc != WFQ_OK) err = wfq_last_error();
        if (rc == WFQ_OK) {
            job->q_re.assign((size_t)S * job->n, 0.0);
            job->q_im.assign((size_t)S * job->n, 0.0);
            job->a_re.assign((size_t)S * 3, 0.0);
            job->a_im.assign((size_t)S * 3, 0.0);
            job->info.assign(S, wfq_result{});
            rc = wfq_solve(h, job->omegas.data(), job->n_omega, job->dirs.data(), job->n_dir, srv->cfg.tol,
                           &srv->cfg.opts, job->q_re.data(), job->q_im.data(), job->a_re.data(), job->a_im.data(),
                           job->info.data());
            if (rc != WFQ_OK) err = wfq_last_error();
        }
    } catch (const std::bad_alloc&) {
        rc = WFQ_ENOMEM;
        err = "host allocation failed";
    } catch (const std::exception& e) {
        rc = WFQ_EDEVICE;
        err = e.what();
    }
    wfq_destroy(h);
    std::lock_guard<std::mutex> lk(srv->mu);
    job->status = rc;
    job->error = err;
    job->done = true;
    job->t_done = srv->now_ms();
    srv->reserved -= job->footprint;
    srv->resident -= 1;
    srv->latencies.push_back(job->t_done - job->t_submit);
    srv->jobs_done += 1;
    srv->systems_done += S;
    if (srv->resident == 0 && srv->busy_since >= 0) {
        srv->busy_ms += job->t_done - srv->busy_since;
        srv->busy_since = -1;
    }
    srv->cv.notify_all();
    srv->done_cv.notify_all();
}

// One worker of the pool: admits the job at the head of the queue when its footprint fits (or when
// nothing is resident), fails a job that can never fit, and exits once the server stops and the
// queue is empty. At most max_jobs jobs are resident because there are max_jobs workers.
void worker_loop(wfq_server* srv) {
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        srv->cv.wait(lk, [&] {
            if (srv->queue.empty()) return srv->stopping;
            const auto& j = srv->queue.front();
            return j->footprint > srv->budget || srv->reserved + j->footprint <= srv->budget || srv->resident == 0;
        });
        if (srv->queue.empty()) break;   // stopping and nothing left
        auto job = srv->queue.front();
        srv->queue.pop_front();
        if (job->footprint > srv->budget) {
            // can never fit: fail it instead of blocking the queue
            job->status = WFQ_ENOMEM;
            job->error = "job footprint exceeds the server's device budget";
            job->done = true;
            job->t_admit = job->t_done = srv->now_ms();
            srv->done_cv.notify_all();
            srv->cv.notify_all();
            continue;
        }
        job->t_admit = srv->now_ms();
        srv->reserved += job->footprint;
        srv->resident += 1;
        srv->max_resident = std::max(srv->max_resident, srv->resident);
        if (srv->busy_since < 0) srv->busy_since = job->t_admit;
        srv->cv.notify_all();   // the next job may fit beside this one
        lk.unlock();
        run_job(srv, job);
        lk.lock();
    }
}

int copy_out(wfq_server* s, const std::shared_ptr<Job>& job, double* q_re, double* q_im, double* alpha_re,
             double* alpha_im, wfq_result* info, wfq_job_timing* timing) {
    const size_t S = (size_t)job->n_omega * job->n_dir;
    if (!job->q_re.empty()) {
        if (q_re) std::memcpy(q_re, job->q_re.data(), S * job->n * 8);
        if (q_im) std::memcpy(q_im, job->q_im.data(), S * job->n * 8);
        if (alpha_re) std::memcpy(alpha_re, job->a_re.data(), S * 3 * 8);
        if (alpha_im) std::memcpy(alpha_im, job->a_im.data(), S * 3 * 8);
        if (info) std::memcpy(info, job->info.data(), S * sizeof(wfq_result));
    }
    if (timing) {
        timing->t_submit_ms = job->t_submit;
        timing->t_admit_ms = job->t_admit;
        timing->t_done_ms = job->t_done;
        timing->latency_ms = job->t_done - job->t_submit;
        timing->status = job->status;
        timing->n_systems = (int32_t)S;
    }
    const int rc = job->status;
    if (rc != WFQ_OK) wfq::set_error(rc, job->error);
    s->jobs.erase(job->ticket);
    return rc;
}

}  // namespace

extern "C" {

int wfq_serve(const wfq_serve_cfg* c, wfq_server** out) {
    if (out) *out = nullptr;
    if (!c || !out) {
        wfq::set_error(WFQ_EINVAL, "cfg and out must not be NULL");
        return WFQ_EINVAL;
    }
    if (c->max_jobs < 1 || c->max_jobs > kMaxWorkers || c->max_queue < 1 || !(c->tol > 0.0 && c->tol < 1.0)) {
        wfq::set_error(WFQ_EINVAL, "need max_jobs in [1, 64], max_queue >= 1, tol in (0, 1)");
        return WFQ_EINVAL;
    }
    if (c->opts.restart < 1 || c->opts.max_iter < 1 || c->opts.precision < 0 || c->opts.precision > 2 ||
        (c->opts.algorithm != WFQ_GMRES && c->opts.algorithm != WFQ_QMR && c->opts.algorithm != WFQ_MSGMRES) ||
        c->opts.shift_dim < 0 || c->opts.shift_dim > 4096 || (c->opts.algorithm != WFQ_QMR && c->opts.restart > 256)) {
        wfq::set_error(WFQ_EINVAL, "invalid solver options");
        return WFQ_EINVAL;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || c->device < 0 || c->device >= count) {
        wfq::set_error(WFQ_EDEVICE, "no such HIP device");
        return WFQ_EDEVICE;
    }
    if (hipSetDevice(c->device) != hipSuccess) {
        wfq::set_error(WFQ_EDEVICE, "hipSetDevice failed");
        return WFQ_EDEVICE;
    }
    auto* s = new wfq_server();
    s->cfg = *c;
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    s->budget = c->device_budget ? c->device_budget : (uint64_t)(0.9 * (double)free_b);
    s->t0 = Clock::now();
    try {
        for (int k = 0; k < c->max_jobs; ++k) s->workers.emplace_back(worker_loop, s);
    } catch (const std::exception&) {
        // could not start the pool: stop the workers that did start and report it
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stopping = true;
            s->cv.notify_all();
        }
        for (auto& t : s->workers) t.join();
        delete s;
        wfq::set_error(WFQ_ENOMEM, "could not start the worker threads");
        return WFQ_ENOMEM;
    }
    *out = s;
    return WFQ_OK;
}

int wfq_submit(wfq_server* s, const wfq_job* job, uint64_t* ticket) {
    if (!s || !job || !ticket || !job->geom.xyz || job->geom.n < 2 || job->n_omega < 1 || job->n_dir < 1 ||
        !job->omegas_eV || !job->dirs) {
        wfq::set_error(WFQ_EINVAL, "invalid job");
        return WFQ_EINVAL;
    }
    for (int k = 0; k < job->n_omega; ++k)
        if (!(job->omegas_eV[k] > 0.0)) {
            wfq::set_error(WFQ_ESINGULAR, "omega <= 0 makes the system singular");
            return WFQ_ESINGULAR;
        }
    auto j = std::make_shared<Job>();
    j->n = job->geom.n;
    j->xyz.assign(job->geom.xyz, job->geom.xyz + 3 * job->geom.n);
    if (job->geom.eta) j->eta.assign(job->geom.eta, job->geom.eta + job->geom.n);
    if (job->geom.species) j->species_idx.assign(job->geom.species, job->geom.species + job->geom.n);
    j->params = job->params;
    if (job->params.n_species > 0) {
        if (!job->params.species) {
            wfq::set_error(WFQ_EINVAL, "n_species > 0 needs the species table");
            return WFQ_EINVAL;
        }
        j->species.assign(job->params.species, job->params.species + job->params.n_species);
    }
    j->params.species = nullptr;   // rewired to the job's copy when it runs
    j->n_omega = job->n_omega;
    j->n_dir = job->n_dir;
    j->omegas.assign(job->omegas_eV, job->omegas_eV + job->n_omega);
    j->dirs.assign(job->dirs, job->dirs + 3 * job->n_dir);
    j->footprint = estimate_footprint(*j, s->cfg);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
        wfq::set_error(WFQ_EINVAL, "server is stopping");
        return WFQ_EINVAL;
    }
    if ((int)s->queue.size() >= s->cfg.max_queue) {
        wfq::set_error(WFQ_EAGAIN, "queue full");
        return WFQ_EAGAIN;
    }
    j->ticket = s->next_ticket++;
    j->t_submit = s->now_ms();
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *ticket = j->ticket;
    s->cv.notify_all();
    return WFQ_OK;
}

int wfq_poll(wfq_server* s, uint64_t ticket, double* q_re, double* q_im, double* alpha_re, double* alpha_im,
             wfq_result* info, wfq_job_timing* timing) {
    if (!s) {
        wfq::set_error(WFQ_EINVAL, "server is NULL");
        return WFQ_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) {
        wfq::set_error(WFQ_ENOTFOUND, "unknown ticket");
        return WFQ_ENOTFOUND;
    }
    if (!it->second->done) {
        wfq::set_error(WFQ_EAGAIN, "not done yet");
        return WFQ_EAGAIN;
    }
    auto job = it->second;
    return copy_out(s, job, q_re, q_im, alpha_re, alpha_im, info, timing);
}

int wfq_wait(wfq_server* s, uint64_t ticket, double* q_re, double* q_im, double* alpha_re, double* alpha_im,
             wfq_result* info, wfq_job_timing* timing) {
    if (!s) {
        wfq::set_error(WFQ_EINVAL, "server is NULL");
        return WFQ_EINVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) {
        wfq::set_error(WFQ_ENOTFOUND, "unknown ticket");
        return WFQ_ENOTFOUND;
    }
    auto job = it->second;
    s->done_cv.wait(lk, [&] { return job->done; });
    return copy_out(s, job, q_re, q_im, alpha_re, alpha_im, info, timing);
}

int wfq_serve_stats(wfq_server* s, wfq_stats* out) {
    if (!s || !out) {
        wfq::set_error(WFQ_EINVAL, "bad arguments");
        return WFQ_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> lat = s->latencies;
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
        if (lat.empty()) return 0.0;
        size_t k = (size_t)std::ceil(p * lat.size()) - 1;
        return lat[std::min(k, lat.size() - 1)];
    };
    const double now = s->now_ms();
    double busy = s->busy_ms + (s->busy_since >= 0 ? now - s->busy_since : 0.0);
    out->jobs_done = s->jobs_done;
    out->systems_done = s->systems_done;
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->solves_per_s = now > 0 ? s->systems_done / (now / 1000.0) : 0.0;
    out->busy_frac = now > 0 ? busy / now : 0.0;
    out->max_resident = s->max_resident;
    return WFQ_OK;
}

void wfq_serve_stop(wfq_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv.notify_all();
    }
    // the workers drain the queue, finish their jobs and exit
    for (auto& t : s->workers)
        if (t.joinable()) t.join();
    delete s;
}

}  // extern "C"
