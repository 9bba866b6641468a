// Batched solver drivers (host side). One call solves every (frequency, field) system of one
// structure; systems share each block product with T.
#pragma once

#include "common.h"

namespace wfq {

struct SolveOutputs {
    double* q_re = nullptr;       // [S][n] (device when on_device, else host), may be NULL
    double* q_im = nullptr;
    double* alpha_re = nullptr;   // [S][3] (device when on_device, else host), may be NULL
    double* alpha_im = nullptr;
    wfq_result* info = nullptr;   // host [S], may be NULL
    bool on_device = false;
};

// omegas in eV (> 0), dirs [n_dir][3] unit vectors. Returns the worst per-system status.
int solve_all(Structure& S, const double* omegas_eV, int n_omega, const double* dirs, int n_dir, double tol,
              const wfq_solve_opts& o, const SolveOutputs& out, hipStream_t st, KernelStat* stats);

// Bytes of device work space a batch of `batch` systems needs (GMRES basis, QMR vectors, blocks).
uint64_t batch_bytes(const Structure& S, const wfq_solve_opts& o, int batch, int n_dir);

}  // namespace wfq
