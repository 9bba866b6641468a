"""MI355X (gfx950) library for the omegaFQ plasmonic response problem: batched Krylov solves of
(L T + z I) q = E0 L r_k with hand-written HIP kernels. See include/wfq.h for the C interface."""

from .wfq import (  # noqa: F401
    Handle, Server, WfqError, load,
    wfq_build, wfq_destroy, wfq_solve, wfq_solve_dev, wfq_info, wfq_sample_T, wfq_export_L,
    wfq_apply_T, wfq_apply_op, wfq_rhs, wfq_kernel_stats, wfq_tx_variants, wfq_tune,
    wfq_serve, wfq_submit, wfq_poll, wfq_wait, wfq_serve_stats, wfq_serve_stop, wfq_last_error,
)
