/*
 * wfq.h - C interface of the MI355X (gfx950) omegaFQ response library.
 *
 * Problem (Lafiosca, Giovannini, Benzi, Cappelli, arXiv 2103.00438, Section
 * "Theoretical Model" and subsection "Properties of the omegaFQ linear system"):
 * N atoms at positions r_i carry complex charges q. For a uniform field of
 * amplitude E0 along unit direction k and angular frequency omega, q solves
 *
 *     (L T + z(omega) I) q = b_k,      b_k = E0 L (r . k),
 *
 * which is Eq. (wfq-a-matrix), (A - z I) q = R, multiplied by -1, with
 *   T = D       damped Coulomb matrix, Eq. (d-matrix): T_ij = erf(r_ij / sqrt(d_i^2 + d_j^2)) / r_ij,
 *               T_ii = eta_i, d_i = sqrt(2/pi) / eta_i (width-from-hardness equation);
 *   L = P - Kbar  Eqs. (k-tot-factor), (a-matrix-product): Kbar_ij = (1 - f(r_ij)) / r_ij with the
 *               Fermi damping f of Eq. (fermi), P_ii = sum_k Kbar_ik;
 *   z(omega) = -(omega^2 + i omega / tau) / W   Eq. (z-def), W = 2 n0 A (effective area folded in);
 *   R, V       Eqs. (r-vector-def) and (potential), V_i = -E0 (r_i . k).
 * The polarisability returned is alpha_lk = sum_i r_{i,l} q_i^(k) / E0, whose diagonal gives the
 * absorption cross section of Eq. (long-cross), sigma_k = (4 pi omega / c) Im alpha_kk.
 *
 * Units at this interface: positions in Angstrom, frequencies in eV, everything else in Hartree
 * atomic units (eta, W, tau, E0). Inside, the library works in atomic units and may reorder atoms;
 * every output is returned in the caller's atom order.
 *
 * Ownership: every input pointer is read during the call only; the caller keeps ownership. A
 * handle owns all device memory of one structure (T copies, L, work space) until wfq_destroy.
 * Calls on one handle must not overlap (a handle is single-threaded); distinct handles may be used
 * from distinct threads. Errors: every int-returning function returns 0 (WFQ_OK) or a WFQ_E* code
 * and stores a message readable with wfq_last_error() on the calling thread. Arguments are checked
 * before any device work is issued; on an argument error nothing is modified.
 */
#ifndef WFQ_H
#define WFQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define WFQ_OK             0
#define WFQ_EINVAL         1  /* invalid argument (N < 2, NaN/Inf, coincident atoms, eta <= 0, ...) */
#define WFQ_ENOMEM         2  /* device footprint exceeds the budget or the device is out of memory */
#define WFQ_EDEVICE        3  /* HIP runtime error or no usable gfx950 device */
#define WFQ_ESINGULAR      4  /* omega <= 0: z = 0 and L T is singular (rows of L sum to zero) */
#define WFQ_ENOCONV        5  /* some system did not reach tol within max_iter (results still filled) */
#define WFQ_EBREAKDOWN     6  /* QMR breakdown that the GMRES fallback could not repair */
#define WFQ_ENUMERIC       7  /* NaN or Inf met during a solve */
#define WFQ_EAGAIN         8  /* serving queue full, or result not ready yet */
#define WFQ_EDISCONNECTED  9  /* warning from wfq_build: the Kbar graph is not connected */
#define WFQ_ENOTFOUND     10  /* unknown serving ticket */

/* ------------------------------------------------------------------ enumerations */
#define WFQ_PREC_FP64  0      /* precision of the T products inside the Krylov iterations */
#define WFQ_PREC_FP32  1
#define WFQ_PREC_BF16  2

#define WFQ_GMRES      0      /* restarted GMRES(m), Saad & Schultz (Section "Solution strategies") */
#define WFQ_QMR        1      /* J-symmetric QMR from BCG with J = T, no look-ahead (same section) */
#define WFQ_MSGMRES    2      /* multi-shift GMRES: one real Krylov basis of L T per field direction
                                 serves every frequency (the frequency is only the diagonal shift z of
                                 Eq. wfq-a-matrix; shift invariance of Krylov spaces, conclusions) */

#define WFQ_TMODE_AUTO    0   /* stored T when it fits the budget, else on the fly */
#define WFQ_TMODE_STORED  1   /* dense T kept in device memory */
#define WFQ_TMODE_OTF     2   /* T elements recomputed in every product (matrix-free section) */

/* bits of wfq_params.store_mask: which stored copies of T wfq_build creates */
#define WFQ_STORE_FP64  1u
#define WFQ_STORE_FP32  2u
#define WFQ_STORE_BF16  4u

/* wfq_params.material: how the Drude prefactor W = 2 n0 A of Eq. (z-def) is obtained */
#define WFQ_MATERIAL_W          0   /* W given in wfq_params.W */
#define WFQ_MATERIAL_GRAPHENE2D 1   /* 2D sheet (honeycomb, nearest-neighbour distance lattice_nn): the Drude
                                       weight of the sheet is eps_F / pi (atomic units), Eqs. (2d-eff-mass),
                                       (n-2d) read as the Drude weight of a 2D electron gas */
#define WFQ_MATERIAL_METAL3D    2   /* FCC metal (nearest-neighbour distance lattice_nn): Drude weight
                                       n_e / m* with n_e = valence / (volume per atom), n0 of the
                                       Theoretical Model section with m* the effective mass */

typedef struct wfq_handle wfq_handle;
typedef struct wfq_server wfq_server;

typedef struct {
    int64_t        n;       /* number of atoms, >= 2 */
    const double*  xyz;     /* [n][3] positions, Angstrom, host memory */
    const double*  eta;     /* [n] per-atom hardness (Hartree), or NULL (species or wfq_params.eta) */
    const int32_t* species; /* [n] species index of each atom, 0 .. n_species - 1, or NULL (all species 0);
                               used when wfq_params.n_species > 0 */
} wfq_geometry;

/* one atomic species: hardness and the equilibrium distance r0 of Eq. (fermi); a pair of species
 * (a, b) uses r0_ab = (r0_a + r0_b) / 2 */
typedef struct {
    double eta;   /* Hartree, > 0 */
    double r0;    /* Angstrom, > 0 */
} wfq_species;

typedef struct {
    double   eta;            /* hardness (Hartree) when wfq_geometry.eta is NULL; > 0 */
    double   r0;             /* equilibrium distance r0 of Eq. (fermi), Angstrom; > 0 */
    double   fermi_d;        /* d of Eq. (fermi); > 0 */
    double   fermi_s;        /* s of Eq. (fermi); > 0 */
    double   cutoff_eps;     /* Kbar_ij kept where 1 - f(r_ij) >= cutoff_eps; in (0, 0.5) */
    double   W;              /* 2 n0 A (atomic units); > 0 */
    double   tau;            /* Drude relaxation time (atomic units); > 0 */
    int32_t  t_mode;         /* WFQ_TMODE_* */
    uint32_t store_mask;     /* WFQ_STORE_* bits; 0 = FP64 and FP32 */
    uint64_t device_budget;  /* bytes the handle may use on the device; 0 = 90% of free memory */
    int32_t  device;         /* HIP device ordinal */
    /* material (Theoretical Model section): with material != WFQ_MATERIAL_W and W == 0 the library
       computes W from the material data by the Drude sum-rule closure W = 2 Omega D / S, where Omega is
       the area (2D) or volume (3D) per atom of the ideal lattice, D the Drude weight of the material and
       S = sum_j (1 - f(r_0j)) x_0j^2 / r_0j over one site's ideal-lattice neighbours inside the cutoff
       (so that W R^T L R per atom equals Omega D, the macroscopic Drude response, through the
       high-frequency term R^T L R / z); a W > 0 given above overrides it */
    int32_t  material;       /* WFQ_MATERIAL_* */
    double   fermi_energy;   /* WFQ_MATERIAL_GRAPHENE2D: Fermi energy eps_F (eV), > 0 */
    double   valence;        /* WFQ_MATERIAL_METAL3D: free electrons per atom, > 0 */
    double   eff_mass;       /* WFQ_MATERIAL_METAL3D: effective mass m* (electron masses); 0 = 1 */
    double   lattice_nn;     /* nearest-neighbour distance of the ideal lattice (Angstrom); 0 = r0 of species 0 */
    /* species: n_species > 0 gives every atom the {eta, r0} of its species (wfq_geometry.species;
       wfq_geometry.eta, when not NULL, still overrides eta per atom); 0 = one species {eta, r0} above */
    int32_t            n_species;
    const wfq_species* species;   /* [n_species], host memory, read during the call */
} wfq_params;

/*
 * wfq_material_weight - the W that wfq_build would use for these parameters (the override, or the
 * sum-rule closure of the material), computed on the host; no device is needed. WFQ_EINVAL for an
 * unknown material or missing material data.
 */
int wfq_material_weight(const wfq_params* p, double* W);

typedef struct {
    int32_t algorithm;   /* WFQ_GMRES, WFQ_QMR or WFQ_MSGMRES */
    int32_t restart;     /* GMRES and MSGMRES: Krylov dimension m per refinement cycle (1..256);
                            QMR: steps between FP64 checks (>= 1) */
    int32_t max_iter;    /* cap on T products per system (inner iterations); > 0 */
    int32_t precision;   /* WFQ_PREC_*: precision of T inside the iterations (FP64 refinement always) */
    double  E0;          /* field amplitude (atomic units); 0 means 1 */
    int32_t max_batch;   /* systems solved together; 0 = as many as fit the budget */
    int32_t timing;      /* nonzero: time every kernel launch with HIP events (wfq_kernel_stats) */
    int32_t escalate;    /* nonzero: a system whose FP64 residual stalls moves to the next precision */
    int32_t progress;    /* nonzero: one line on stderr per refinement point and every 10 inner steps */
    int32_t shift_dim;   /* MSGMRES: largest dimension of the shared basis (0 = 400, at most 4096).
                            Per direction the Arnoldi process runs on the real matrix L T from b_k until
                            every frequency's shifted least-squares residual is <= tol ||b_k|| or the
                            dimension is reached; each system then continues from that iterate in
                            batched GMRES(restart) with FP64 refinement (usually: one FP64 residual).
                            Device memory per direction: 8 (shift_dim + 1) N_p bytes for the basis, and
                            as much again in FP64 solves, which keep the products T u_j so that the FP64
                            residual of the shared-basis iterates needs no further product of T. */
    int32_t graphs;      /* nonzero: for structures of at most 8192 atoms (whose inner steps are read back in
                            chunks of 8) and for the multi-shift phase, a chunk of steps whose launch
                            sequence repeats (same first step, length and list sizes) is captured as a HIP
                            graph the second time it occurs and replayed after that; results are bitwise
                            the same as without. The inner kernels of such small solves run back to back
                            on the device already, so replays gain only a few percent, while each capture
                            costs milliseconds: off by default. Needs a stream other than the null stream
                            (wfq_solve_dev). Graphs and the work space stay on the handle until a solve of
                            another shape or wfq_destroy. */
    int32_t warm_start;  /* GMRES only, nonzero: warm starts across neighbouring frequencies instead of
                            q0 = 0 (the paper's protocol). Per direction, the systems of a batch sorted by
                            frequency: every second one and the highest are solved first from q0 = 0; each
                            of the others then starts from the linear interpolation in z of its two solved
                            neighbours (q depends on the frequency only through z) and runs batched
                            GMRES with FP64 refinement from there. Needs n_omega >= 3 (else ignored);
                            WFQ_EINVAL with another algorithm. */
    int32_t block_jacobi; /* GMRES only, nonzero: right preconditioning with the exact 64 x 64 diagonal
                            blocks M_s of L T + z_s I over runs of 64 atoms in the library's internal
                            (spatially sorted) order, so GMRES runs on (L T + z_s I) M_s^-1 and minimises
                            the true residual (a project extension; the paper runs its solvers
                            unpreconditioned). Each block is inverted once per solve in FP64 (Gauss-Jordan,
                            partial pivoting) and kept in complex FP32: every system holds N x 64 entries
                            (512 bytes per atom) and each inner step reads them once. The rounded inverse
                            is the preconditioner on both sides, so the solution is unchanged. The block
                            products keep the chosen precision. A singular block gives NaN and the
                            system ends with WFQ_ENUMERIC. Needs the stored FP64 T (WFQ_EINVAL otherwise, and with another
                            algorithm or with warm_start). */
    double  qmr_breakdown; /* QMR: a step breaks down (no look-ahead) when |sigma| <= qmr_breakdown ||T p|| ||q||,
                            sigma = p^T T q the bilinear form of the step; 0 = 1e-14. Broken-down systems
                            continue in GMRES from their QMR iterate (in groups that fit the budget left by
                            the QMR work space; WFQ_EBREAKDOWN if none fits or GMRES does not converge).
                            A large value forces the fallback (for tests of that path). */
    double  ms_relax;    /* MSGMRES with precision FP32 or BF16 (and the FP64 copy of T): 0 = every product of
                            the shared basis in `precision`; otherwise the products start with FP64 T and
                            switch to `precision` once every unconverged frequency's residual estimate is
                            <= the switch level times ||b_k|| (an inexact Krylov process tolerates larger
                            product errors as the residual falls). ms_relax > 0 is the level itself; < 0
                            chooses it from the measured relative error delta of one product in `precision`:
                            0.5 tol / (100 delta), clipped to [tol, 1]. Every result still ends with the FP64
                            residual check and, where needed, batched GMRES in `precision`. */
    int32_t recycle;     /* GMRES only, 0 = off; k in [1, 8]: subspace recycling across neighbouring frequencies
                            (a project extension next to the shift structure the paper's conclusions point
                            to; the paper starts every solve from q0 = 0). Per direction, every second
                            frequency (sorted) and the highest are solved from zero; each other one is
                            solved by GMRES augmented with a recycle space (GCRO) spanned by the solutions
                            of its k nearest solved frequencies: every cycle starts from the residual
                            projected off C = A U and every Krylov vector is kept orthogonal to C. Needs
                            at least three frequencies (else plain GMRES); not with block_jacobi; replaces
                            warm_start. */
} wfq_solve_opts;

typedef struct {
    int32_t status;      /* WFQ_OK, WFQ_ENOCONV, WFQ_EBREAKDOWN, WFQ_ENUMERIC for this system */
    int32_t iters;       /* inner iterations (one T product each) */
    int32_t cycles;      /* FP64 refinement cycles (GMRES restarts / QMR checks) */
    int32_t precision;   /* precision of the last cycle (after any escalation) */
    double  relres;      /* FP64 true relative residual ||b - (L T + z I) q|| / ||b|| */
    double  rmse;        /* ||b - (L T + z I) q|| / sqrt(N), size-independent measure of Eq. (rmse) */
    double  err_est;     /* bound on the relative error of q in the Coulomb norm |v|_T = sqrt(v^H T v):
                            |q - q*|_T / |q*|_T <= err_est, q* the exact solution. L T is self-adjoint in
                            the T inner product with real eigenvalues, so |(L T + z I)^-1|_T <= 1 / |Im z|;
                            with |r|_T <= sqrt(rho_T) |r|_2 (rho_T the largest row sum of T) and
                            eps = sqrt(rho_T) |r|_2 / (|Im z| |q|_T), err_est = eps / (1 - eps) (infinite
                            when eps >= 1). Exact up to the FP64 rounding of r. The 2-norm relative error
                            is at most sqrt(kappa_2(T)) err_est. */
    double  t_done_ms;   /* completion time of this system, measured from the start of the call */
    double  sigma;       /* absorption cross section for this field direction k, Eq. (long-cross):
                            sigma_k = (4 pi omega / c) Im(k . alpha), alpha the induced dipole per unit
                            field, omega in Hartree, c = 137.035999084: bohr^2 */
} wfq_result;

/*
 * wfq_build - set up one structure on the device: unit conversion, spatial reordering, widths,
 * the sparse L (cell-list neighbour search within the cutoff radius r_c = s r0 (1 + ln(1/eps - 1)/d))
 * and the dense T copies requested by store_mask (computed in FP64, stored with round to nearest
 * even). Returns WFQ_EDISCONNECTED (with a valid handle) when the Kbar graph has more than one
 * connected component: each component then conserves its own charge and solves remain valid.
 * On any other error *out is set to NULL.
 */
int wfq_build(const wfq_geometry* g, const wfq_params* p, wfq_handle** out);

/* wfq_destroy - release every resource of the handle (NULL is accepted). */
void wfq_destroy(wfq_handle* h);

/*
 * wfq_solve - solve all n_omega * n_dir systems of Eq. (wfq-a-matrix) for the given frequencies
 * (eV, each > 0) and unit field directions dirs[n_dir][3], to relative FP64 residual <= tol, starting
 * from q0 = 0 (the paper's protocol in Section "Numerical Results"). Systems sharing the handle's T
 * are solved together in batches: one block product T X serves every active system. The inner
 * iterations use T in o->precision; every FP64 refinement point recomputes the true residual with
 * the FP64 operator. Outputs (host memory, any may be NULL):
 *   q_re, q_im         [n_omega][n_dir][n] charges in the caller's atom order;
 *   alpha_re, alpha_im [n_omega][n_dir][3] alpha[l] for field direction k (complex);
 *   info               [n_omega][n_dir] per-system results.
 * Returns the worst per-system status (WFQ_ENOCONV etc.); outputs are filled in every case except
 * argument and device errors. The handle keeps the solve's device work space (and pinned host
 * mirrors) until a solve of another shape or wfq_destroy, so repeated solves of one shape allocate
 * nothing.
 */
int wfq_solve(wfq_handle* h, const double* omegas_eV, int32_t n_omega,
              const double* dirs, int32_t n_dir, double tol, const wfq_solve_opts* o,
              double* q_re, double* q_im, double* alpha_re, double* alpha_im, wfq_result* info);

/*
 * wfq_solve_dev - as wfq_solve, but q_re/q_im/alpha_re/alpha_im are device pointers (same layouts,
 * may be NULL) and all work is ordered on the HIP stream `stream` (a hipStream_t, NULL = the null
 * stream). The call returns after the results are written (it synchronises the stream).
 */
int wfq_solve_dev(wfq_handle* h, const double* omegas_eV, int32_t n_omega,
                  const double* dirs, int32_t n_dir, double tol, const wfq_solve_opts* o,
                  double* q_re_dev, double* q_im_dev, double* alpha_re_dev, double* alpha_im_dev,
                  wfq_result* info, void* stream);

/*
 * wfq_isotropic_sigma - Eq. (iso-cross): sigma(omega) = (1/3) sum_k sigma_k(omega) over three
 * orthonormal field directions. `dirs` [3][3] are the directions of a wfq_solve call with n_dir = 3
 * (rows orthonormal to 1e-9, else WFQ_EINVAL) and `info` its [n_omega][3] results; writes
 * sigma_iso [n_omega] (bohr^2). Host only, no device needed.
 */
int wfq_isotropic_sigma(const double* dirs, const wfq_result* info, int32_t n_omega, double* sigma_iso);

/* ------------------------------------------------------------------ single steps (for checks)
 * These expose one stage of the path each, in the caller's atom order, so that every stage can be
 * compared with an independent implementation. They are not needed to solve.
 */

/* number of atoms and of nonzeros of L (including the diagonal) */
int wfq_info(const wfq_handle* h, int64_t* n, int64_t* nnz_L, int64_t* bytes_device);

/* T_ij for `count` index pairs (caller order) from the stored copy of the given precision, widened
 * to double. Fails with WFQ_EINVAL if that copy was not built. */
int wfq_sample_T(const wfq_handle* h, int32_t precision, const int64_t* i, const int64_t* j,
                 int64_t count, double* out);

/* L as triplets (row, col, value), caller order, nnz_L entries, row-major by internal order. */
int wfq_export_L(const wfq_handle* h, int64_t* rows, int64_t* cols, double* vals);

/* Y = T X for ncol real host vectors X[ncol][n] (caller order), with T in `precision`
 * (WFQ_PREC_FP32/BF16 round X to that precision and accumulate in FP32), Y[ncol][n] in double. */
int wfq_apply_T(wfq_handle* h, int32_t precision, int32_t ncol, const double* X, double* Y);

/* As wfq_apply_T, but through block-product variant `variant` (an index into the list of
 * wfq_tx_variants for this precision) instead of the automatic choice, so that every shape the
 * autotuner may pick can be checked. Stored T only; WFQ_EINVAL for an unknown variant, one that
 * cannot take ncol columns, or a matrix-free handle. */
int wfq_apply_T_variant(wfq_handle* h, int32_t precision, int32_t variant, int32_t ncol, const double* X, double* Y);

/* Y = (L T + z_s I) X_s for S complex vectors (planar re/im, [S][n] each), T in `precision`. */
int wfq_apply_op(wfq_handle* h, int32_t precision, int32_t S, const double* z_re, const double* z_im,
                 const double* X_re, const double* X_im, double* Y_re, double* Y_im);

/*
 * wfq_apply_op_noalloc - as wfq_apply_op, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): it calls no hipMalloc, hipFree or
 * other allocating routine. Inputs and outputs are device pointers: z_re_dev, z_im_dev [nsys];
 * X_re_dev, X_im_dev, Y_re_dev, Y_im_dev [nsys][n] in the caller's atom order. Work is only
 * enqueued on `stream` (a hipStream_t; kernel launches only, no copies, memsets or host
 * synchronisation), so Y is ready when the stream reaches that point. Its intermediates live in one
 * static device array of wfq_noalloc_scratch_bytes() = 256 MiB per GPU, set up by wfq_build on that
 * device and held until the process ends: calls needing more (about 16 nsys N + 256 N (s + 4) bytes
 * for a T copy of s bytes per element, N padded to 256) fail with WFQ_ENOMEM before any work. Every
 * call on one GPU shares that array, from any handle: calls whose work overlaps on the device race
 * (order them on one stream or synchronise between them); each call rewrites everything it reads.
 */
int wfq_apply_op_noalloc(wfq_handle* h, int32_t precision, int32_t nsys, const double* z_re_dev,
                         const double* z_im_dev, const double* X_re_dev, const double* X_im_dev,
                         double* Y_re_dev, double* Y_im_dev, void* stream);
uint64_t wfq_noalloc_scratch_bytes(void);

/* b = E0 L (r . k) for n_dir directions: out[n_dir][n] */
int wfq_rhs(wfq_handle* h, const double* dirs, int32_t n_dir, double E0, double* out);

/* ------------------------------------------------------------------ block-product tuning
 * The block product T X has several kernel shapes (MFMA tiles of different sizes, a narrow
 * streaming kernel). wfq_tx_variants lists them for a precision: *count entries, names[k] (static
 * strings) and max_ncol[k] (largest column count the shape accepts); NULL arrays query *count.
 * wfq_tune times every applicable shape on random columns for each ncols[q] (reps launches each on
 * the handle's stream), writes the average times to ms[q][k] (negative: not applicable) and keeps
 * the fastest shape per ncol in the handle; later products with n columns use the shape tuned for
 * the smallest tuned ncol >= n (the largest tuned one beyond that). Untuned handles use a built-in
 * choice by column count. */
int wfq_tx_variants(int32_t precision, int32_t* count, const char** names, int32_t* max_ncol);
int wfq_tune(wfq_handle* h, int32_t precision, const int32_t* ncols, int32_t n_ncols, int32_t reps, double* ms,
             int32_t* chosen);

/* per-kernel timings gathered by solves run with opts.timing != 0 (since the last reset):
 * for kernel class c < *n_classes: names[c] (static strings), launches[c], total_ms[c],
 * flops[c] and bytes[c] (algorithmic counts summed over launches). Pass NULL arrays to query
 * *n_classes. reset != 0 clears the counters after reading. */
int wfq_kernel_stats(wfq_handle* h, int32_t* n_classes, const char** names, int64_t* launches,
                     double* total_ms, double* flops, double* bytes, int32_t reset);

/* ------------------------------------------------------------------ serving
 * A request loop for spectrum jobs of different structures arriving over time. Each job is one
 * geometry + parameters + frequency list + field directions. Jobs are admitted in arrival order
 * while their device footprint (T copies, L, Krylov bases) fits the budget and a slot is free (a job
 * is always admitted when nothing else is resident; a job whose footprint exceeds the whole budget
 * ends with WFQ_ENOMEM); admitted jobs run on their own streams and overlap on the device.
 * Submission never blocks. Every call is thread-safe; a ticket is retrieved (poll/wait returning a
 * final status) once.
 */
typedef struct {
    uint64_t device_budget;   /* bytes for all resident jobs; 0 = 90% of free memory */
    int32_t  max_jobs;        /* concurrently resident jobs (slots), 1..64; wfq_serve starts one worker
                                 thread per slot, wfq_serve_stop joins them */
    int32_t  max_queue;       /* waiting jobs before submit returns WFQ_EAGAIN, >= 1 */
    int32_t  device;          /* HIP device ordinal */
    wfq_solve_opts opts;      /* solver options applied to every job */
    double   tol;             /* relative residual target of every job */
} wfq_serve_cfg;

typedef struct {
    wfq_geometry   geom;      /* copied at submit */
    wfq_params     params;    /* copied at submit (t_mode, device and budget are taken from the server) */
    const double*  omegas_eV; /* [n_omega], copied at submit */
    int32_t        n_omega;
    const double*  dirs;      /* [n_dir][3], copied at submit */
    int32_t        n_dir;
} wfq_job;

typedef struct {
    double t_submit_ms;       /* all times from server start */
    double t_admit_ms;
    double t_done_ms;
    double latency_ms;        /* t_done - t_submit */
    int32_t status;
    int32_t n_systems;
} wfq_job_timing;

typedef struct {
    int64_t jobs_done;
    int64_t systems_done;
    double  p50_ms;           /* job latency percentiles over completed jobs */
    double  p99_ms;
    double  solves_per_s;     /* systems completed per second of server wall time */
    double  busy_frac;        /* fraction of wall time with at least one job running */
    int32_t max_resident;     /* most jobs resident at once */
} wfq_stats;

int wfq_serve(const wfq_serve_cfg* c, wfq_server** out);
int wfq_submit(wfq_server* s, const wfq_job* job, uint64_t* ticket);
/* non-blocking: WFQ_EAGAIN until the job is done; outputs as in wfq_solve (host, may be NULL) */
int wfq_poll(wfq_server* s, uint64_t ticket, double* q_re, double* q_im, double* alpha_re,
             double* alpha_im, wfq_result* info, wfq_job_timing* timing);
/* blocking variant of wfq_poll */
int wfq_wait(wfq_server* s, uint64_t ticket, double* q_re, double* q_im, double* alpha_re,
             double* alpha_im, wfq_result* info, wfq_job_timing* timing);
int wfq_serve_stats(wfq_server* s, wfq_stats* out);
/* stop accepting jobs, finish the running ones, release everything (NULL accepted) */
void wfq_serve_stop(wfq_server* s);

/* thread-local message of the last failing call on this thread ("" if none) */
const char* wfq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WFQ_H */
