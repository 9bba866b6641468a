// Launch wrappers of the Krylov-side kernels (restarted GMRES with CGS2 Arnoldi, J-symmetric QMR,
// FP64 refinement residuals, observables). All vectors are FP64 complex in planar layout: for
// system s and vector slot j the real plane starts at base + s * sys_stride + j * vec_stride and the
// imaginary plane npad entries later. Systems are addressed by id; every launch takes a device list
// `sys` of the nsys system ids it works on (the active set).
#pragma once

#include "common.h"

namespace wfq {

struct Basis {
    double* base = nullptr;
    int64_t sys_stride = 0;  // doubles between systems
    int64_t vec_stride = 0;  // doubles between vector slots of one system
    int64_t npad = 0;
};

// rows handled by one wave in the chunked reductions (64 lanes x 8 rows)
constexpr int kWaveRows = 512;
inline int64_t wave_chunks(int64_t n) { return (n + kWaveRows - 1) / kWaveRows; }

// X[2k + plane][i] = cast(V(sys[k], j)[plane][i] * scale[sys[k]]) for i < npad (scale may be NULL);
// with write_back the scaled FP64 value is also stored back into V. prec = WFQ_PREC_*.
// With run != NULL, systems with run[s] == 0 get zero columns (and V is left alone).
void pack_columns(int prec, const Basis& V, const int* sys, int nsys, int j, const double* scale, bool write_back,
                  void* X, int64_t ld, hipStream_t st, const int* run = nullptr);

// V(s, jdst) = L Y[2k, 2k+1] + z_s V(s, jsrc) for the nsys systems (Y in FP32 or FP64); with
// y_by_sys the rows of Y are addressed by system id (Y[2s, 2s+1]) instead of list position k; with
// shift_src the shifted term is taken from that basis instead (shift_src(s, jsrc)).
void spmm_shift(const Structure& S, bool y_is_f64, const void* Y, int64_t ld, const int* sys, int nsys,
                const double2* z, const Basis& V, int jsrc, int jdst, hipStream_t st, bool y_by_sys = false,
                const Basis* shift_src = nullptr);

// As spmm_shift (list positions, no y_by_sys), first interleaving the two planes of each system's
// product into Yp (nsys x ld pairs, same element type as Y) so that the sparse product gathers both
// with one load; falls back to spmm_shift where the neighbour lists are too long for row blocks.
void spmm_shift_pairs(const Structure& S, bool y_is_f64, const void* Y, int64_t ld, void* Yp, const int* sys,
                      int nsys, const double2* z, const Basis& V, int jsrc, int jdst, hipStream_t st,
                      const Basis* shift_src = nullptr);

// V(s, jdst) = L Y_s + z_s V(s, jsrc) for the nsys listed systems, with Y already interleaved and
// addressed by system id: Yp[s][i] = (re, im) pairs, ld pairs per system (FP64).
void spmm_shift_interleaved(const Structure& S, const double* Yp, int64_t ld, const int* sys, int nsys,
                            const double2* z, const Basis& V, int jsrc, int jdst, hipStream_t st);

// h[s][i] = sum_wc partial[s][i][wc] for i <= j (skipping systems with active[s] == 0)
void reduce_dots(int64_t n, const int* sys, int nsys, int j, const double2* partial, int mdim, double2* h,
                 hipStream_t st, const int* active = nullptr);
// ---- Arnoldi with one reduction per step (dcgs.hip): classical Gram-Schmidt with delayed
// reorthogonalisation. Step k (0 .. m) of a cycle: slot k holds u (one projection pass, unit norm;
// at k = m the unnormalised w'), slot k + 1 holds z = (L T + z I) u for k < m.
struct DcgsArgs {
    const double2* dots;   // [S][2 mdim] reduced fused dots: a = Q^H u (0..k-1), alpha (k), b = Q^H z, beta
    double2* hp;           // [S][mdim] first-pass coefficients of the newest column
    double2* H;            // [S][mdim][mdim] Hessenberg matrix before rotations, column-major
    double2* R;            // [S][mdim][mdim] rotated columns (R[s][c][i] = R_ic)
    double* cs;            // [S][mdim]
    double2* sn;           // [S][mdim]
    double2* g;            // [S][mdim + 1]
    double* est;           // [S] |g_{c+1}| after column c
    const double* tol_abs; // [S]
    int* flags;            // [S] bit0 converged, bit1 happy breakdown, bit2 NaN
    int* ksteps;           // [S] completed columns in this cycle
    int* run;              // [S] 1 while stepping; cleared with a flag
    double* nu;            // [S] |w'| of the previous step
    double* inv_h;         // [S] 1 / nu (the next product is taken of w' / nu)
    double2* gamma;        // [S]
    double* inv_rho;       // [S]
    double* norm2;         // [S][nwc] chunk partials of |w'|^2
};
// partial[s][t][wc]: the fused dots of step k over 512-row chunks (2 k + 2 entries; k + 1 without z)
void dcgs_dots(const Basis& V, int64_t n, const int* sys, int nsys, int k, bool with_z, double2* partial, int mdim,
               const int* run, hipStream_t st);
// column k - 1 of H completed and rotated (k >= 1), the step's update coefficients (with_z)
void dcgs_coeff(const int* sys, int nsys, int k, bool with_z, int mdim, const DcgsArgs& a, hipStream_t st);
// q_k into slot k, w' into slot k + 1, then nu and inv_h
void dcgs_update(const Basis& V, int64_t n, const int* sys, int nsys, int k, int mdim, const DcgsArgs& a,
                 hipStream_t st);

// y = R^-1 g over the first k[s] steps
void tri_solve(const int* sys, int nsys, const int* ksteps, int mdim, const double2* R, const double2* g,
               double2* y, hipStream_t st);
// x(s) += sum_{i < k[s]} y[s][i] V(s, i)
void x_update(const Basis& V, const Basis& x, int64_t n, const int* sys, int nsys, const int* ksteps,
              const double2* y, int mdim, hipStream_t st);

// r(s) = b[dir[s]] - (L Y[2k,2k+1] + z_s x(s)) written to V(s, 0); norm2[s][blk] partial |r|^2;
// with Y = T x, qtq[s][blk] (if not NULL) the partial sums of x^H T x
void residual(const Structure& S, const double* Y, int64_t ld, const int* sys, int nsys, const double2* z,
              const Basis& x, const double* b, const int* dir, const Basis& V, double* norm2, int nblk,
              double* qtq, hipStream_t st);
inline int resid_blocks(int64_t n) { return (int)((n + 255) / 256); }
// out[s] = sqrt(sum_b norm2[s][b]) for b < nb
void sumsq(const int* sys, int nsys, const double* norm2, int nb, double* out, hipStream_t st);

// V(s, 0) = b[dir[s]] (x0 = 0), norm2[s][blk] partial |b|^2
void copy_rhs(const Structure& S, const int* sys, int nsys, const double* b, const int* dir, const Basis& V,
              double* norm2, int nblk, hipStream_t st);

// Warm start across neighbouring frequencies: x(sys[k]) = x(a) + t[k] (x(b) - x(a)) with a = src_a[k],
// b = src_b[k] (linear interpolation in the shift z between two solved systems of one direction).
void interp_start(const int* sys, int nsys, const int* src_a, const int* src_b, const double2* t, const Basis& x,
                  int64_t n, hipStream_t st);

// alpha[s][l] = sum_i r_{i,l} x(s)_i / E0  (complex, l = x, y, z)
void observables(const Structure& S, const int* sys, int nsys, const Basis& x, double E0, double2* alpha,
                 hipStream_t st);
// q_out[s][perm[i]] = x(s)_i (caller atom order); q_re / q_im may be NULL
void scatter_q(const Structure& S, const int32_t* perm, const int* sys, int nsys, const Basis& x, double* q_re,
               double* q_im, hipStream_t st);

// ---- J-symmetric QMR from BCG (qmr.hip). Slots of the per-system basis Q:
// 0 r, 1 p, 2 T p, 3 q = M p, 4 x (BCG), 5 xq (QMR iterate), 6 s (QMR residual).
constexpr int kQmrSlots = 7;
// partial[s][blk] of rho = r^T (T r), T r read from the packed block Y (rows 2k, 2k+1)
void qmr_rho(bool y_is_f64, const void* Y, int64_t ld, const int* sys, int nsys, const Basis& Q, int64_t n,
             double2* partial, int nblk, hipStream_t st);
// beta = rho_new / rho_old (0 where first[s]); p = r + beta p; T p = T r + beta T p
// (T p is also written to tpb as (re, im) pairs, ld pairs per system id (FP64), the gather source of qmr_q)
void qmr_dirs(bool y_is_f64, const void* Y, int64_t ld, const int* sys, int nsys, const Basis& Q, int64_t n,
              const double2* rho_new, const double2* rho_old, const int* first, double* tpb, hipStream_t st);
// q = L (T p) + z p with partials of sigma = (T p)^T q and of ||T p||^2, ||q||^2
void qmr_q(const Structure& S, const int* sys, int nsys, const Basis& Q, const double2* z, const double* tpb,
           double2* part_sig, double2* part_nrm, int nblk, hipStream_t st);
// sigma[s] and breakdown flags (bit 3: Lanczos breakdown when |sigma| <= thr ||T p|| ||q||, bit 2: NaN)
void qmr_sigma(const int* sys, int nsys, const double2* part_sig, const double2* part_nrm, int nblk,
               const double2* rho, double2* sigma, int* flags, double thr, hipStream_t st);
// alpha = rho / sigma; x += alpha p; r -= alpha q; partials of ||r||^2
void qmr_xr(const int* sys, int nsys, const Basis& Q, int64_t n, const double2* rho, const double2* sigma,
            double* norm2, int nblk, hipStream_t st);
// tau^2 and eta of the smoothing from ||r||^2; clears first[s]
void qmr_weights(const int* sys, int nsys, const double* rn_part, int nblk, double* tau2, double* eta, int* first,
                 hipStream_t st);
// xq += eta (x - xq); s += eta (r - s); partials of ||s||^2
void qmr_smooth(const int* sys, int nsys, const Basis& Q, int64_t n, const double* eta, double* norm2, int nblk,
                hipStream_t st);
// restart from the QMR iterate: x = xq, p = T p = 0, s = r (r must hold the residual of xq)
void qmr_restart(const int* sys, int nsys, const Basis& Q, hipStream_t st);
// out[s] = sum_b partial[s][b]
void reduce_complex(const int* sys, int nsys, const double2* partial, int nb, double2* out, hipStream_t st);

// ---- multi-shift GMRES (mshift.hip): one real Arnoldi basis per field direction, shared by the
// frequencies of that direction. Real basis of direction d, slot j at V + (d * mdim1 + j) * npad;
// `dirs` lists the ndir directions a launch works on; partial / h arrays hold pslots entries per
// direction; Hessenberg column j of direction d at H + (d * m + j) * (m + 1).
constexpr int kMsGroup = 8;   // systems per group in ms_xupdate
// X[c] = cast(V(d_c, j) * scale[d_c]) and V(d_c, j) *= scale[d_c]
void ms_pack(int prec, double* V, int64_t npad, int mdim1, int j, const int* dirs, int ndir, const double* scale,
             void* X, int64_t ld, hipStream_t st);
// V(d_c, jdst) = L Y[c]; with TV != NULL also TV(d_c, jdst - 1) = Y[c] (rows >= n: 0), the product
// T v_j kept beside the basis (same layout as V)
// With Yi (FP64 products of at most 4 columns) the neighbours' values are gathered from the
// interleaved copy of Y (rows of 4 doubles) that the narrow product can write beside it.
void ms_spmm(const Structure& S, bool y_is_f64, const void* Y, int64_t ld, const int* dirs, int ndir, double* V,
             int mdim1, int jdst, double* TV, hipStream_t st, const double* Yi = nullptr);
// partial[d][i][wc] = chunk sums of V(d, i) . V(d, jw), i < nvec; self_norm: slot nvec = ||V(d, jw)||^2
void ms_dot(const double* V, int64_t n, int64_t npad, int mdim1, int nvec, int jw, const int* dirs, int ndir,
            double* partial, int pslots, bool self_norm, hipStream_t st);
// h[d][i] = sum over chunks of partial[d][i], i < count
void ms_reduce(const int* dirs, int ndir, const double* partial, int pslots, int64_t n, int count, double* h,
               hipStream_t st);
// V(d, jw) -= sum_{i < nvec} h[d][i] V(d, i); norm (may be NULL): sums of V(d, jw)^2 over 64-row
// blocks, [d][npad / 64]
void ms_update(double* V, int64_t n, int64_t npad, int mdim1, int nvec, int jw, const int* dirs, int ndir,
               const double* h, int pslots, double* norm, hipStream_t st);
// One-reduction Arnoldi step k (DCGS2) on the real bases: fused dots of slot k (u) and, with z, slot
// k + 1 against slots 0..k into partial[d][e][wc] (ps >= 2 k + 2 entries per direction; reduce with
// ms_reduce over 2 k + 2, or k + 1 without z)
void ms_dcgs_dot(const double* V, int64_t n, int64_t npad, int mdim1, int k, bool with_z, const int* dirs, int ndir,
                 double* partial, int ps, hipStream_t st);
// from the dots: column k-1 of H, column k of S (Sm may be NULL), and with z gamma, 1 / rho and the
// next first-pass coefficients hp ([d][m + 1]); nu = |p| of the previous step
void ms_dcgs_coeff(const int* dirs, int ndir, int k, bool with_z, int m, const double* dots, int ps, double* hp,
                   double* H, double* Sm, const double* nu, const double* inv_h, double* gam, double* inv_rho,
                   hipStream_t st);
// q_k into slot k, p' into slot k + 1, nu = |p'| and inv_h = 1 / nu (norm: [d][npad / 64] block sums)
void ms_dcgs_update(double* V, int64_t n, int64_t npad, int mdim1, int k, const int* dirs, int ndir,
                    const double* dots, int ps, const double* gam, const double* inv_rho, double* norm,
                    double* nu, double* inv_h, hipStream_t st);
// y[s] <- S^-1 y[s] over k[s] entries (S of direction sdir[s], columns in the layout of H)
void ms_sinv(const int* sys, int nsys, const int* ksteps, int m, const double* Sm, const int* sdir, double2* y,
             hipStream_t st);
// Givens step j of each listed system on Hbar + z Ibar of its direction (flags: bit0 converged, bit1 breakdown, bit2 NaN);
// systems with run[s] == 0 are skipped, ksteps[s] = j + 1 is recorded and run[s] cleared when a flag
// is raised. cs, sn, g and the packed R are system-minor: entry e of system s at e * S + s.
void ms_givens(const int* sys, int nsys, int j, int m, const int* sdir, const double2* z, const double* H, double* cs,
               double2* sn, double2* g, double2* R, int64_t S, double* est, const double* tol_abs, int* flags,
               int* run, int* ksteps, hipStream_t st);
// y = R^-1 g over k[s] columns (system-minor R and g as above)
void ms_solve(const int* sys, int nsys, const int* ksteps, int m, const double2* R, int64_t S, const double2* g,
              double2* y, hipStream_t st);
// x(s) = V(d, 0..k[s]-1) y[s] for groups of kMsGroup systems (grp_sys entries -1 = none)
void ms_xupdate(const double* V, int64_t n, int64_t npad, int mdim1, const int* grp_sys, const int* grp_dir, int ngrp,
                const int* ksteps, const double2* y, int m, const Basis& X, hipStream_t st);
// The same combination of the kept products, T x(s) = TV(d, 0..k[s]-1) y[s], packed as the block
// products pack their output: real part in column 2 pos[s] of Y, imaginary part in column
// 2 pos[s] + 1 (leading dimension ld >= npad); systems with pos[s] < 0 are skipped.
void ms_txupdate(const double* TV, int64_t n, int64_t npad, int mdim1, const int* grp_sys, const int* grp_dir,
                 int ngrp, const int* ksteps, const double2* y, int m, const int* pos, double* Y, int64_t ld,
                 hipStream_t st);

// ---- block-Jacobi right preconditioning (64-atom diagonal blocks of L T + z I)
//
// bj_setup: C_b = (L T)_bb into C ([npad/64][64][64], FP64; needs the stored FP64 T), then
// P_sb = (C_b + z_s I)^-1 for the nsys listed systems into P ([B][npad/64][64 x 64] complex FP32,
// column-major; inverted in FP64).
void bj_setup(const Structure& S, const int* sys, int nsys, const double2* z, double* C, float2* P,
              hipStream_t st);
// v = V(s, j) * scale[s] (written back), u = P_s v into U(s) and into X[2k + plane] in precision prec
// (zero columns where run[s] == 0; scale and run may be NULL), for the nsys listed systems.
void bj_pack(int prec, const Basis& V, int j, const int* sys, int nsys, const double* scale, const float2* P,
             int64_t npad, const Basis& U, void* X, int64_t ld, const int* run, hipStream_t st);
// X(s) += P_s U(s) for the nsys listed systems
void bj_add(const int* sys, int nsys, const float2* P, int64_t npad, const Basis& U, const Basis& X, hipStream_t st);

// ---- subspace recycling across frequencies (recycle.hip): GMRES augmented with a fixed recycle
// space per system, C = A U' orthonormal (k[s] <= kmax vectors in the layout of Basis)
struct RecycleSpace {
    Basis C, U;                // C_i and U'_i of every system
    int kmax = 0;
    int* kk = nullptr;         // [B] vectors of each system's space (0: none)
    double2* part = nullptr;   // [B][kmax][chunks] partial dots
    double2* coef = nullptr;   // [B][kmax] coefficients of the last projection (C^H v)
    double2* Bm = nullptr;     // [B][kmax][mdim] B = C^H A Q of the current cycle
};
// V(s, j) -= C C^H V(s, j) for the listed systems (coef keeps C^H V(s, j)); with X, X(s) += U' C^H V(s, j);
// with norm2, the 256-row block partials of |V(s, j)|^2 afterwards (nblk blocks)
void rc_project(const RecycleSpace& R, const Basis& V, int j, const Basis* X, const int* sys, int nsys,
                const int* run, int64_t n, double* norm2, int nblk, hipStream_t st);
// column k of B from the projection coefficients of step k's product and the step's DCGS dots / 1 / rho
void rc_bcol(const RecycleSpace& R, const int* sys, int nsys, const int* run, int k, int mdim, const double2* dots,
             const double* inv_rho, hipStream_t st);
// X(s) -= U' (B y) over the completed columns ksteps[s]
void rc_xfix(const RecycleSpace& R, const Basis& X, const int* sys, int nsys, const int* ksteps, const double2* y,
             int mdim, int64_t n, hipStream_t st);
// C_i = b - r_a + (z_s - z_a) x_a, U_i = x_a for the neighbours a = nbr[t][i] (-1: zero vector) of the
// listed target systems; r_a = V(a, 0) (the final FP64 residual of a), x_a = X(a)
void rc_init(const RecycleSpace& R, const Basis& V, const Basis& X, const double* b, const int* dir, const double2* z,
             const int* sys, int nsys, const int* nbr, int64_t n, hipStream_t st);
// one Gram-Schmidt pass of vector i against vectors 0 .. i-1 (C and U alike), |C_i|^2 block partials
void rc_orth_step(const RecycleSpace& R, int i, const int* sys, int nsys, int64_t n, double* norm2, int nblk,
                  hipStream_t st);
// C_i *= inv[s], U_i *= inv[s]
void rc_scale(const RecycleSpace& R, int i, const int* sys, int nsys, const double* inv, hipStream_t st);

}  // namespace wfq
