/*
 * dwfmg — domain-wall fermion multigrid hot path for MI355X (gfx950).
 *
 * C ABI of the library.  Every field is a device pointer to C-contiguous
 * memory owned by the caller; the library never frees a caller buffer.
 * Streams are HIP streams passed as `void*` (NULL = the default stream); all
 * work is ordered on that stream.  Every entry point returns a status code
 * (DWF_OK = 0, > 0 soft, < 0 hard) and never throws across the boundary.
 *
 * Physics follows Brower, Clark, Howarth, Weinberg, "Multigrid for Chiral
 * Lattice Fermions: Domain Wall" (arXiv:2004.07732):
 *   D_W(M)  : 2-d Wilson kernel with U(1) links                  (Sec. 2)
 *   D_DW(m) : Shamir domain-wall operator                          (eq. DWoperator)
 *   D_PV    : Pauli-Villars operator D_DW(1)                       (Sec. 2.2)
 *   A       : D_PV^dagger D_DW, the approximate PV-preconditioned
 *             operator the multigrid iterates on                   (eq. NormalExp, Sec. 2.3)
 *   coarse  : Galerkin kernel P^dagger D_W P with wall-only transfer and a
 *             reduced fifth extent on coarse levels                (Sec. 2.3, eq. coarsenDW,
 *                                                                   eq. TruncProjectInterpolate)
 *
 * Conventions
 *   - Lattice Lx x Ly, periodic; site index y*Lx + x.
 *   - gamma_1 = sigma_1 (x), gamma_2 = sigma_2 (y), gamma_5 = sigma_3, so
 *     spin component 0 is chirality +, component 1 is chirality -.
 *   - Links U: complex [2][Ly][Lx], mu = 0 is the x direction.
 *   - 5-d fermion fields: complex [nrhs][Ls][Ly][Lx][2]; slice s = 0..Ls-1
 *     stands for the paper's s = 1..Ls.
 *   - Complex numbers are interleaved (re, im): complex128 = two doubles,
 *     complex64 = two floats.
 *   - M5 is the paper's signed bulk mass (domain-wall regime -2 < M5 < 0;
 *     the free-field optimum is -1).  A "domain-wall height" quoted as a
 *     positive 1.0 is passed as M5 = -1.0.
 */
#ifndef DWFMG_H
#define DWFMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define DWF_OK             0
#define DWF_NOT_CONVERGED  1   /* soft: stats filled, x holds the best iterate      */
#define DWF_EINVAL        -1   /* bad argument (sizes, null pointer, tolerance)      */
#define DWF_EHIP          -2   /* a HIP runtime call failed                          */
#define DWF_EBREAKDOWN    -3   /* Krylov breakdown (zero or non-finite norm)         */
#define DWF_ENAN          -4   /* non-finite value in the input or the iteration     */
#define DWF_ENOSETUP      -5   /* context missing or not set up                      */
#define DWF_EUNSUPPORTED  -6   /* a size or option the library does not support      */
#define DWF_ESCRATCH      -7   /* input larger than the static scratch of an
                                  allocation-free entry point                        */

/* ---------------------------------------------------------------- flags */
#define DWF_DAGGER     1       /* apply the adjoint                                  */
#define DWF_PREC_F32   2       /* fields (and U) are complex64 instead of complex128 */
#define DWF_PV_SOURCE  4       /* mg_solve: solve D_DW x = D_PV b (the propagator
                                  form of Sec. 2.2) instead of D_DW x = b          */

/* dwf_pv_apply modes */
#define DWF_PV          0      /* out = D_PV psi                                     */
#define DWF_PV_DAG      1      /* out = D_PV^dagger psi                              */
#define DWF_PVDAG_DW    2      /* out = D_PV^dagger D_DW(m) psi   (operator A)       */
#define DWF_PVDAG_DW_DAG 3     /* out = D_DW(m)^dagger D_PV psi   (A^dagger)         */
#define DWF_PVINV_DW    4      /* out = D_PV^-1 D_DW(m) psi (the exactly preconditioned
                                  operator of Sec. 2.2) by an inner CGNR solve      */

/* precision of a multigrid level's storage / arithmetic */
#define DWF_P_F64   0
#define DWF_P_F32   1
#define DWF_P_BF16  2          /* coarse links only: bfloat16 storage, FP32 arithmetic */
#define DWF_P_F16   3          /* coarse links only: binary16 storage, FP32 arithmetic */

#define DWF_MAX_LEVELS 3       /* coarse levels below the fine one                   */
#define DWF_PV_POLY_MAX 3      /* highest power of D_PV D_PV^dag in the PV polynomial */

/* transfer between levels */
#define DWF_TRANSFER_WALL 0
#define DWF_TRANSFER_BULK 1
#define DWF_TRANSFER_SLICE1 2

/* coarsest-level solver */
#define DWF_COARSEST_CGNR 0
#define DWF_COARSEST_GCR  1

/* ---------------------------------------------------------------- operators */

/* out = D_DW(m_f) psi (or D_DW(m_f)^dagger psi with DWF_DAGGER), eq. DWoperator.
 * U [2][Ly][Lx], psi and out [nrhs][Ls][Ly][Lx][2]; complex128, or complex64
 * with DWF_PREC_F32.  psi and out must not overlap.  Lx, Ly >= 1, Ls >= 1,
 * nrhs >= 1.  Asynchronous on `stream`.  Returns DWF_EINVAL on bad sizes or
 * null pointers, DWF_EHIP if the launch fails. */
int dwf_apply(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs,
              double m_f, double M5, int flags, void* stream);

/* Launch configuration of the fine D_DW stencil (every operator above and every
 * fine-level apply inside the solvers goes through it).  The results do not
 * depend on it: all configurations evaluate each site with the same expression
 * and agree bit for bit.  By default (DWF_FINE_AUTO) the library times the
 * candidates once per lattice shape, column count, precision and adjoint flag
 * and keeps the fastest.  dwf_fine_config pins one for all later calls in the
 * process: shape DWF_FINE_ROW (any lattice) or one of the tiled shapes (used
 * only where Lx and Ly divide into its tiles; elsewhere the automatic choice
 * applies), chunk = slices walked per thread, 1 <= chunk <= 4095 (capped at
 * Ls).  shape = DWF_FINE_AUTO restores the automatic choice (chunk ignored).
 * Returns DWF_EINVAL for an unknown shape or a chunk out of range. */
#define DWF_FINE_AUTO        -1
#define DWF_FINE_ROW          0   /* one thread per site, neighbours through the caches */
#define DWF_FINE_TILE_64x8    1   /* LDS tile of 64 x 8 sites per workgroup             */
#define DWF_FINE_TILE_32x16   2
#define DWF_FINE_TILE_128x4   3
int dwf_fine_config(int shape, int chunk);

/* Launch configuration of the fine-level operator A = D_PV^dagger D_DW(m) (eq.
 * NormalExp) inside the multigrid solver (mg_solve, mg_level_op MG_OP_A on level
 * 0; not the polynomial-corrected form).  DWF_FINE_A_TWO applies the two stencils
 * (each with its dwf_fine_config choice) through an intermediate field; the fused
 * shapes apply both in one launch over LDS tiles of the given size, evaluating the
 * intermediate on every tile and its one-site ring and never storing it (the
 * lattice must divide into the tiles; FP64 fields only with DWF_FINE_A_16x8, whose
 * LDS fits).  Both forms evaluate every site with the same arithmetic, to rounding
 * (FMA contraction may differ between the kernels).  By default (DWF_FINE_A_AUTO)
 * the library times the candidates once per lattice shape, column count and
 * precision and keeps the fused launch only when it is more than 3% faster.
 * dwf_fine_a_config pins a choice for later calls (chunk = output slices per
 * workgroup, 1..4095, capped at Ls; ignored for DWF_FINE_A_TWO and
 * DWF_FINE_A_AUTO); a pinned fused shape that does not fit a lattice falls back to
 * the automatic choice there.  Returns DWF_EINVAL for an unknown shape or a chunk
 * out of range.  dwf_fine_a_chosen reports the automatic choice made for a shape
 * (prec: 0 FP64, DWF_PREC_F32 FP32): DWF_OK with *shape and *chunk, or
 * DWF_EINVAL if none was made yet. */
#define DWF_FINE_A_AUTO   -1
#define DWF_FINE_A_TWO     0   /* two stencil launches through an intermediate field  */
#define DWF_FINE_A_16x16   1   /* one fused launch, LDS tiles of 16 x 16 sites        */
#define DWF_FINE_A_32x8    2
#define DWF_FINE_A_16x8    3
int dwf_fine_a_config(int shape, int chunk);
int dwf_fine_a_chosen(int prec, int Lx, int Ly, int Ls, int nrhs, int* shape, int* chunk);

/* Pauli-Villars forms (Sec. 2.2, eq. NormalExp): see the DWF_PV* modes.  The
 * product modes use a library-owned intermediate field (allocated on first use
 * and kept until dwf_release_scratch; a call on one stream waits, on the
 * device, for the previous call's use of it on another).  Same layout rules as
 * dwf_apply.
 * DWF_PVINV_DW (FP64 only; DWF_EUNSUPPORTED with DWF_PREC_F32) applies D_DW(m)
 * and then solves D_PV out = D_DW psi for each right-hand side by CGNR to a
 * relative residual of 1e-12 (D_PV is well conditioned: its free-field singular
 * values are at least 1).  It allocates the solver's work vectors for the
 * call, synchronises `stream`, and returns DWF_NOT_CONVERGED if the inner solve
 * stops at its cap of 10000 iterations. */
int dwf_pv_apply(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs,
                 double m_f, double M5, int mode, int flags, void* stream);

/* Allocation-free variant of dwf_pv_apply, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Modes DWF_PV, DWF_PV_DAG, DWF_PVDAG_DW and
 * DWF_PVDAG_DW_DAG give the same results as dwf_pv_apply, bit for bit;
 * DWF_PVINV_DW returns DWF_EUNSUPPORTED (its inner solver allocates).  The
 * intermediate field of the product modes lives in a static device array of
 * dwf_pv_apply_noalloc_max_bytes() bytes (64 MiB) per GPU, reserved when the
 * library's code object is loaded on that GPU and held until the process
 * ends; a product whose intermediate field (16 B per complex entry in FP64,
 * 8 B in FP32: 2 Lx Ly Ls nrhs entries) is larger returns DWF_ESCRATCH.  The
 * call allocates nothing, never synchronises and never times the stencil (it
 * uses a pinned or already-tuned launch configuration, else the heuristic
 * one).  Every call on one GPU shares that GPU's array: calls whose work
 * overlaps on the device (two streams, or two threads) race and give wrong
 * results; order them on one stream.  The calling thread's current device must
 * be the device of `stream`.  Same layout rules and errors as dwf_pv_apply. */
int dwf_pv_apply_noalloc(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs,
                         double m_f, double M5, int mode, int flags, void* stream);
size_t dwf_pv_apply_noalloc_max_bytes(void);

/* Polynomial correction of the PV preconditioning (the remark after eq.
 * NormalExp; App. A): out = D_PV^dag p(D_PV D_PV^dag) D_DW(m_f) psi with
 * p(X) = sum_{k=0}^{order} c[k] X^k (host array of order + 1 real coefficients,
 * 0 <= order <= DWF_PV_POLY_MAX); with DWF_DAGGER the adjoint
 * D_DW(m_f)^dag p(D_PV D_PV^dag) D_PV psi.  order = 0 with c = {1} is
 * DWF_PVDAG_DW.  2 order + 2 stencil applications (Horner's scheme); three
 * library-owned intermediate fields as for dwf_pv_apply.  Same layout rules as
 * dwf_apply; DWF_EINVAL for a bad order, null or non-finite coefficients. */
int dwf_pv_poly_apply(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs,
                      double m_f, double M5, const double* c, int order, int flags, void* stream);

/* Coefficients c[0..order] (host array) of the polynomial p of degree `order`
 * that minimises max |1 - x p(x)| over [lam_min, lam_max] (1 - x p(x) is the
 * scaled Chebyshev polynomial T_{order+1}), a weighting of the correction over
 * the whole spectrum, as App. A asks for; x p(x) then lies in (0, 2) on the
 * interval.  For D_PV D_PV^dag take lam_min = 1 (its spectrum starts there, App.
 * A) and lam_max its largest eigenvalue (25 on the free field at M5 = -1).
 * Host only.  DWF_EINVAL unless 0 <= order <= DWF_PV_POLY_MAX and
 * 0 < lam_min < lam_max. */
int dwf_pv_poly_chebyshev(int order, double lam_min, double lam_max, double* c);

/* out = D_W(M) psi (or its adjoint) on 2-d fields [nrhs][Ly][Lx][2] (Sec. 2). */
int dwf_wilson_apply(const void* U, const void* psi, void* out, int Lx, int Ly, int nrhs,
                     double M, int flags, void* stream);

/* out = Gamma_5 psi with Gamma_5 = gamma_5 R, (R psi)_s = psi_{Ls+1-s} (Sec. 2.1).
 * Bit-exact (sign flips and a permutation). complex128, or complex64 with DWF_PREC_F32. */
int dwf_gamma5R(const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, int flags, void* stream);

/* U(1) gauge transformation: Ug_mu(x) = (g(x) U_mu(x)) g(x+mu)^*, psig(x) = g(x) psi(x)
 * for every slice, spin and rhs.  g [Ly][Lx] complex128.  Either output may be
 * NULL to skip it.  Products are rounded one operation at a time (no fused
 * multiply-add) so the result is reproducible bit for bit. */
int dwf_gauge_transform(const void* U, const void* g, const void* psi, void* Ug, void* psig,
                        int Lx, int Ly, int Ls, int nrhs, void* stream);

/* Precision conversion of any complex array of n elements:
 * dwf_pack:   complex128 -> complex64 (round to nearest);
 * dwf_unpack: complex64  -> complex128 (exact). */
int dwf_pack(const void* in_c128, void* out_c64, size_t n, void* stream);
int dwf_unpack(const void* in_c64, void* out_c128, size_t n, void* stream);

/* Fermion force for S = phi^dagger (D^dagger D)^{-1} phi, D = D_DW(m):
 * with Y = D^{-dagger} phi and X = D^{-1} Y,
 *   F_mu(x) = dS/dtheta_mu(x)
 *           = 2 Re sum_{rhs,s} [ i U_mu(x) Y_s(x)^dag (1-gamma_mu)/2 X_s(x+mu)
 *                               - i U_mu(x)^* Y_s(x+mu)^dag (1+gamma_mu)/2 X_s(x) ].
 * U [2][Ly][Lx] complex128, X, Y [nrhs][Ls][Ly][Lx][2] complex128, F [2][Ly][Lx] double
 * (overwritten). */
int dwf_force(const void* U, const void* X, const void* Y, double* F, int Lx, int Ly, int Ls,
              int nrhs, void* stream);

/* Bandwidth reference for the stencil figures: copies `bytes` (a multiple of 16,
 * both pointers 16-byte aligned, not overlapping) from src to dst with the
 * library's streaming copy kernel, once to warm up and then `iters` times
 * between two HIP events on `stream`; *gb_per_s = 2 bytes iters / time (read
 * plus write).  Synchronises `stream`. */
int dwf_copy_bandwidth(const void* src, void* dst, size_t bytes, int iters, double* gb_per_s, void* stream);

/* Compact U(1) links from their angles (the differentiation form's variables):
 * U_mu(x) = exp(i theta_mu(x)); theta [2][Ly][Lx] double, U [2][Ly][Lx]
 * complex128 (device).  Asynchronous on `stream`. */
int dwf_links_from_theta(const double* theta, void* U, int Lx, int Ly, void* stream);

/* out[c] = |x_c|^2 (FP64 accumulation, deterministic order) for ncol columns
 * of n complex128 each; out is a device array of ncol doubles. */
int dwf_norm2(const void* x, size_t n, int ncol, double* out, void* stream);

/* ---------------------------------------------------------------- multigrid */
typedef struct dwf_mg dwf_mg;

/* Parameters of the K-cycle; dwf_mg_default_params fills the values of the
 * paper's parameter table (Table kcycle) for `nlevels` coarse levels. */
typedef struct {
    int    nlevels;                       /* coarse levels, 1..DWF_MAX_LEVELS           */
    int    nvec[DWF_MAX_LEVELS];          /* generated near-null vectors per level      */
    int    block[DWF_MAX_LEVELS][2];      /* aggregate size (bx, by) per level          */
    int    Ls_coarse[DWF_MAX_LEVELS];     /* fifth extent on each coarse level, 2..32   */
    int    link_prec[DWF_MAX_LEVELS];     /* DWF_P_* storage of each coarse kernel      */
    int    vec_prec[DWF_MAX_LEVELS];      /* DWF_P_F64 / DWF_P_F32 Krylov vectors       */
    int    fine_prec;                     /* DWF_P_F64 or DWF_P_F32 inner fine solve    */
    double m_setup;                       /* mass of the setup Wilson kernel            */
    int    setup_iters;                   /* CG iterations per null vector (max)        */
    double setup_tol;                     /* |B v| <= setup_tol |B v0|                  */
    int    outer_restart;                 /* fine flexible GCR restart length           */
    int    smooth_iters;                  /* post-smoothing GCR steps (all levels),
                                             0..16, or up to 64 with a restart          */
    int    smooth_restart;                /* restart length of the post-smoothing GCR,
                                             0..16 (0: no restart, all smooth_iters
                                             steps in one cycle, the paper's smoother;
                                             each cycle continues from the residual of
                                             the previous one)                          */
    int    inter_maxit;                   /* intermediate GCR max iterations            */
    double inter_tol;                     /* intermediate GCR relative tolerance        */
    int    inter_restart;
    int    coarsest_maxit;                /* coarsest CGNR max iterations               */
    double coarsest_tol;                  /* coarsest CGNR relative tolerance           */
    double inner_tol;                     /* relative tolerance of one inner solve      */
    int    max_iters;                     /* cap on fine GCR iterations per solve       */
    int    max_outer;                     /* cap on defect-correction steps             */
    int    coarsest_nev;                  /* deflate the coarsest solve (CGNR or GCR)
                                             with this many lowest eigenvectors of
                                             A^dag A: every call starts from
                                             V Lambda^-1 V^dag A^dag b (0: off; needs
                                             FP64 coarsest vectors)                     */
    int    eig_degree;                    /* degree of the Chebyshev polynomial that
                                             accelerates the Lanczos eigensolve
                                             (0: chosen from the spectral bounds)       */
    int    eig_maxit;                     /* thick-restart Lanczos cycles (max)         */
    double eig_tol;                       /* |H v - lambda v| / lambda of the kept pairs */
    int    coarsest_solver;               /* DWF_COARSEST_CGNR (Table 2) or
                                             DWF_COARSEST_GCR: restarted GCR on A itself,
                                             |r| <= coarsest_tol |b|                     */
    int    coarsest_restart;              /* GCR restart length on the coarsest (<= 16) */
    int    transfer;                      /* DWF_TRANSFER_WALL: restrict / prolong the
                                             walls only (eq. TruncProjectInterpolate, the
                                             paper's method); DWF_TRANSFER_BULK: the 2-d
                                             prolongator on every slice (Sec. 4.1's
                                             alternative; needs Ls_coarse equal to the
                                             finer level's Ls on every level);
                                             DWF_TRANSFER_SLICE1: a test toggle for the
                                             reading of the transfer's "s = 1": both
                                             chiralities on the unpermuted first slice
                                             (fine and coarse) instead of the wall pair
                                             P- psi_1 + P+ psi_Ls of the permuted basis
                                             (Sec. 2.2)                                */
    int    pv_poly_order;                 /* 0: the fine-level operator is the paper's
                                             A = D_PV^dag D_DW; K = 1..DWF_PV_POLY_MAX:
                                             A_p = D_PV^dag p(D_PV D_PV^dag) D_DW with
                                             p(X) = sum_{k<=K} pv_poly[k] X^k (the
                                             correction the paper leaves for future
                                             work, Sec. 2.3 and App. A); the outer
                                             solve, the smoother and the right-hand side
                                             D_PV^dag p(.) r all use it; coarse levels
                                             are unchanged                              */
    double pv_poly[DWF_PV_POLY_MAX + 1];  /* c_0..c_K (see dwf_pv_poly_chebyshev)     */
    double stagnation_ratio;              /* an outer defect-correction step stagnates
                                             when the worst relative residual is above
                                             this times its value after the previous
                                             step (default 0.9; 0 disables): the solve
                                             then promotes every 16-bit coarse kernel to
                                             its FP64 Galerkin links and continues, or
                                             with none left stops (DWF_NOT_CONVERGED).
                                             The last steps of a solve legitimately
                                             gain only about 2x (the inner tolerance
                                             then asks for just enough to reach the
                                             target), so values near 0.5 stop solves
                                             that would converge                       */
} dwf_mg_params;

typedef struct {
    int       status;                     /* same code as the return value              */
    int       outer_steps;                /* defect-correction steps                    */
    int       fine_iters;                 /* fine flexible-GCR iterations (max over rhs) */
    long long fine_applies;               /* fine D_DW, D_DW^dag, D_PV, D_PV^dag applications */
    long long level_iters[DWF_MAX_LEVELS];/* Krylov iterations summed over calls        */
    long long level_calls[DWF_MAX_LEVELS];/* solves on each coarse level                */
    double    true_rel_residual;          /* max over rhs of |b - D_DW x| / |b| (FP64)  */
    double    solve_ms;                   /* wall time of the solve                     */
    int       escalations;                /* stagnations answered by promoting the
                                             16-bit coarse links to FP64 (the hierarchy
                                             keeps them for later solves)               */
} dwf_solve_stats;

void dwf_mg_default_params(dwf_mg_params* p, int nlevels);

/* Device memory of a hierarchy, in bytes: the levels' operators and
 * prolongators, the setup relaxation and (with coarsest_nev > 0) eigensolver
 * temporaries, and every solve buffer for up to max_nrhs right-hand sides per
 * group (the setup temporaries share bytes with the solve buffers).  Host only,
 * no device work.  0 when the arguments would make mg_setup return an error. */
size_t mg_workspace_bytes(int Lx, int Ly, int Ls, int max_nrhs, const dwf_mg_params* params);

/* Build the hierarchy for gauge field U (complex128 [2][Ly][Lx], device).
 * null_starts[l] (device, complex128 [nvec_l][Ly_l][Lx_l][n_l]) are the
 * starting vectors of level l's setup relaxation, with n_0 = 2 and
 * n_l = 2*nvec_{l-1}; they are copied, not kept.  Per level: CG on
 * D_W(m_setup) D_W(m_setup)^dagger v = 0 (Sec. 3.1), chiral doubling, block
 * Gram-Schmidt, Galerkin kernel.
 * Memory: every device buffer of the hierarchy is carved from `workspace`
 * (caller-owned device memory of ws_bytes >= mg_workspace_bytes(Lx, Ly, Ls,
 * max_nrhs, params), 256-byte aligned), which must outlive the context; with
 * workspace == NULL the library makes that one allocation itself and frees it
 * in mg_destroy.  After mg_setup returns, no call on the context allocates
 * device memory.  (With coarsest_nev > 0 the setup's dense eigensolver steps
 * call rocBLAS / rocSOLVER, which keep their own device workspace in the
 * context's library handle until mg_destroy.)  The context also owns a HIP
 * stream, events and pinned host mirrors for scalar read-back.
 * Errors: DWF_EINVAL (sizes not divisible by the blocks, nvec larger than the
 * block dimension, Ls < 2, a coarse Ls outside 2..32, max_nrhs outside
 * 1..4096, a workspace too small or misaligned), DWF_EUNSUPPORTED (2*nvec not
 * in {4,8,12,16,24,32,48,64}), DWF_EBREAKDOWN (dependent null vectors),
 * DWF_EHIP. */
int mg_setup(dwf_mg** out, const void* U, int Lx, int Ly, int Ls, double m_f, double M5,
             const dwf_mg_params* params, const void* const* null_starts, int max_nrhs,
             void* workspace, size_t ws_bytes, void* stream);

/* Solve D_DW(m_f) x = b (or, with flags = DWF_PV_SOURCE, D_DW(m_f) x = D_PV b)
 * for nrhs right-hand sides b, x [nrhs][Ls][Ly][Lx][2] complex128 (device):
 * flexible GCR on D_PV^dagger D_DW with the K-cycle as preconditioner (Sec. 2.3
 * summary) inside an FP64 defect correction, until |b' - D_DW x| <= tol |b'|
 * for every rhs, b' being the right-hand side of the system solved (FP64 true
 * residual).  Right-hand sides are solved in groups of at most the context's
 * max_nrhs; the statistics add up over the groups (true_rel_residual is the
 * worst).  x is overwritten (zero initial guess).  Synchronises `stream` at
 * the end.  Returns DWF_NOT_CONVERGED when the caps are hit (x is the last
 * iterate), DWF_EINVAL for an unknown flag. */
int mg_solve(dwf_mg* mg, const void* b, void* x, int nrhs, double tol, int flags, dwf_solve_stats* st,
             void* stream);

/* Batched multi-lattice solve: solves ctx[i] for nrhs[i] right-hand sides
 * b[i] -> x[i] (layouts and flags as for mg_solve) for i < nctx, all at once.
 * Each context works on its own HIP stream from its own host thread, so
 * lattices of different sizes proceed concurrently on the GPU; every context
 * still converges on its own FP64 true residual.  stats may be NULL, else an
 * array of nctx.  Waits for `stream` before starting and returns when all are
 * done.  Returns the worst status (hard errors before soft ones). Contexts
 * must be distinct. */
int mg_solve_batch(int nctx, dwf_mg* const* ctx, const void* const* b, void* const* x, const int* nrhs,
                   double tol, int flags, dwf_solve_stats* stats, void* stream);

/* ---------------------------------------------------------------- Krylov baselines */
#define DWF_KRYLOV_CGNR     0
#define DWF_KRYLOV_BICGSTAB 1

/* Solve D_DW(m_f) x = b without multigrid, by one of the two methods the paper
 * compares its multigrid solver with (Sec. 3, Fig. iterationscompare):
 *   DWF_KRYLOV_CGNR      CG on D_DW^dagger D_DW x = D_DW^dagger b, stopping on
 *                        |b - D_DW x| <= tol |b| (residual kept by recursion);
 *   DWF_KRYLOV_BICGSTAB  BiCGStab(ell) (ell = 1..16; the paper uses 6) on
 *                        D_PV^dagger D_DW x = D_PV^dagger b, stopping on the
 *                        residual of that system; if |b - D_DW x| is then
 *                        above tol |b| it restarts from x with a tighter
 *                        tolerance.
 * FP64, one right-hand side: U [2][Ly][Lx], b and x [Ls][Ly][Lx][2]
 * complex128 device arrays (x overwritten; it starts from zero).  maxit caps
 * CG iterations or BiCGStab cycles.  stats (host, may be NULL): fine_iters =
 * iterations or cycles, fine_applies = applications of D_DW, D_DW^dagger and
 * D_PV^dagger (the paper's count), true_rel_residual, solve_ms.  Allocates its
 * work vectors (about 2 ell + 5 fields) for the duration of the call and
 * synchronises the stream.  DWF_NOT_CONVERGED (x = last iterate) when maxit
 * is reached; DWF_EBREAKDOWN on a vanishing inner product. */
int dwf_krylov_solve(const void* U, const void* b, void* x, int Lx, int Ly, int Ls, double m_f, double M5,
                     int method, int ell, double tol, int maxit, dwf_solve_stats* stats, void* stream);

/* Replace the fine-level gauge field of a built hierarchy (complex128
 * [2][Ly][Lx], copied).  The coarse levels are kept: they remain a valid
 * preconditioner for a nearby field (a molecular-dynamics step, a finite
 * difference), while every solve still converges on the true residual of the
 * new D_DW. */
int mg_update_links(dwf_mg* mg, const void* U, void* stream);

/* Level operators of a built hierarchy, for testing and diagnostics.  Fields
 * are complex128 in the level's layout ([ncol][Ls_l][Ly_l][Lx_l][n_l]; 2-d
 * fields have Ls_l = 1) and are converted to the level's working precision.
 * They run in the context's solve buffers: 1 <= ncol <= max_nrhs (else
 * DWF_EINVAL); synchronises `stream`. */
#define MG_OP_DW         0     /* D_DW(m)                                         */
#define MG_OP_DW_DAG     1
#define MG_OP_PV         2     /* D_PV                                            */
#define MG_OP_PV_DAG     3
#define MG_OP_A          4     /* D_PV^dag D_DW(m)                                */
#define MG_OP_WILSON     5     /* 2-d kernel D_W(M) at M = the `mass` argument    */
#define MG_OP_WILSON_DAG 6
#define MG_OP_RESTRICT   7     /* level l -> l+1 wall restriction                 */
#define MG_OP_PROLONG    8     /* level l+1 -> l wall prolongation                */
#define MG_OP_KCYCLE     9     /* one application of level l's preconditioner    */
int mg_level_op(dwf_mg* mg, int level, int op, const void* in, void* out, int ncol, double mass,
                void* stream);

/* Timing of one level operator (the kernels the solve runs, on the level's
 * working precision and storage; ncol <= max_nrhs): `in` (complex128, as for mg_level_op) is
 * converted once, then the operator runs `iters` times back to back on
 * `stream`, bracketed by HIP events; *avg_ms receives the mean time per
 * application.  Ops: MG_OP_DW, MG_OP_DW_DAG, MG_OP_PV, MG_OP_PV_DAG, MG_OP_A. */
int mg_time_op(dwf_mg* mg, int level, int op, const void* in, int ncol, int iters, double* avg_ms,
               void* stream);

/* Copy out level l's prolongator V[y][x][c][j][k] (complex128,
 * Ly_l*Lx_l*2*nc*nvec) or coarse kernel (level l+1) in stencil form
 * diag[Y][X][n][n] then hop[4][Y][X][n][n] (h = +x, -x, +y, -y), complex128. */
int mg_export(dwf_mg* mg, int level, void* prolongator, void* coarse_kernel, void* stream);

/* Deflation space of the coarsest level (Sec. 3, Table 1: the coarsest level
 * deflated with its lowest eigenvectors).  H = A^dag A of the coarsest level;
 * its lowest eigenpairs come from a thick-restart Lanczos process on a
 * Chebyshev polynomial of H, finished by a Rayleigh-Ritz step on H itself.
 * Fills the number of eigenpairs kept, the Lanczos steps taken and the worst
 * relative residual |H v - lambda v| / lambda of the kept pairs; `lambdas`
 * (host, may be NULL, nev entries) receives the eigenvalues in ascending
 * order.  DWF_ENOSETUP without a set-up hierarchy. */
int mg_deflation_info(const dwf_mg* mg, int* nev, int* iters, double* worst_residual, double* lambdas);

/* Launch configuration of level l's matrix-core coarse stencil (l >= 1, BF16 or
 * FP16 links with 2 nvec a multiple of 16) for ncol right-hand sides: the tile
 * width (2, 4 or 8 (slice, rhs) columns per matrix-core tile) and the tiles one
 * workgroup processes.  The library times the candidates at the first solve
 * with ncol columns (DWF_AUTOTUNE=0: the heuristic, the narrowest tile that holds
 * every column and all tiles in one workgroup); before that this reports the
 * heuristic.  Widths 2 and 4 add the site-local terms before the hops, width 8
 * after them, so a different width can change results by FP32 rounding (far below
 * the BF16/FP16 split's 2^-16 relative).  DWF_EUNSUPPORTED for a level
 * without the matrix-core path. */
int mg_coarse_config(const dwf_mg* mg, int level, int ncol, int dagger, int* tile_width, int* tiles_per_block);

/* Geometry of level l: fills Lx, Ly, Ls, dof per site and nvec (0 on the coarsest). */
int mg_level_info(const dwf_mg* mg, int level, int* Lx, int* Ly, int* Ls, int* n, int* nvec);

int mg_destroy(dwf_mg* mg);

/* Release the library-owned scratch field of dwf_pv_apply. */
int dwf_release_scratch(void);

const char* dwf_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* DWFMG_H */
