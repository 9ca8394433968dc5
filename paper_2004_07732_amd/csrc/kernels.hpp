// Internal launch interface between the host orchestration and the HIP kernels.
#pragma once

#include <mutex>

#include "common.hpp"

namespace dwf {

// One process-wide lock around HIP calls that must not overlap a graph capture
// on another thread: capture itself, device and pinned-host allocation and
// release, and the autotuner's timing runs.  Recursive, so a holder may call
// into code that takes it again.
std::recursive_mutex& runtime_mutex();


// ------------------------------------------------------------ reductions
// Deterministic two-kernel reduction: every block writes its partial sums to
// `partial`; a one-block-per-column finaliser adds them in block order.
// Partial-sum blocks per column: enough waves in flight to stream a coarse
// vector (a few MB) at full bandwidth, few enough that a finaliser adds the
// partials of one quantity with a handful of loads per thread.
constexpr int kRedBlocks = 2048;
struct RedWork {
    double* partial = nullptr;     // [ncol][nq][nblk]
    int nblk = 0;                  // blocks per column
    int max_cols = 0;
    int max_q = 0;
};

// Krylov scalars of one column, resident on the device
struct CgScal {
    double zz, zz0, alpha, beta, tol2;
    int done, iters;
};

struct GcrScal;  // defined in blas.hip

// ------------------------------------------------------------ fine operators
template <typename R>
hipError_t fine_dw(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, const cpx<R>* b,
                   int Lx, int Ly, int Ls, int ncol, double m, double M5, bool dagger,
                   const int* skip, int skip_stride, hipStream_t st);
// the same operator without the autotuner's timing runs (a pinned or previously
// tuned configuration, else the heuristic one): no synchronisation, no events
template <typename R>
hipError_t fine_dw_untimed(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, int Lx, int Ly, int Ls, int ncol,
                           double m, double M5, bool dagger, hipStream_t st);
// pin the fine stencil's launch configuration (shape -1: automatic choice);
// returns false for an unknown shape or chunk
bool set_fine_config(int shape, int chunk);
// out = D_PV^dag D_DW(m) in on the fine level (the operator A of eq. NormalExp): two
// stencil launches through tmp, or one fused launch that keeps the intermediate in LDS
// (tmp then untouched), whichever the timed choice or the pin selects
template <typename R>
hipError_t fine_a(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, cpx<R>* tmp, int Lx, int Ly, int Ls, int ncol,
                  double m, double M5, const int* skip, int skip_stride, hipStream_t st);
// pin the fine A's configuration: shape -1 timed choice, 0 two launches, k >= 1 fused tile
// shape k with the given slice chunk; false for an unknown shape or chunk
bool set_fine_a_config(int shape, int chunk);
// the timed choice for a shape (false if none was made yet)
bool fine_a_chosen(int prec_bytes, int Lx, int Ly, int Ls, int ncol, int* shape, int* chunk);
template <typename R>
hipError_t wilson2d(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, int Lx, int Ly, int ncol,
                    double M, bool dagger, hipStream_t st);

// ------------------------------------------------------------ coarse operator
// Coarse links in "column" layout: per coarse site, five n x n blocks
// (d = 0 site-diagonal, 1: +x, 2: -x, 3: +y, 4: -y), each stored as
// blk[k][i] (row index i fastest).
struct CoarseGeom {
    int Lx, Ly, Ls, n;             // coarse extents and dof per site (n = 2 nvec)
};
// largest coarse fifth extent (the bulk transfer keeps the fine Ls on every level)
constexpr int kMaxCoarseLs = 32;
// LDS entries (complex, arithmetic type) per wavefront of the VALU coarse kernel:
// the five staged neighbour vectors of all slices, and the partition sums of a
// pass of 8 slices when 64 / n > 1 lanes share a row.  With one pass (Ls <= 8)
// the sums overwrite the staged vectors, which are dead by then.
__host__ __device__ constexpr int coarse_lds_per_wave(int n, int Ls) {
    return Ls <= 8 ? ((5 * n > 64) ? 5 * n : 64) * Ls : 5 * n * Ls + ((n <= 64 && 64 / n > 1) ? 8 * 64 : 0);
}
template <typename T>
hipError_t coarse_apply(const void* links, int link_prec, const cpx<T>* in, cpx<T>* out,
                        const CoarseGeom& g, int ncol, double m, double M5, bool dagger,
                        bool wilson_mode, double wilson_mass, const int* skip, int skip_stride,
                        hipStream_t st);

// Matrix-core path (BF16 or FP16 links stored in MFMA fragment order per
// site, n a multiple of 16); coarse_apply dispatches to it by itself for such levels.
bool coarse_mfma_supported(int n, int link_prec);
template <typename T>
hipError_t coarse_apply_mfma(const void* links, int link_prec, const cpx<T>* in, cpx<T>* out, const CoarseGeom& g,
                             int ncol, double m, double M5, bool dagger, const int* skip, int sks, hipStream_t st);
hipError_t convert_links_fragment16(const cpx<double>* in, void* out, int link_prec, int nsites, int n,
                                    hipStream_t st);
// launch configuration the matrix-core path uses for this shape (the tuned one
// once a call has timed it, else the heuristic): tile width and tiles per workgroup
bool coarse_mfma_config(int link_prec, int vec_prec, const CoarseGeom& g, int ncol, bool dagger, int* tw, int* tpb);
// the matrix-core stencil with input and output vectors of different precisions (the
// intermediate of the coarsest A: FP64 in, FP32 out, then FP32 in, FP64 out; the kernel's
// accumulation is FP32, so an FP32 intermediate holds exactly what an FP64 one would)
template <typename TI, typename TO>
hipError_t coarse_apply_mfma_io(const void* links, int link_prec, const cpx<TI>* in, cpx<TO>* out, const CoarseGeom& g,
                                int ncol, double m, double M5, bool dagger, const int* skip, int sks, hipStream_t st);
// complex 16-bit entries of that storage: the site term and the two forward hops
// (the backward hops are the sigma_3-adjoints of the neighbours' forward hops)
size_t links_fragment16_entries(int nsites, int n);

// ------------------------------------------------------------ BLAS-1 (T = float/double)
template <typename T> hipError_t vzero(cpx<T>* x, size_t n, hipStream_t st);
template <typename Ti, typename To> hipError_t vconvert(const cpx<Ti>* in, cpx<To>* out, size_t n, hipStream_t st);
// y += x (mixed precision allowed: x in Tx, y in Ty)
template <typename Tx, typename Ty> hipError_t vadd(const cpx<Tx>* x, cpx<Ty>* y, size_t n, hipStream_t st);
template <typename T> hipError_t vsub(const cpx<T>* a, const cpx<T>* b, cpx<T>* out, size_t n, hipStream_t st);
// y = a x + b y with real a, b (b == 0 overwrites y)
template <typename T> hipError_t vaxpby(double a, const cpx<T>* x, double b, cpx<T>* y, size_t n, hipStream_t st);

// dst = src for `words` 16-byte words (a streaming copy: the bandwidth reference)
hipError_t stream_copy(const void* src, void* dst, size_t words, hipStream_t st);

// per column: out[c] = |x_c|^2
template <typename T>
hipError_t norm2(const cpx<T>* x, size_t n, int ncol, double* out, const RedWork& rw, hipStream_t st);
// per column: out[c] = <a_c, b_c>
template <typename T>
hipError_t cdot(const cpx<T>* a, const cpx<T>* b, size_t n, int ncol, double* out2, const RedWork& rw, hipStream_t st);

// ---- CG family (homogeneous setup CG and CGNR), scalars in CgScal[ncol]
// s.zz = |v|^2 ; s.zz0 = s.zz ; s.done = (zz == 0) ; s.iters = 0
template <typename T>
hipError_t cg_init(const cpx<T>* v, size_t n, int ncol, CgScal* s, double tol, const RedWork& rw, hipStream_t st);
// s.alpha = s.zz / |w|^2  (0 when done)
template <typename T>
hipError_t cg_alpha(const cpx<T>* w, size_t n, int ncol, CgScal* s, const RedWork& rw, hipStream_t st);
// x += alpha p ; r -= alpha w    (skipped when done)
template <typename T>
hipError_t cg_update_xr(cpx<T>* x, cpx<T>* r, const cpx<T>* p, const cpx<T>* w, size_t n, int ncol,
                        const CgScal* s, hipStream_t st);
// znew = |z|^2; unless done: done = znew <= tol2 zz0, beta = znew / zz, zz = znew, iters++
template <typename T>
hipError_t cg_beta(const cpx<T>* z, size_t n, int ncol, CgScal* s, int maxit, const RedWork& rw, hipStream_t st);
// s.zz0 = ref[c] (a reference norm other than the starting residual), done re-evaluated
hipError_t cg_set_ref(CgScal* s, const double* ref, int ncol, hipStream_t st);
// p = z + beta p   (skipped when done)
template <typename T>
hipError_t cg_update_p(cpx<T>* p, const cpx<T>* z, size_t n, int ncol, const CgScal* s, hipStream_t st);

// ---- GCR with classical Gram-Schmidt and a deferred solution update
// Scalars per column (double): D[kmax][kmax] complex (D[j][i] = <w_i, w_j>),
// nn[kmax] (|w_j|^2 after orthogonalisation), wr[kmax] complex (<w_j, r_j>),
// gam[kmax] complex, rr (|r|^2), stop flag.
struct GcrDev {
    double* D;      // [ncol][kmax][kmax][2]
    double* nn;     // [ncol][kmax]
    double* wr;     // [ncol][kmax][2]
    double* gam;    // [ncol][kmax][2]
    double* rr;     // [ncol]
    int* stop;      // [ncol]  1: column takes no update (2: not finite)
    double* bb;     // [ncol]  |b|^2 of the device-driven solve
    int* it;        // [ncol]  iterations of the device-driven solve
    int* stop2;     // [ncol]  second stop buffer of the fused iteration (written while `stop` is read)
    double* tot;    // [ncol][kGcrTot]  inner products of the fused iteration
    int kmax;
};
constexpr int kGcrTot = 40;
// D[c][j][i] = <W_i, w>, i < j;  W_i = W + i*wstride
template <typename T>
hipError_t gcr_multidot(const cpx<T>* W, size_t wstride, int j, const cpx<T>* w, size_t n, int ncol,
                        const GcrDev& g, const RedWork& rw, hipStream_t st);
// w -= sum_{i<j} D[j][i]/nn[i] W_i ; nn[j] = |w|^2 ; wr[j] = <w, r>
template <typename T>
hipError_t gcr_orth(const cpx<T>* W, size_t wstride, int j, cpx<T>* w, const cpx<T>* r, size_t n,
                    int ncol, const GcrDev& g, const RedWork& rw, hipStream_t st);
// r -= (wr[j]/nn[j]) w ; rr = |r|^2 (when want_norm) ; copy of the new r to `copy` (may be null)
template <typename T>
hipError_t gcr_rupdate(const cpx<T>* w, cpx<T>* r, cpx<T>* copy, int j, size_t n, int ncol,
                       bool want_norm, const GcrDev& g, const RedWork& rw, hipStream_t st);
// device-driven GCR: bb = rr (= |b|^2), it = 0, stop = 1 when bb == 0, 2 when not finite
hipError_t gcr_dev_init(int ncol, const GcrDev& g, hipStream_t st);
// Fused GCR iteration j (device-driven solve, no preconditioner), three launches:
//   dots:   tot = [|w|^2, <w, r>, <W_i, w> (i < j)] in one pass;
//   update: every block derives c_i = <W_i, w>/nn_i, |w'|^2 = |w|^2 - sum |<W_i, w>|^2/nn_i and
//           a = <w, r>/|w'|^2 (r is orthogonal to every W_i, so <w', r> = <w, r>), then in one pass
//           w' = w - sum c_i W_i, r -= a w', copy = r; block 0 stores nn_j, wr_j, D[j][.], the new
//           |r|^2 = |r|^2 - |<w, r>|^2/|w'|^2 and the stop flag into `stop_out` (while `stop_in`
//           is only read).  A column already stopped only sets copy = 0, so that every
//           direction a later solution update reads was written in this cycle.
template <typename T>
hipError_t gcr_fused_step(const cpx<T>* W, size_t wstride, int j, cpx<T>* w, cpx<T>* r, cpx<T>* copy, size_t n,
                          int ncol, double tol2, const int* stop_in, int* stop_out, const GcrDev& g,
                          const RedWork& rw, hipStream_t st);
// Gram-form GCR step j (restart cycles of at most kGramMax steps), three launches: the
// multi-dot of w_j = W_j against W_0..W_{j-1} and r0, a finaliser that solves
// G y = b (G_il = <W_i, W_l>, b_i = <W_i, r0>, i, l <= j) once per column, and one pass
// out = r0 - sum_{i<=j} y_i W_i.  Keeps G's rows in g.D / g.nn, b in g.wr and y in g.gam; the
// new residual norm |r0|^2 - Re <b, y> (g.rr holds the cycle's |r0|^2) decides the stop flag
// in stop_out (1 at or below tol2 |b|^2, 2 if not finite); a stopped column's directions are
// zero and its coefficients stay those of the step it stopped at.
constexpr int kGramMax = 7;   // (the finaliser runs one wave per inner product: 2 j + 3 <= 16 waves)
template <typename T>
hipError_t gcr_gram_step(const cpx<T>* W, size_t wstride, int j, const cpx<T>* r0, cpx<T>* out, size_t n, int ncol,
                         double tol2, const int* stop_in, int* stop_out, const GcrDev& g, const RedWork& rw,
                         hipStream_t st);
// The last Gram-form step (j = k - 1) of a cycle whose starting residual is P_0, fused with
// the cycle's solution update: multi-dot and finaliser as in gcr_gram_step (g.rr becomes the
// next cycle's |r0|^2), then one pass x += sum_{i<k} y_i P_i, P_0 = P_0 - sum_{i<k} y_i W_i (the
// next cycle's residual and first direction); the stop flags of stop_out become g.stop.
template <typename T>
hipError_t gcr_gram_last(cpx<T>* P, const cpx<T>* W, size_t stride_v, int k, cpx<T>* x, size_t n, int ncol,
                         double tol2, const int* stop_in, int* stop_out, const GcrDev& g, const RedWork& rw,
                         hipStream_t st);
// next restart cycle on the recursive residual: P0 = r, and the stop flags of the
// cycle's last step (stop_src) become g.stop
template <typename T>
hipError_t gcr_restart(const cpx<T>* r, cpx<T>* P0, size_t n, int ncol, const int* stop_src, const GcrDev& g,
                       hipStream_t st);
// back substitution for gam over directions 0..k-1
hipError_t gcr_solve(int k, int ncol, const GcrDev& g, hipStream_t st);
// x (+)= sum_{i<k} gam[i] P_i ; `accumulate` false overwrites x
template <typename T, typename Tx>
hipError_t gcr_xupdate(const cpx<T>* P, size_t pstride, int k, cpx<Tx>* x, size_t n, int ncol,
                       bool accumulate, const GcrDev& g, hipStream_t st);
// gcr_solve followed by gcr_xupdate in one launch (each block substitutes for itself)
template <typename T, typename Tx>
hipError_t gcr_solve_xupdate(const cpx<T>* P, size_t pstride, int k, cpx<Tx>* x, size_t n, int ncol,
                             bool accumulate, const GcrDev& g, hipStream_t st);
// gcr_solve_xupdate (accumulating) and gcr_restart (P_0 = r, stop flags from stop_src)
// in one launch for k <= 8
template <typename T>
hipError_t gcr_solve_xupdate_restart(cpx<T>* P, size_t pstride, int k, cpx<T>* x, size_t n, int ncol, const cpx<T>* r,
                                     const int* stop_src, const GcrDev& g, hipStream_t st);

// ------------------------------------------------------------ transfer (Sec. 2.3)
// Prolongator V[site][c][j][k] (nc internal dof per chirality, nvec coarse vectors).
struct TransferGeom {
    int Lx, Ly, Ls;        // fine level
    int nc;                // internal dof per chirality on the fine level
    int bx, by;            // aggregate
    int Lsc, nvec;         // coarse fifth extent, coarse vectors per chirality
    int literal = 0;       // 1: both chiralities on the unpermuted first slice (test toggle)
};
template <typename T>
hipError_t restrict_wall(const cpx<T>* V, const cpx<T>* r, cpx<T>* rc, const TransferGeom& g, int ncol, hipStream_t st);
// bulk transfer: the 2-d prolongator on every slice (Lsc == Ls)
template <typename T>
hipError_t restrict_bulk(const cpx<T>* V, const cpx<T>* r, cpx<T>* rc, const TransferGeom& g, int ncol, hipStream_t st);
template <typename T>
hipError_t prolong_bulk(const cpx<T>* V, const cpx<T>* ec, cpx<T>* e, const TransferGeom& g, int ncol, hipStream_t st);
template <typename T>
hipError_t prolong_wall(const cpx<T>* V, const cpx<T>* ec, cpx<T>* e, const TransferGeom& g, int ncol, hipStream_t st);

// ------------------------------------------------------------ setup
// v[k][site][n] (n = 2 nc) -> V[site][c][j][k]
hipError_t chiral_columns(const cpx<double>* v, cpx<double>* V, int nsites, int nc, int nvec, hipStream_t st);
// block classical Gram-Schmidt, twice, per aggregate and chirality; bad[0] set on breakdown
hipError_t block_orthonormalize(cpx<double>* V, int Lx, int Ly, int nc, int nvec, int bx, int by,
                                int* bad, hipStream_t st);
// coarse kernel P^dagger D_W(0) P from the fine links (level 0)
hipError_t galerkin_fine(const cpx<double>* U, const cpx<double>* V, cpx<double>* links,
                         int Lx, int Ly, int nvec, int bx, int by, hipStream_t st);
// coarse kernel P^dagger S P from a coarse kernel S in column layout (level >= 1)
hipError_t galerkin_coarse(const cpx<double>* S, const cpx<double>* V, cpx<double>* links,
                           int Lx, int Ly, int nc, int nvec, int bx, int by, hipStream_t st);
// convert FP64 links to the storage precision
hipError_t convert_links(const cpx<double>* in, void* out, int prec, size_t n, hipStream_t st);
// stencil form (diag, hop[4]) row-major [site][n][n] -> complex128 export
hipError_t export_links(const cpx<double>* links, cpx<double>* out, int nsites, int n, hipStream_t st);

// ------------------------------------------------------------ utilities
template <typename R>
hipError_t gamma5R(const cpx<R>* in, cpx<R>* out, int V, int Ls, int ncol, hipStream_t st);
hipError_t gauge_transform(const cpx<double>* U, const cpx<double>* g, const cpx<double>* psi,
                           cpx<double>* Ug, cpx<double>* psig, int Lx, int Ly, int Ls, int ncol,
                           hipStream_t st);
hipError_t force(const cpx<double>* U, const cpx<double>* X, const cpx<double>* Y, double* F,
                 int Lx, int Ly, int Ls, int ncol, hipStream_t st);
// U = exp(i theta) for n angles
hipError_t links_from_theta(const double* theta, cpx<double>* U, long long n, hipStream_t st);
// copy up to kPublishItems blocks of 32-bit words from device memory to host-coherent
// memory (device views), then store the next sequence number to *seq (release, system
// scope).  The number is one more than the device counter *ctr, which the kernel
// advances, so that a launch captured in a graph publishes a new number on every replay.
constexpr int kPublishItems = 3;
struct PublishArgs {
    const uint32_t* src[kPublishItems];
    uint32_t* dst[kPublishItems];
    int words[kPublishItems];
    unsigned* seq;
    unsigned* ctr;
};
hipError_t publish_to_host(const PublishArgs& a, hipStream_t st);
// scalar finiteness check: flag[0] = 1 if any entry of x is not finite
template <typename T>
hipError_t check_finite(const cpx<T>* x, size_t n, int* flag, hipStream_t st);

}  // namespace dwf
