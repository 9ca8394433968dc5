// Host-side multigrid hierarchy and Krylov drivers (internal).
#pragma once

#include <rocblas/rocblas.h>

#include <map>
#include <tuple>
#include <vector>

#include "../../include/dwfmg.h"
#include "kernels.hpp"

namespace dwf {

struct Level {
    int Lx = 0, Ly = 0, Ls = 0;   // extents; Ls is the fifth extent on this level
    int n = 2;                    // dof per 2-d site (2 on the fine level, 2 nvec above)
    int nsites = 0;
    bool fine = true;
    int vec_prec = P_F64;         // working precision of this level's Krylov vectors
    // fine level operator
    cpx<double>* U64 = nullptr;
    cpx<float>* U32 = nullptr;
    // coarse level operator: FP64 master copy and working storage
    cpx<double>* links64 = nullptr;
    void* links = nullptr;
    int link_prec = P_F64;
    // prolongator to the next level (absent on the coarsest)
    int nvec_next = 0, bx = 0, by = 0;
    cpx<double>* V64 = nullptr;
    cpx<float>* V32 = nullptr;

    size_t vec_elems() const { return (size_t)Ls * nsites * n; }   // complex per column
    size_t field2d_elems() const { return (size_t)nsites * n; }
};

// Buffers of one level's solvers, sized for `ncol` columns.  Typed at run time
// by the level's vector precision.
struct LevelWork {
    int ncol = 0;
    int kmax = 0;                 // flexible GCR restart length (0: none)
    int ksmooth = 0;
    void* P = nullptr;            // [kmax] directions
    void* W = nullptr;            // [kmax] A directions
    void* r = nullptr;
    void* x = nullptr;
    void* tmp = nullptr;
    void* tmp2 = nullptr;
    void* rhs = nullptr;
    void* Ps = nullptr;           // [ksmooth+1] smoother directions
    void* Ws = nullptr;           // [ksmooth]
    void* rs = nullptr;
    void* zt = nullptr;           // K-cycle output scratch
    void* py = nullptr;           // fine level with the PV polynomial: p(X) w and X's intermediate
    void* pz = nullptr;
    // coarse-grid buffers of the K-cycle on this level (level l's precision)
    void* rc_local = nullptr;     // restricted residual in this level's precision
    void* ec_local = nullptr;
    // CGNR (coarsest level)
    void* cp = nullptr;
    void* cw = nullptr;
    void* cz = nullptr;
    GcrDev gcr{};                 // outer / intermediate GCR scalars
    GcrDev gsm{};                 // smoother scalars
    CgScal* cg = nullptr;
};

struct SolveCounters {
    long long fine_applies = 0;
    long long level_iters[DWF_MAX_LEVELS] = {0, 0, 0};
    long long level_calls[DWF_MAX_LEVELS] = {0, 0, 0};
};

class Hierarchy {
public:
    Hierarchy() = default;
    ~Hierarchy();

    int setup(const cpx<double>* U, int Lx, int Ly, int Ls, double m, double M5,
              const dwf_mg_params& p, const void* const* null_starts, hipStream_t st);
    int solve(const cpx<double>* b, cpx<double>* x, int ncol, double tol, dwf_solve_stats* stats,
              hipStream_t st);
    int level_op(int level, int op, const cpx<double>* in, cpx<double>* out, int ncol, double mass,
                 hipStream_t st);
    int export_level(int level, cpx<double>* V, cpx<double>* kernel, hipStream_t st);
    int time_op(int level, int op, const cpx<double>* in, int ncol, int iters, double* avg_ms, hipStream_t st);
    int update_links(const cpx<double>* U, hipStream_t st);
    hipStream_t stream() const { return st_; }

    std::vector<Level> levels;
    dwf_mg_params prm{};
    double m = 0.0, M5 = 0.0;

private:
    std::vector<void*> allocs_;
    std::vector<LevelWork> work_;
    RedWork rw_{};
    int work_cols_ = 0;
    // pinned host mirrors for scalar read-back
    double* h_scal_ = nullptr;
    int* h_int_ = nullptr;
    CgScal* h_cg_ = nullptr;
    int* d_flag_ = nullptr;
    int scal_cols_ = 0;
    cpx<double>* r64_ = nullptr;
    cpx<double>* t64_ = nullptr;
    cpx<double>* y64_ = nullptr;   // PV polynomial of the FP64 right-hand side
    cpx<double>* z64_ = nullptr;
    int r64_cols_ = 0;
    SolveCounters cnt_{};
    // solves run on a stream of the context, so that fixed launch sequences
    // (a chunk of coarsest CGNR iterations, a GCR smoother) can be captured
    // once as HIP graphs and replayed
    hipStream_t st_ = nullptr;
    hipEvent_t ev_in_ = nullptr;
    bool use_graphs_ = true;
    bool capturing_ = false;
    using GraphKey = std::tuple<int, int, int, const void*, const void*>;   // kind, level, ncol, ptrs
    std::map<GraphKey, hipGraphExec_t> graphs_;
    template <class F> int run_graph(const GraphKey& key, hipStream_t st, F&& enqueue);
    void clear_graphs();

public:
    // coarsest-level deflation (lowest eigenpairs of A^dag A on the coarsest level)
    int deflation_setup(hipStream_t st);
    int def_nev_ = 0;
    int eig_iters_ = 0;
    double eig_worst_ = 0.0;
    std::vector<double> def_lam_host_;

private:
    int deflate_guess(int l, const cpx<double>* z, cpx<double>* x, int ncol, hipStream_t st);
    void destroy_blas();
    rocblas_handle blas_ = nullptr;
    cpx<double>* def_V_ = nullptr;
    double* def_lam_ = nullptr;
    cpx<double>* def_C_ = nullptr;
    double* def_ref_ = nullptr;   // |A^dag b|^2 per column, the CGNR reference
    int def_ref_cols_ = 0;

    void* dalloc(size_t bytes);
    int ensure_work(int ncol, hipStream_t st);
    int ensure_scalars(int maxc);
    int alloc_level_work(int l, int ncol);

    // operators on level l in precision T
    template <typename T> hipError_t apply_dw(int l, const cpx<T>* in, cpx<T>* out, double mass, bool dag,
                                              int ncol, hipStream_t st, const int* skip = nullptr);
    // stencil applications of one A (or A^dag) on level l
    int a_cost(int l) const { return (l == 0 && prm.pv_poly_order > 0) ? 2 * prm.pv_poly_order + 2 : 2; }
    // y = p(X) w on the fine level, X = D_PV D_PV^dag, p from prm.pv_poly (z: scratch)
    template <typename T> hipError_t pv_poly(const cpx<T>* w, cpx<T>* y, cpx<T>* z, int ncol, hipStream_t st,
                                             const int* skip = nullptr);
    template <typename T> hipError_t apply_A(int l, const cpx<T>* in, cpx<T>* out, cpx<T>* tmp, int ncol,
                                             hipStream_t st, const int* skip = nullptr);
    template <typename T> hipError_t apply_Adag(int l, const cpx<T>* in, cpx<T>* out, cpx<T>* tmp, int ncol,
                                                hipStream_t st, const int* skip = nullptr);
    template <typename T> hipError_t apply_wilson(int l, const cpx<T>* in, cpx<T>* out, double mass,
                                                  bool dag, int ncol, hipStream_t st);
    template <typename T> hipError_t restrict_to(int l, const cpx<T>* r, void* rc_next, int ncol, hipStream_t st);
    template <typename T> hipError_t prolong_from(int l, const void* ec_next, cpx<T>* e, int ncol, hipStream_t st);

    // solvers
    template <typename T> int kcycle(int l, const cpx<T>* r, cpx<T>* z, int ncol, hipStream_t st);
    template <typename T> int smooth(int l, const cpx<T>* r, cpx<T>* z, int ncol, hipStream_t st);
    template <typename T> int coarse_solve(int l, const void* rhs, void* x, int ncol, hipStream_t st);
    template <typename T> int cgnr(int l, const cpx<T>* b, cpx<T>* x, int ncol, hipStream_t st);
    template <typename T> int fgcr(int l, const cpx<T>* b, cpx<T>* x, int ncol, const double* rel_tol,
                                   int maxit, int restart, int* iters_out, hipStream_t st);
    template <typename T> int gcr_plain(int l, const cpx<T>* b, cpx<T>* x, int ncol, double tol, int maxit,
                                        int restart, int* iters_out, hipStream_t st);
    int null_vectors(int l, const cpx<double>* start, cpx<double>* v, hipStream_t st);
};

// ------------------------------------------------------------ Krylov baselines (krylov.hip)
int krylov_solve(const cpx<double>* U, const cpx<double>* b, cpx<double>* x, int Lx, int Ly, int Ls, double m,
                 double M5, int method, int ell, double tol, int maxit, dwf_solve_stats* stats, hipStream_t st);

}  // namespace dwf
