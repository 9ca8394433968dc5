// Host-side multigrid hierarchy and Krylov drivers (internal).
#pragma once

#include <rocblas/rocblas.h>

#include <algorithm>
#include <cstdint>
#include <initializer_list>
#include <map>
#include <set>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/dwfmg.h"
#include "kernels.hpp"
#include "task.hpp"

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
    int ksmooth = 0;              // post-smoothing steps
    int kscycle = 0;              // steps per smoothing cycle (the GCR restart length)
    void* P = nullptr;            // [kmax] directions
    void* W = nullptr;            // [kmax] A directions
    void* r = nullptr;
    void* x = nullptr;
    void* tmp = nullptr;
    void* tmp2 = nullptr;
    void* rhs = nullptr;
    void* Ps = nullptr;           // [kscycle+1] smoother directions
    void* Ws = nullptr;           // [kscycle]
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

// Device memory of a hierarchy: one arena, the caller's workspace or a single
// library allocation, carved once at setup.  In counting mode nothing is
// dereferenced: take() only advances the offset (the size query).
struct Arena {
    char* base = nullptr;
    size_t cap = 0, off = 0;
    bool counting = false;
    void* take(size_t bytes) {
        const size_t o = (off + 255) & ~size_t(255);
        if (o + bytes > cap || o + bytes < o) return nullptr;
        off = o + bytes;
        return counting ? reinterpret_cast<void*>(uintptr_t(256) + o) : base + o;
    }
};

// partial-sum blocks of the deflated start's projections
constexpr int kDeflBlocks = 256;

// Dimensions of the coarsest-level eigensolver: nk Ritz vectors kept at a thick
// restart, a Lanczos basis of m (+1) columns, for nev wanted pairs of n entries.
inline void deflation_dims(int nev, size_t n, int& nk, int& m) {
    nk = (int)std::min<size_t>((size_t)nev + std::max(16, nev / 4), n - 1);
    m = (int)std::min<size_t>((size_t)nk + std::max(32, nev / 2), n);
}

class Hierarchy {
public:
    Hierarchy() = default;
    ~Hierarchy();

    // Build the hierarchy in `ws` (ws_bytes, 256-byte aligned) or, with ws ==
    // nullptr, in one device allocation of workspace_bytes(); solves take at
    // most max_ncol right-hand sides at a time.
    int setup(const cpx<double>* U, int Lx, int Ly, int Ls, double m, double M5,
              const dwf_mg_params& p, const void* const* null_starts, int max_ncol, void* ws,
              size_t ws_bytes, hipStream_t st);
    // bytes of device memory a hierarchy needs (every level, setup and solve
    // buffers for max_ncol columns); 0 if the layout cannot be formed
    static size_t workspace_bytes(int Lx, int Ly, int Ls, const dwf_mg_params& p, int max_ncol);
    // solves ncol right-hand sides, in groups of at most max_ncol
    int solve(const cpx<double>* b, cpx<double>* x, int ncol, double tol, int flags, dwf_solve_stats* stats,
              hipStream_t st);
    // the same solve as a coroutine (the batched driver runs several at once)
    Task solve_task(const cpx<double>* b, cpx<double>* x, int ncol, double tol, int flags, dwf_solve_stats* stats,
                    hipStream_t st);
    int max_ncol() const { return max_ncol_; }

    // Batched driving from one host thread.  In batch mode a read-back point of
    // the solve records an event on the context's stream and suspends the solve
    // unless the event has completed; poll() resumes the suspended solve once
    // its event has completed (or failed) and says whether it did.
    void set_batch(bool on) { batch_ = on; }
    bool poll();
    int level_op(int level, int op, const cpx<double>* in, cpx<double>* out, int ncol, double mass,
                 hipStream_t st);
    int export_level(int level, cpx<double>* V, cpx<double>* kernel, hipStream_t st);
    int coarse_config(int level, int ncol, bool dagger, int* tw, int* tpb) const;
    int time_op(int level, int op, const cpx<double>* in, int ncol, int iters, double* avg_ms, hipStream_t st);
    int update_links(const cpx<double>* U, hipStream_t st);
    hipStream_t stream() const { return st_; }

    std::vector<Level> levels;
    dwf_mg_params prm{};
    double m = 0.0, M5 = 0.0;

private:
    Arena ws_{};
    void* ws_owned_ = nullptr;    // the arena, when the library allocated it
    int max_ncol_ = 0;
    std::vector<std::pair<void*, size_t>> zero_at_setup_;   // flags that start at zero
    std::vector<LevelWork> work_;
    RedWork rw_{};
    // pinned, host-coherent mirrors for scalar read-back, and the sequence word the
    // publishing kernel stores last (host pointers; the device views are looked up)
    double* h_scal_ = nullptr;
    int* h_int_ = nullptr;
    CgScal* h_cg_ = nullptr;
    unsigned* h_seq_ = nullptr;
    struct HostView { char* host = nullptr; char* dev = nullptr; size_t bytes = 0; };
    HostView views_[4];
    unsigned pub_ = 0;            // sequence number of the last publishing launch enqueued
    unsigned* d_pub_ctr_ = nullptr;   // its device counterpart, advanced by the kernel
    int* d_flag_ = nullptr;
    cpx<double>* r64_ = nullptr;
    cpx<double>* t64_ = nullptr;
    cpx<double>* y64_ = nullptr;   // PV polynomial of the FP64 right-hand side
    cpx<double>* z64_ = nullptr;
    cpx<double>* bp64_ = nullptr;  // D_PV b for DWF_PV_SOURCE
    // setup temporaries (they overlap the solve buffers, which setup does not use)
    struct SetupTmp {
        cpx<double>* v = nullptr;
        cpx<double>* r = nullptr;
        cpx<double>* p = nullptr;
        cpx<double>* t = nullptr;
        cpx<double>* q = nullptr;
        CgScal* s = nullptr;
    } stmp_{};
    // eigensolver temporaries of the deflation setup (also overlapping the solve buffers)
    struct DeflTmp {
        int nk = 0, m = 0;
        cpx<double> *Vb = nullptr, *Ub = nullptr, *HUb = nullptr, *Xb = nullptr, *Wb = nullptr;
        cpx<double> *P0 = nullptr, *P1 = nullptr, *P2 = nullptr, *Hh = nullptr, *t1 = nullptr, *t2 = nullptr;
        cpx<double> *G = nullptr, *Ysd = nullptr, *cdev = nullptr;
        double *lam = nullptr, *E = nullptr, *nrm = nullptr;
        int* info = nullptr;
    } dtmp_{};
    int plan(int Lx, int Ly, int Ls, int max_ncol);
    std::set<int> coarse_tuned_;   // column counts whose coarse launch configurations were timed
    Task solve_group(const cpx<double>* b, cpx<double>* x, int ncol, double tol, int flags, dwf_solve_stats* stats,
                     hipStream_t st);
    // read-back point: the host needs the stream's work done (scalars copied
    // to the pinned mirrors).  Outside batch mode: hipStreamSynchronize.
    bool batch_ = false;
    hipEvent_t wait_ev_ = nullptr;
    std::coroutine_handle<> wait_h_{};
    hipError_t* wait_slot_ = nullptr;
    unsigned wait_seq_ = 0;       // batch mode: the sequence number a suspended read waits for
    // Scalar read-back: a one-wavefront kernel stores the device words into the host
    // mirrors and then a new sequence number (publish_to_host); the host spins on the
    // number for up to kSpinMs (a stream synchronisation after that).  About 8 us
    // from the end of the GPU work to the next launch, against about 25 us for a
    // device-to-host copy followed by hipStreamSynchronize.
    struct HostCopy { void* host; const void* dev; size_t bytes; };
    static constexpr int kSpinMs = 20;
    hipError_t publish(hipStream_t st, std::initializer_list<HostCopy> items, unsigned* value);
    bool seq_arrived(unsigned v) const { return __atomic_load_n(h_seq_, __ATOMIC_ACQUIRE) == v; }
    hipError_t wait_published(unsigned v, hipStream_t st) const;
    struct HostRead {
        Hierarchy* h;
        hipStream_t st;
        unsigned v;
        hipError_t err;
        bool await_ready() {
            if (err != hipSuccess) return true;
            if (!h->batch_) {
                err = h->wait_published(v, st);
                return true;
            }
            if (h->seq_arrived(v)) return true;
            err = hipEventRecord(h->wait_ev_, st);   // lets poll() tell a finished stream from a slow one
            return err != hipSuccess;
        }
        void await_suspend(std::coroutine_handle<> c) {
            h->wait_h_ = c;
            h->wait_slot_ = &err;
            h->wait_seq_ = v;
        }
        hipError_t await_resume() const { return err; }
    };
    HostRead read_back(hipStream_t st, std::initializer_list<HostCopy> items) {
        unsigned v = 0;
        const hipError_t e = publish(st, items, &v);
        return HostRead{this, st, v, e};
    }
    // wait for a number whose publishing launch is already enqueued (inside a graph)
    HostRead wait_for(hipStream_t st, unsigned v) { return HostRead{this, st, v, hipSuccess}; }
    struct StreamWait {
        Hierarchy* h;
        hipStream_t st;
        hipError_t err = hipSuccess;
        bool await_ready() {
            if (!h->batch_) {
                err = hipStreamSynchronize(st);
                return true;
            }
            err = hipEventRecord(h->wait_ev_, st);
            if (err != hipSuccess) return true;
            const hipError_t q = hipEventQuery(h->wait_ev_);
            if (q == hipErrorNotReady) return false;
            err = q;
            return true;
        }
        void await_suspend(std::coroutine_handle<> c) {
            h->wait_h_ = c;
            h->wait_slot_ = &err;
        }
        hipError_t await_resume() const { return err; }
    };
    StreamWait sync(hipStream_t st) { return StreamWait{this, st}; }
    // runs a task to completion outside batch mode (it never suspends there)
    static int run(Task t) {
        t.start();
        return t.done() ? t.result() : DWF_EHIP;
    }
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
    bool promote_coarse_links();

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
    cpx<double>* def_C_ = nullptr;   // projections of the deflated start [ncol][nev]
    double* def_part_ = nullptr;     // their per-block partial sums
    double* def_ref_ = nullptr;   // |A^dag b|^2 per column, the CGNR reference

    void* dalloc(size_t bytes) { return ws_.take(bytes < 256 ? 256 : bytes); }
    int check_cols(int ncol) const { return (ncol >= 1 && ncol <= max_ncol_) ? DWF_OK : DWF_EINVAL; }
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

    // solvers (coroutines: they contain read-back points)
    template <typename T> Task kcycle(int l, const cpx<T>* r, cpx<T>* z, int ncol, hipStream_t st);
    template <typename T> int smooth(int l, const cpx<T>* r, cpx<T>* z, int ncol, hipStream_t st);
    template <typename T> Task coarse_solve(int l, const void* rhs, void* x, int ncol, hipStream_t st);
    template <typename T> Task cgnr(int l, const cpx<T>* b, cpx<T>* x, int ncol, hipStream_t st);
    template <typename T> Task fgcr(int l, const cpx<T>* b, cpx<T>* x, int ncol, const double* rel_tol,
                                    int maxit, int restart, int* iters_out, hipStream_t st);
    template <typename T> Task gcr_plain(int l, const cpx<T>* b, cpx<T>* x, int ncol, double tol, int maxit,
                                         int restart, int* iters_out, hipStream_t st);
    int null_vectors(int l, const cpx<double>* start, cpx<double>* v, hipStream_t st);
};

// ------------------------------------------------------------ Krylov baselines (krylov.hip)
int krylov_solve(const cpx<double>* U, const cpx<double>* b, cpx<double>* x, int Lx, int Ly, int Ls, double m,
                 double M5, int method, int ell, double tol, int maxit, dwf_solve_stats* stats, hipStream_t st);

}  // namespace dwf
