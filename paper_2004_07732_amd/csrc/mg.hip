// Host orchestration of the domain-wall multigrid (Sec. 2.3 summary, Sec. 3.1,
// Table kcycle): setup of the hierarchy, the K-cycle, flexible GCR on
// D_PV^dagger D_DW, CGNR on the coarsest level, and an FP64 defect correction
// around a lower-precision inner solve.
//
// Krylov scalars never leave the device inside an iteration: reductions
// finalise their own coefficients (see blas.hip).  The host reads scalars back
// once per fine or intermediate GCR iteration (to decide convergence) and once
// per chunk of coarsest CGNR iterations; within a chunk a per-column `done`
// flag turns the remaining launches into no-ops, so the iteration count is
// exactly that of a loop that tests convergence after every iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <set>

#include <cstdio>
#include <cstdlib>

#include "mg.hpp"

namespace dwf {

// with DWF_VERBOSE set, a failing HIP call is reported with its place
static void report_hip(hipError_t e, int line) {
    static const bool on = std::getenv("DWF_VERBOSE") != nullptr;
    if (on) std::fprintf(stderr, "[dwfmg] HIP error '%s' at mg.hip:%d\n", hipGetErrorString(e), line);
}
// with DWF_VERBOSE set, the outer defect correction reports its residual per step
static bool verbose_solve() {
    static const bool on = std::getenv("DWF_VERBOSE") != nullptr;
    return on;
}
#define HIPCHK(...)                                 \
    do {                                            \
        hipError_t e_ = (__VA_ARGS__);              \
        if (e_ != hipSuccess) {                     \
            report_hip(e_, __LINE__);               \
            return DWF_EHIP;                        \
        }                                           \
    } while (0)

// the same inside coroutines
#define CO_HIPCHK(...)                              \
    do {                                            \
        hipError_t e_ = (__VA_ARGS__);              \
        if (e_ != hipSuccess) {                     \
            report_hip(e_, __LINE__);               \
            co_return DWF_EHIP;                     \
        }                                           \
    } while (0)

namespace {
template <typename T> inline cpx<T>* C(void* p) { return reinterpret_cast<cpx<T>*>(p); }
template <typename T> inline const cpx<T>* C(const void* p) { return reinterpret_cast<const cpx<T>*>(p); }
template <typename T> constexpr int prec_of() { return std::is_same<T, float>::value ? P_F32 : P_F64; }
constexpr int kCgChunk = 16;
const int kSkipStride = (int)(sizeof(CgScal) / sizeof(int));
// longest smoother restart cycle that takes the Gram-form GCR step
constexpr int kGramSteps = 6;
static_assert(kGramSteps <= kGramMax, "the Gram step kernels cover the cycle");
inline const int* cg_skip(const CgScal* s) { return s ? &s[0].done : nullptr; }
}  // namespace

Hierarchy::~Hierarchy() {
    if (st_) (void)hipStreamSynchronize(st_);
    clear_graphs();
    destroy_blas();
    std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
    if (ws_owned_) (void)hipFree(ws_owned_);
    if (h_scal_) (void)hipHostFree(h_scal_);
    if (h_int_) (void)hipHostFree(h_int_);
    if (h_cg_) (void)hipHostFree(h_cg_);
    if (h_seq_) (void)hipHostFree(h_seq_);
    if (ev_in_) (void)hipEventDestroy(ev_in_);
    if (wait_ev_) (void)hipEventDestroy(wait_ev_);
    if (st_) (void)hipStreamDestroy(st_);
}

std::recursive_mutex& runtime_mutex() {
    static std::recursive_mutex m;
    return m;
}

bool Hierarchy::poll() {
    if (!wait_h_) return false;
    hipError_t res = hipSuccess;
    if (!(wait_seq_ && seq_arrived(wait_seq_))) {
        const hipError_t q = hipEventQuery(wait_ev_);
        if (q == hipErrorNotReady) return false;
        // the stream has finished: a published number is visible by now unless it failed
        res = q;
        if (res == hipSuccess && wait_seq_ && !seq_arrived(wait_seq_)) res = hipErrorUnknown;
    }
    if (wait_slot_) *wait_slot_ = res;
    std::coroutine_handle<> h = wait_h_;
    wait_h_ = nullptr;
    wait_slot_ = nullptr;
    wait_seq_ = 0;
    h.resume();
    return true;
}

hipError_t Hierarchy::publish(hipStream_t st, std::initializer_list<HostCopy> items, unsigned* value) {
    PublishArgs a{};
    int k = 0;
    for (const HostCopy& c : items) {
        if (k == kPublishItems || c.bytes % 4 != 0 || c.bytes / 4 > (size_t)INT32_MAX) return hipErrorInvalidValue;
        char* dst = nullptr;
        for (const HostView& v : views_)
            if (v.host && (char*)c.host >= v.host && (char*)c.host + c.bytes <= v.host + v.bytes)
                dst = v.dev + ((char*)c.host - v.host);
        if (!dst) return hipErrorInvalidValue;
        a.src[k] = reinterpret_cast<const uint32_t*>(c.dev);
        a.dst[k] = reinterpret_cast<uint32_t*>(dst);
        a.words[k] = (int)(c.bytes / 4);
        ++k;
    }
    a.seq = reinterpret_cast<unsigned*>(views_[3].dev);
    a.ctr = d_pub_ctr_;
    // the kernel publishes one more than its counter; outside a capture the host's count
    // advances with it (a captured launch advances it at every replay: see the caller)
    if (!capturing_) *value = ++pub_;
    return publish_to_host(a, st);
}

hipError_t Hierarchy::wait_published(unsigned v, hipStream_t st) const {
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 1;; ++spin) {
        if (seq_arrived(v)) return hipSuccess;
        if ((spin & 1023u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(kSpinMs)) break;
    }
    // long GPU work (or a failure): block in the runtime instead of spinning
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    return seq_arrived(v) ? hipSuccess : hipErrorUnknown;
}

void Hierarchy::clear_graphs() {
    for (auto& kv : graphs_) (void)hipGraphExecDestroy(kv.second);
    graphs_.clear();
}

// Capture `enqueue` (a fixed sequence of launches on `st`) once per key as a
// HIP graph, then replay it.  The captured sequence contains kernel launches
// only (no memset or copy nodes).
template <class F>
int Hierarchy::run_graph(const GraphKey& key, hipStream_t st, F&& enqueue) {
    auto it = graphs_.find(key);
    if (it == graphs_.end()) {
        std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        capturing_ = true;
        const int e = enqueue();
        capturing_ = false;
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(st, &g);
        if (e != DWF_OK || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return e != DWF_OK ? e : DWF_EHIP;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return DWF_EHIP;
        it = graphs_.emplace(key, ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, st));
    return DWF_OK;
}

// ------------------------------------------------------------ level operators
template <typename T>
hipError_t Hierarchy::apply_dw(int l, const cpx<T>* in, cpx<T>* out, double mass, bool dag, int ncol,
                               hipStream_t st, const int* skip) {
    const Level& L = levels[l];
    const int stride = skip ? kSkipStride : 1;
    if (L.fine) {
        const cpx<T>* U;
        if constexpr (std::is_same<T, float>::value) U = L.U32; else U = L.U64;
        return fine_dw<T>(U, in, out, nullptr, L.Lx, L.Ly, L.Ls, ncol, mass, M5, dag, skip, stride, st);
    }
    CoarseGeom g{L.Lx, L.Ly, L.Ls, L.n};
    return coarse_apply<T>(L.links, L.link_prec, in, out, g, ncol, mass, M5, dag, false, 0.0, skip, stride, st);
}

// Polynomial correction of the PV preconditioning (remark after eq. NormalExp,
// App. A): y = p(X) w, X = D_PV D_PV^dag, by Horner's scheme (y = c_K w, then
// y = c_k w + X y), on the fine level
template <typename T>
hipError_t Hierarchy::pv_poly(const cpx<T>* w, cpx<T>* y, cpx<T>* z, int ncol, hipStream_t st, const int* skip) {
    const int K = prm.pv_poly_order;
    const size_t n = levels[0].vec_elems() * ncol;
    hipError_t e = vaxpby<T>(prm.pv_poly[K], w, 0.0, y, n, st);
    for (int k = K - 1; k >= 0 && e == hipSuccess; --k) {
        e = apply_dw<T>(0, y, z, 1.0, true, ncol, st, skip);
        if (e == hipSuccess) e = apply_dw<T>(0, z, y, 1.0, false, ncol, st, skip);
        if (e == hipSuccess) e = vaxpby<T>(prm.pv_poly[k], w, 1.0, y, n, st);
    }
    return e;
}

// A = D_PV^dag D_DW (on the fine level with the PV polynomial: D_PV^dag p(X) D_DW)
template <typename T>
hipError_t Hierarchy::apply_A(int l, const cpx<T>* in, cpx<T>* out, cpx<T>* tmp, int ncol, hipStream_t st,
                              const int* skip) {
    if (l == 0 && prm.pv_poly_order == 0) {
        if (!capturing_) cnt_.fine_applies += a_cost(0);
        const Level& L = levels[0];
        const cpx<T>* U;
        if constexpr (std::is_same<T, float>::value) U = L.U32; else U = L.U64;
        return fine_a<T>(U, in, out, tmp, L.Lx, L.Ly, L.Ls, ncol, m, M5, skip, skip ? kSkipStride : 1, st);
    }
    if constexpr (std::is_same<T, double>::value) {
        const Level& L = levels[l];
        if (!L.fine && L.Ls <= kMaxCoarseLs && coarse_mfma_supported(L.n, L.link_prec)) {
            // FP64 coarse vectors on the matrix cores: the stencil accumulates in FP32, so
            // its output holds FP32 values, and the intermediate D_DW in is kept in FP32
            // (half its bytes); under the same launch configurations A in is the same, bit
            // for bit, as with an FP64 intermediate
            const CoarseGeom g{L.Lx, L.Ly, L.Ls, L.n};
            const int stride = skip ? kSkipStride : 1;
            cpx<float>* t = reinterpret_cast<cpx<float>*>(tmp);
            hipError_t e = coarse_apply_mfma_io<double, float>(L.links, L.link_prec, in, t, g, ncol, m, M5, false,
                                                               skip, stride, st);
            if (e != hipSuccess) return e;
            return coarse_apply_mfma_io<float, double>(L.links, L.link_prec, t, out, g, ncol, 1.0, M5, true, skip,
                                                       stride, st);
        }
    }
    hipError_t e = apply_dw<T>(l, in, tmp, m, false, ncol, st, skip);
    if (e != hipSuccess) return e;
    if (l == 0 && !capturing_) cnt_.fine_applies += a_cost(0);
    if (l == 0 && prm.pv_poly_order > 0) {
        cpx<T>* y = C<T>(work_[0].py);
        e = pv_poly<T>(tmp, y, C<T>(work_[0].pz), ncol, st, skip);
        if (e != hipSuccess) return e;
        return apply_dw<T>(l, y, out, 1.0, true, ncol, st, skip);
    }
    return apply_dw<T>(l, tmp, out, 1.0, true, ncol, st, skip);
}

// A^dag = D_DW^dag D_PV (with the PV polynomial: D_DW^dag p(X) D_PV; p(X) is Hermitian)
template <typename T>
hipError_t Hierarchy::apply_Adag(int l, const cpx<T>* in, cpx<T>* out, cpx<T>* tmp, int ncol, hipStream_t st,
                                 const int* skip) {
    hipError_t e = apply_dw<T>(l, in, tmp, 1.0, false, ncol, st, skip);
    if (e != hipSuccess) return e;
    if (l == 0 && !capturing_) cnt_.fine_applies += a_cost(0);
    if (l == 0 && prm.pv_poly_order > 0) {
        cpx<T>* y = C<T>(work_[0].py);
        e = pv_poly<T>(tmp, y, C<T>(work_[0].pz), ncol, st, skip);
        if (e != hipSuccess) return e;
        return apply_dw<T>(l, y, out, m, true, ncol, st, skip);
    }
    return apply_dw<T>(l, tmp, out, m, true, ncol, st, skip);
}

template <typename T>
hipError_t Hierarchy::apply_wilson(int l, const cpx<T>* in, cpx<T>* out, double mass, bool dag, int ncol,
                                   hipStream_t st) {
    const Level& L = levels[l];
    if (L.fine) {
        const cpx<T>* U;
        if constexpr (std::is_same<T, float>::value) U = L.U32; else U = L.U64;
        return wilson2d<T>(U, in, out, L.Lx, L.Ly, ncol, mass, dag, st);
    }
    // the 2-d kernel is only used by the setup and by diagnostics: FP64 links
    CoarseGeom g{L.Lx, L.Ly, 1, L.n};
    return coarse_apply<T>(L.links64, P_F64, in, out, g, ncol, 0.0, M5, dag, true, mass, nullptr, 1, st);
}

template <typename T>
hipError_t Hierarchy::restrict_to(int l, const cpx<T>* r, void* rc_next, int ncol, hipStream_t st) {
    const Level& L = levels[l];
    const Level& N = levels[l + 1];
    TransferGeom g{L.Lx, L.Ly, L.Ls, L.n / 2, L.bx, L.by, N.Ls, L.nvec_next};
    g.literal = prm.transfer == DWF_TRANSFER_SLICE1 ? 1 : 0;
    const cpx<T>* V;
    if constexpr (std::is_same<T, float>::value) V = L.V32; else V = L.V64;
    const bool bulk = prm.transfer == DWF_TRANSFER_BULK;
    auto R = [&](cpx<T>* dst) { return bulk ? restrict_bulk<T>(V, r, dst, g, ncol, st) : restrict_wall<T>(V, r, dst, g, ncol, st); };
    if (N.vec_prec == prec_of<T>()) return R(C<T>(rc_next));
    cpx<T>* loc = C<T>(work_[l].rc_local);
    hipError_t e = R(loc);
    if (e != hipSuccess) return e;
    const size_t n = N.vec_elems() * ncol;
    if constexpr (std::is_same<T, float>::value) return vconvert<float, double>(loc, C<double>(rc_next), n, st);
    else return vconvert<double, float>(loc, C<float>(rc_next), n, st);
}

template <typename T>
hipError_t Hierarchy::prolong_from(int l, const void* ec_next, cpx<T>* e, int ncol, hipStream_t st) {
    const Level& L = levels[l];
    const Level& N = levels[l + 1];
    TransferGeom g{L.Lx, L.Ly, L.Ls, L.n / 2, L.bx, L.by, N.Ls, L.nvec_next};
    g.literal = prm.transfer == DWF_TRANSFER_SLICE1 ? 1 : 0;
    const cpx<T>* V;
    if constexpr (std::is_same<T, float>::value) V = L.V32; else V = L.V64;
    const bool bulk = prm.transfer == DWF_TRANSFER_BULK;
    auto P = [&](const cpx<T>* src) { return bulk ? prolong_bulk<T>(V, src, e, g, ncol, st) : prolong_wall<T>(V, src, e, g, ncol, st); };
    if (N.vec_prec == prec_of<T>()) return P(C<T>(ec_next));
    cpx<T>* loc = C<T>(work_[l].ec_local);
    const size_t n = N.vec_elems() * ncol;
    hipError_t err;
    if constexpr (std::is_same<T, float>::value) err = vconvert<double, float>(C<double>(ec_next), loc, n, st);
    else err = vconvert<float, double>(C<float>(ec_next), loc, n, st);
    if (err != hipSuccess) return err;
    return P(loc);
}

// ------------------------------------------------------------ work buffers
int Hierarchy::alloc_level_work(int l, int ncol) {
    const Level& L = levels[l];
    LevelWork& w = work_[l];
    w.ncol = ncol;
    const size_t vb = L.vec_elems() * cplx_bytes(L.vec_prec) * ncol;
    const bool coarsest = (l == (int)levels.size() - 1);
    const bool coarsest_gcr = coarsest && prm.coarsest_solver == DWF_COARSEST_GCR;
    w.kmax = (l == 0) ? prm.outer_restart : (coarsest ? (coarsest_gcr ? prm.coarsest_restart : 0) : prm.inter_restart);
    w.ksmooth = coarsest ? 0 : prm.smooth_iters;
    w.kscycle = (prm.smooth_restart > 0 && prm.smooth_restart < w.ksmooth) ? prm.smooth_restart : w.ksmooth;
    auto A = [&](size_t bytes) { return dalloc(bytes); };
    w.r = A(vb); w.x = A(vb); w.tmp = A(vb); w.tmp2 = A(vb); w.rhs = A(vb);
    if (!w.r || !w.x || !w.tmp || !w.tmp2 || !w.rhs) return DWF_EINVAL;
    if (l == 0 && prm.pv_poly_order > 0) {
        w.py = A(vb); w.pz = A(vb);
        if (!w.py || !w.pz) return DWF_EINVAL;
    }
    if (w.kmax > 0) {
        w.P = A(vb * w.kmax);
        w.W = A(vb * w.kmax);
        if (!w.P || !w.W) return DWF_EINVAL;
    }
    if (w.ksmooth > 0) {
        w.Ps = A(vb * (w.kscycle + 1));
        w.Ws = A(vb * w.kscycle);
        w.rs = A(vb);
        w.zt = A(vb);
        if (!w.Ps || !w.Ws || !w.rs || !w.zt) return DWF_EINVAL;
    }
    if (!coarsest) {
        const Level& N = levels[l + 1];
        const size_t cb = N.vec_elems() * cplx_bytes(L.vec_prec) * ncol;
        w.rc_local = A(cb);
        w.ec_local = A(cb);
        if (!w.rc_local || !w.ec_local) return DWF_EINVAL;
    } else {
        w.cp = A(vb); w.cw = A(vb); w.cz = A(vb);
        w.cg = (CgScal*)A(sizeof(CgScal) * ncol);
        if (!w.cp || !w.cw || !w.cz || !w.cg) return DWF_EINVAL;
    }
    auto mk_gcr = [&](GcrDev& g, int kmax) -> int {
        g.kmax = kmax;
        g.D = (double*)A(sizeof(double) * 2 * kmax * kmax * ncol);
        g.nn = (double*)A(sizeof(double) * kmax * ncol);
        g.wr = (double*)A(sizeof(double) * 2 * kmax * ncol);
        g.gam = (double*)A(sizeof(double) * 2 * kmax * ncol);
        g.rr = (double*)A(sizeof(double) * ncol);
        g.stop = (int*)A(sizeof(int) * ncol);
        g.bb = (double*)A(sizeof(double) * ncol);
        g.it = (int*)A(sizeof(int) * ncol);
        g.stop2 = (int*)A(sizeof(int) * ncol);
        g.tot = (double*)A(sizeof(double) * kGcrTot * ncol);
        if (!g.D || !g.nn || !g.wr || !g.gam || !g.rr || !g.stop || !g.bb || !g.it || !g.stop2 || !g.tot)
            return DWF_EINVAL;
        zero_at_setup_.emplace_back(g.stop, sizeof(int) * ncol);
        return DWF_OK;
    };
    if (w.kmax > 0 && mk_gcr(w.gcr, w.kmax) != DWF_OK) return DWF_EINVAL;
    if (w.ksmooth > 0 && mk_gcr(w.gsm, w.kscycle) != DWF_OK) return DWF_EINVAL;
    return DWF_OK;
}

// ------------------------------------------------------------ CGNR (coarsest level)
template <typename T>
Task Hierarchy::cgnr(int l, const cpx<T>* b, cpx<T>* x, int ncol, hipStream_t st) {
    const Level& L = levels[l];
    LevelWork& w = work_[l];
    const size_t n = L.vec_elems();
    const size_t nt = n * ncol;
    cpx<T>* r = C<T>(w.r);
    cpx<T>* p = C<T>(w.cp);
    cpx<T>* q = C<T>(w.cw);
    cpx<T>* z = C<T>(w.cz);
    cpx<T>* t = C<T>(w.tmp);
    CgScal* s = w.cg;
    const int* skip = cg_skip(s);
    CO_HIPCHK(vzero<T>(x, nt, st));
    CO_HIPCHK(vconvert<T, T>(b, r, nt, st));
    CO_HIPCHK(apply_Adag<T>(l, r, z, t, ncol, st));
    bool deflated = false;
    if constexpr (std::is_same<T, double>::value) {
        if (def_nev_ > 0 && l == (int)levels.size() - 1) {
            // start from e0 = V Lambda^{-1} V^dag A^dag b; keep |A^dag b| as the reference
            CO_HIPCHK(norm2<T>(z, n, ncol, def_ref_, rw_, st));
            if (int e = deflate_guess(l, z, x, ncol, st)) co_return e;
            CO_HIPCHK(apply_A<T>(l, x, q, t, ncol, st));
            CO_HIPCHK(vsub<T>(b, q, r, nt, st));
            CO_HIPCHK(apply_Adag<T>(l, r, z, t, ncol, st));
            deflated = true;
        }
    }
    CO_HIPCHK(cg_init<T>(z, n, ncol, s, prm.coarsest_tol, rw_, st));
    if (deflated) CO_HIPCHK(cg_set_ref(s, def_ref_, ncol, st));
    CO_HIPCHK(vconvert<T, T>(z, p, nt, st));
    const int maxit = prm.coarsest_maxit;
    int iters = 0;
    // one chunk of CGNR iterations; iterations past convergence or maxit are
    // no-ops on the device, so chunks always have the full length
    auto chunk = [&](int len) -> int {
        for (int c = 0; c < len; ++c) {
            HIPCHK(apply_A<T>(l, p, q, t, ncol, st, skip));
            HIPCHK(cg_alpha<T>(q, n, ncol, s, rw_, st));
            HIPCHK(cg_update_xr<T>(x, r, p, q, n, ncol, s, st));
            HIPCHK(apply_Adag<T>(l, r, z, t, ncol, st, skip));
            HIPCHK(cg_beta<T>(z, n, ncol, s, maxit, rw_, st));
            HIPCHK(cg_update_p<T>(p, z, n, ncol, s, st));
        }
        return DWF_OK;
    };
    for (int it0 = 0; it0 < maxit; it0 += kCgChunk) {
        if (use_graphs_ && st == st_) {
            if (int e = run_graph(GraphKey{0, l, ncol, b, x}, st, [&]() { return chunk(kCgChunk); })) co_return e;
        } else {
            if (int e = chunk(kCgChunk)) co_return e;
        }
        CO_HIPCHK(co_await read_back(st, {{h_cg_, s, sizeof(CgScal) * ncol}}));
        bool all = true;
        for (int c = 0; c < ncol; ++c)
            if (!h_cg_[c].done) all = false;
        if (all) break;
    }
    for (int c = 0; c < ncol; ++c) iters = std::max(iters, h_cg_[c].iters);
    if (maxit <= 0) iters = 0;
    cnt_.level_iters[l - 1] += iters;
    cnt_.level_calls[l - 1] += 1;
    for (int c = 0; c < ncol; ++c)
        if (h_cg_[c].done == 4) co_return DWF_ENAN;
    co_return DWF_OK;
}

// ------------------------------------------------------------ restarted GCR (coarsest level)
// Unpreconditioned GCR(kmax) on A with every decision on the device (the
// stop flags are reset by gcr_dev_init at the start of every solve): each
// cycle runs kmax fused iterations whose kernels turn into no-ops for
// converged columns, then updates x and restarts from the recursive residual
// (in FP64 over the few hundred iterations of a coarsest solve to a loose
// tolerance it stays within rounding of the true one; recomputing it cost two
// coarse stencils per cycle).  The stop decision is the recursive one in either
// case.  The host reads the stop flags once per cycle; a cycle is captured once
// as a HIP graph.
template <typename T>
Task Hierarchy::gcr_plain(int l, const cpx<T>* b, cpx<T>* x, int ncol, double tol, int maxit, int restart,
                         int* iters_out, hipStream_t st) {
    const Level& L = levels[l];
    LevelWork& w = work_[l];
    const size_t n = L.vec_elems();
    const size_t nt = n * ncol;
    const int kmax = std::min(restart, w.kmax);
    if (kmax < 1) co_return DWF_EINVAL;
    cpx<T>* r = C<T>(w.r);
    cpx<T>* P = C<T>(w.P);
    cpx<T>* W = C<T>(w.W);
    cpx<T>* t = C<T>(w.tmp);
    GcrDev& g = w.gcr;
    const double tol2 = tol * tol;
    CO_HIPCHK(vzero<T>(x, nt, st));
    CO_HIPCHK((vconvert<T, T>(b, r, nt, st)));
    CO_HIPCHK((vconvert<T, T>(b, P, nt, st)));   // the first search direction (later cycles: by the residual pass)
    CO_HIPCHK(norm2<T>(b, n, ncol, g.rr, rw_, st));
    CO_HIPCHK(gcr_dev_init(ncol, g, st));
    if constexpr (std::is_same<T, double>::value) {
        if (def_nev_ > 0 && l == (int)levels.size() - 1) {
            // deflated start x0 = V Lambda^{-1} V^dag A^dag b (V: lowest eigenvectors of
            // A^dag A, the right singular vectors of A): the minimiser of |b - A x| over
            // span(V); the tolerance stays relative to |b|.  W_0 is scratch here (the
            // first iteration writes it).
            cpx<T>* z = W;
            CO_HIPCHK(apply_Adag<T>(l, b, z, t, ncol, st));
            if (int e = deflate_guess(l, z, x, ncol, st)) co_return e;
            CO_HIPCHK(apply_A<T>(l, x, z, t, ncol, st));
            CO_HIPCHK(vsub<T>(b, z, r, nt, st));
            CO_HIPCHK((vconvert<T, T>(r, P, nt, st)));
            CO_HIPCHK(norm2<T>(r, n, ncol, g.rr, rw_, st));
        }
    }
    // one restart cycle: kmax fused iterations (inner products, then one pass that orthogonalises
    // the new direction and updates the residual; the stop flags alternate between two buffers so
    // that no kernel writes the flags it reads), the solution update, and the restart.  Cycles
    // of at most kGramSteps take the Gram form instead (the smoother's), with the residual in P_0.
    const bool gram = kmax <= kGramSteps;
    auto cycle = [&]() -> int {
        for (int k = 0; k < kmax; ++k) {
            cpx<T>* Pk = P + (size_t)k * nt;
            cpx<T>* Wk = W + (size_t)k * nt;
            const int* s_in = (k % 2 == 0) ? g.stop : g.stop2;
            int* s_out = (k % 2 == 0) ? g.stop2 : g.stop;
            HIPCHK(apply_A<T>(l, Pk, Wk, t, ncol, st));
            if (gram && k + 1 < kmax) {
                // the next direction: the minimal residual so far, from P_0 (the cycle's residual)
                HIPCHK(gcr_gram_step<T>(W, nt, k, P, P + (size_t)(k + 1) * nt, n, ncol, tol2, s_in, s_out, g, rw_,
                                        st));
            } else if (gram) {
                // and the solution update, P_0 = the next cycle's residual
                HIPCHK(gcr_gram_last<T>(P, W, nt, kmax, x, n, ncol, tol2, s_in, s_out, g, rw_, st));
            } else {
                // the updated residual is the next search direction
                HIPCHK(gcr_fused_step<T>(W, nt, k, Wk, r, k + 1 < kmax ? P + (size_t)(k + 1) * nt : nullptr, n,
                                         ncol, tol2, s_in, s_out, g, rw_, st));
            }
        }
        // solution update, and the next cycle continues from the recursive residual (its
        // norm and the stop flags are those of the last fused step)
        if (!gram)
            HIPCHK(gcr_solve_xupdate_restart<T>(P, nt, kmax, x, n, ncol, r, (kmax % 2 == 0) ? g.stop : g.stop2, g,
                                                st));
        // the cycle ends by publishing the stop flags to the host (part of the graph)
        unsigned v = 0;
        HIPCHK(publish(st, {{h_int_, g.stop, sizeof(int) * ncol}}, &v));
        return DWF_OK;
    };
    const int max_cycles = std::max(1, (maxit + kmax - 1) / kmax);
    for (int c = 0; c < max_cycles; ++c) {
        if (use_graphs_ && st == st_) {
            if (int e = run_graph(GraphKey{2, l, ncol, b, x}, st, cycle)) co_return e;
        } else if (int e = cycle()) {
            co_return e;
        }
        // a replayed cycle publishes without the host's count seeing the launch
        if (use_graphs_ && st == st_) ++pub_;
        CO_HIPCHK(co_await wait_for(st, pub_));
        bool all = true;
        for (int cc = 0; cc < ncol; ++cc)
            if (h_int_[cc] == 0) all = false;
        if (all) break;
    }
    CO_HIPCHK(co_await read_back(st, {{h_int_, g.stop, sizeof(int) * ncol}, {h_int_ + ncol, g.it, sizeof(int) * ncol}}));
    int it = 0, status = DWF_OK;
    for (int cc = 0; cc < ncol; ++cc) {
        it = std::max(it, h_int_[ncol + cc]);
        if (h_int_[cc] == 2) status = DWF_ENAN;
    }
    if (iters_out) *iters_out = it;
    co_return status;
}

// ------------------------------------------------------------ GCR smoother
template <typename T>
int Hierarchy::smooth(int l, const cpx<T>* r, cpx<T>* z, int ncol, hipStream_t st) {
    const Level& L = levels[l];
    LevelWork& w = work_[l];
    const size_t n = L.vec_elems();
    const size_t nt = n * ncol;
    const int ns = w.ksmooth;
    cpx<T>* Ps = C<T>(w.Ps);
    cpx<T>* Ws = C<T>(w.Ws);
    cpx<T>* rs = C<T>(w.rs);
    cpx<T>* t = C<T>(w.tmp);
    cpx<T>* Az = C<T>(w.tmp2);
    // the steps are the fused GCR iteration of the coarsest solve (inner products in
    // one pass, orthogonalisation and residual update in a second) with a stopping
    // threshold that is never met, so that all ns steps are taken.  With a restart
    // length ks < ns the steps run in cycles of ks (the orthogonalisation cost of a
    // step grows with its index in the cycle); each cycle adds its correction to z and
    // the next starts from the recursive residual.
    const int ks = w.kscycle;
    GcrDev& g = w.gsm;
    // Short cycles take the Gram form (the directions' inner products and the cycle's starting
    // residual give each step's minimal residual; no orthogonalised direction and no running
    // residual is stored: two vector passes fewer per step, and the starting residual is the
    // first direction P_0 itself); long ones keep the orthogonalising form, whose accuracy does
    // not depend on the Gram matrix's condition (the square of the directions').
    const bool gram = ks <= kGramSteps;
    auto body = [&]() -> int {
        HIPCHK(apply_A<T>(l, z, Az, t, ncol, st));
        if (gram) {
            HIPCHK(vsub<T>(r, Az, Ps, nt, st));
            HIPCHK(norm2<T>(Ps, n, ncol, g.rr, rw_, st));
        } else {
            HIPCHK(vsub<T>(r, Az, rs, nt, st));
            HIPCHK(vconvert<T, T>(rs, Ps, nt, st));
            HIPCHK(norm2<T>(rs, n, ncol, g.rr, rw_, st));
        }
        HIPCHK(gcr_dev_init(ncol, g, st));
        for (int c0 = 0; c0 < ns; c0 += ks) {
            const int kc = std::min(ks, ns - c0);
            for (int j = 0; j < kc; ++j) {
                cpx<T>* Pj = Ps + (size_t)j * nt;
                cpx<T>* Wj = Ws + (size_t)j * nt;
                const int* s_in = (j % 2 == 0) ? g.stop : g.stop2;
                int* s_out = (j % 2 == 0) ? g.stop2 : g.stop;
                HIPCHK(apply_A<T>(l, Pj, Wj, t, ncol, st));
                if (gram && j + 1 < kc) {
                    // the next direction r_{j+1} = P_0 - sum y_i W_i
                    HIPCHK(gcr_gram_step<T>(Ws, nt, j, Ps, Ps + (size_t)(j + 1) * nt, n, ncol, -1.0, s_in, s_out, g,
                                            rw_, st));
                } else if (gram) {
                    // z += this cycle's correction, P_0 = the next cycle's starting residual
                    HIPCHK(gcr_gram_last<T>(Ps, Ws, nt, kc, z, n, ncol, -1.0, s_in, s_out, g, rw_, st));
                } else {
                    HIPCHK(gcr_fused_step<T>(Ws, nt, j, Wj, rs, (j + 1 < kc) ? Ps + (size_t)(j + 1) * nt : nullptr,
                                             n, ncol, -1.0, s_in, s_out, g, rw_, st));
                }
            }
            const int* s_last = (kc % 2 == 0) ? g.stop : g.stop2;
            if (gram) continue;   // (the last Gram step did the solution update)
            if (c0 + kc < ns) {
                // z += this cycle's correction, P_0 = the residual, the last step's flags to g.stop
                HIPCHK(gcr_solve_xupdate_restart<T>(Ps, nt, kc, z, n, ncol, rs, s_last, g, st));
            } else {
                HIPCHK((gcr_solve_xupdate<T, T>(Ps, nt, kc, z, n, ncol, true, g, st)));
            }
        }
        return DWF_OK;
    };
    if (use_graphs_ && st == st_) {
        if (int e = run_graph(GraphKey{1, l, ncol, r, z}, st, body)) return e;
        if (l == 0) cnt_.fine_applies += a_cost(0) * (ns + 1);
        return DWF_OK;
    }
    return body();
}

// ------------------------------------------------------------ K-cycle
template <typename T>
Task Hierarchy::kcycle(int l, const cpx<T>* r, cpx<T>* z, int ncol, hipStream_t st) {
    LevelWork& wn = work_[l + 1];
    CO_HIPCHK(restrict_to<T>(l, r, wn.rhs, ncol, st));
    int e;
    if (levels[l + 1].vec_prec == P_F32) e = co_await coarse_solve<float>(l + 1, wn.rhs, wn.x, ncol, st);
    else e = co_await coarse_solve<double>(l + 1, wn.rhs, wn.x, ncol, st);
    if (e < 0) co_return e;
    CO_HIPCHK(prolong_from<T>(l, wn.x, z, ncol, st));
    if (work_[l].ksmooth > 0) co_return smooth<T>(l, r, z, ncol, st);
    co_return DWF_OK;
}

template <typename T>
Task Hierarchy::coarse_solve(int l, const void* rhs, void* x, int ncol, hipStream_t st) {
    int it = 0, e;
    if (l == (int)levels.size() - 1) {
        if (prm.coarsest_solver == DWF_COARSEST_CGNR) co_return co_await cgnr<T>(l, C<T>(rhs), C<T>(x), ncol, st);
        e = co_await gcr_plain<T>(l, C<T>(rhs), C<T>(x), ncol, prm.coarsest_tol, prm.coarsest_maxit,
                                  prm.coarsest_restart, &it, st);
    } else {
        std::vector<double> tol(ncol, prm.inter_tol);
        e = co_await fgcr<T>(l, C<T>(rhs), C<T>(x), ncol, tol.data(), prm.inter_maxit, prm.inter_restart, &it, st);
    }
    cnt_.level_iters[l - 1] += it;
    cnt_.level_calls[l - 1] += 1;
    co_return e < 0 ? e : DWF_OK;
}

// ------------------------------------------------------------ flexible GCR with the K-cycle
template <typename T>
Task Hierarchy::fgcr(int l, const cpx<T>* b, cpx<T>* x, int ncol, const double* rel_tol, int maxit, int restart,
                    int* iters_out, hipStream_t st) {
    const Level& L = levels[l];
    LevelWork& w = work_[l];
    const size_t n = L.vec_elems();
    const size_t nt = n * ncol;
    const int kmax = std::min(restart, w.kmax);
    cpx<T>* r = C<T>(w.r);
    cpx<T>* P = C<T>(w.P);
    cpx<T>* W = C<T>(w.W);
    cpx<T>* t = C<T>(w.tmp);
    cpx<T>* t2 = C<T>(w.tmp2);
    GcrDev& g = w.gcr;
    CO_HIPCHK(vzero<T>(x, nt, st));
    CO_HIPCHK(vconvert<T, T>(b, r, nt, st));
    CO_HIPCHK(norm2<T>(b, n, ncol, g.rr, rw_, st));
    CO_HIPCHK(co_await read_back(st, {{h_scal_, g.rr, sizeof(double) * ncol}}));
    std::vector<double> bb(h_scal_, h_scal_ + ncol), rr(bb);
    std::vector<int> stop(ncol, 0);
    int it = 0, k = 0, status = DWF_OK;
    auto push_stop = [&]() -> int {
        for (int c = 0; c < ncol; ++c) h_int_[c] = stop[c];
        HIPCHK(hipMemcpyAsync(g.stop, h_int_, sizeof(int) * ncol, hipMemcpyHostToDevice, st));
        return DWF_OK;
    };
    auto flush = [&]() -> int {
        if (k == 0) return DWF_OK;
        HIPCHK((gcr_solve_xupdate<T, T>(P, nt, k, x, n, ncol, true, g, st)));
        k = 0;
        return DWF_OK;
    };
    while (true) {
        bool all = true, changed = false;
        for (int c = 0; c < ncol; ++c) {
            if (!std::isfinite(rr[c])) { status = DWF_ENAN; stop[c] = 1; changed = true; }
            if (!stop[c] && rr[c] <= rel_tol[c] * rel_tol[c] * bb[c]) { stop[c] = 1; changed = true; }
            if (!stop[c]) all = false;
        }
        if (all || it >= maxit) break;
        if (changed || it == 0) if (int e = push_stop()) co_return e;
        cpx<T>* Pk = P + (size_t)k * nt;
        cpx<T>* Wk = W + (size_t)k * nt;
        {
            const int e = co_await kcycle<T>(l, r, Pk, ncol, st);
            if (e < 0) co_return e;
        }
        CO_HIPCHK(apply_A<T>(l, Pk, Wk, t, ncol, st));
        CO_HIPCHK(gcr_multidot<T>(W, nt, k, Wk, n, ncol, g, rw_, st));
        CO_HIPCHK(gcr_orth<T>(W, nt, k, Wk, r, n, ncol, g, rw_, st));
        CO_HIPCHK(gcr_rupdate<T>(Wk, r, nullptr, k, n, ncol, true, g, rw_, st));
        ++k;
        ++it;
        CO_HIPCHK(co_await read_back(st, {{h_scal_, g.rr, sizeof(double) * ncol}}));
        for (int c = 0; c < ncol; ++c) if (!stop[c]) rr[c] = h_scal_[c];
        bool conv = true;
        for (int c = 0; c < ncol; ++c)
            if (!stop[c] && !(rr[c] <= rel_tol[c] * rel_tol[c] * bb[c])) conv = false;
        if (k == kmax || conv || it >= maxit) {
            if (int e = flush()) co_return e;
            if (!conv && it < maxit) {
                // true residual for the next cycle
                CO_HIPCHK(apply_A<T>(l, x, t2, t, ncol, st));
                CO_HIPCHK(vsub<T>(b, t2, r, nt, st));
                CO_HIPCHK(norm2<T>(r, n, ncol, g.rr, rw_, st));
                CO_HIPCHK(co_await read_back(st, {{h_scal_, g.rr, sizeof(double) * ncol}}));
                for (int c = 0; c < ncol; ++c) if (!stop[c]) rr[c] = h_scal_[c];
            }
        }
    }
    if (int e = flush()) co_return e;
    // clear the stop mask for the next caller of this level's GCR scalars
    std::fill(stop.begin(), stop.end(), 0);
    if (int e = push_stop()) co_return e;
    if (iters_out) *iters_out = it;
    co_return status;
}

// ------------------------------------------------------------ setup
int Hierarchy::null_vectors(int l, const cpx<double>* start, cpx<double>* v, hipStream_t st) {
    const Level& L = levels[l];
    const int nv = prm.nvec[l];
    const size_t n = L.field2d_elems();
    const size_t nt = n * nv;
    cpx<double>* r = stmp_.r;
    cpx<double>* p = stmp_.p;
    cpx<double>* t = stmp_.t;
    cpx<double>* q = stmp_.q;
    CgScal* s = stmp_.s;
    const double ms = prm.m_setup;
    HIPCHK(vconvert<double, double>(start, v, nt, st));
    // r = -B v, B = D_W(ms) D_W(ms)^dagger
    HIPCHK(apply_wilson<double>(l, v, t, ms, true, nv, st));
    HIPCHK(apply_wilson<double>(l, t, q, ms, false, nv, st));
    HIPCHK(vzero<double>(r, nt, st));
    HIPCHK(vsub<double>(r, q, r, nt, st));
    HIPCHK(cg_init<double>(r, n, nv, s, prm.setup_tol, rw_, st));
    HIPCHK(vconvert<double, double>(r, p, nt, st));
    const int maxit = prm.setup_iters;
    for (int it0 = 0; it0 < maxit; it0 += kCgChunk) {
        const int nchunk = std::min(kCgChunk, maxit - it0);
        for (int c = 0; c < nchunk; ++c) {
            HIPCHK(apply_wilson<double>(l, p, t, ms, true, nv, st));
            HIPCHK(cg_alpha<double>(t, n, nv, s, rw_, st));
            HIPCHK(apply_wilson<double>(l, t, q, ms, false, nv, st));
            HIPCHK(cg_update_xr<double>(v, r, p, q, n, nv, s, st));
            HIPCHK(cg_beta<double>(r, n, nv, s, maxit, rw_, st));
            HIPCHK(cg_update_p<double>(p, r, n, nv, s, st));
        }
        unsigned v = 0;
        HIPCHK(publish(st, {{h_cg_, s, sizeof(CgScal) * nv}}, &v));
        HIPCHK(wait_published(v, st));
        bool all = true;
        for (int c = 0; c < nv; ++c) if (!h_cg_[c].done) all = false;
        if (all) break;
    }
    return DWF_OK;
}

// Level geometry from the parameters, and every device buffer carved from the
// arena ws_ (counting mode: sizes only).  Persistent buffers first; then the
// solve buffers for max_ncol columns, with the setup and eigensolver
// temporaries laid over the same bytes (setup finishes before any solve).
int Hierarchy::plan(int Lx, int Ly, int Ls, int max_ncol) {
    const dwf_mg_params& p = prm;
    levels.clear();
    work_.clear();
    zero_at_setup_.clear();
    max_ncol_ = max_ncol;
    Level f;
    f.Lx = Lx; f.Ly = Ly; f.Ls = Ls; f.n = 2; f.nsites = Lx * Ly; f.fine = true;
    f.vec_prec = p.fine_prec;
    levels.push_back(f);
    for (int l = 0; l < p.nlevels; ++l) {
        Level& L = levels[l];
        const int nv = p.nvec[l], bx = p.block[l][0], by = p.block[l][1];
        L.nvec_next = nv; L.bx = bx; L.by = by;
        Level c;
        c.Lx = L.Lx / bx; c.Ly = L.Ly / by; c.Ls = p.Ls_coarse[l]; c.n = 2 * nv;
        c.nsites = c.Lx * c.Ly; c.fine = false;
        c.vec_prec = p.vec_prec[l];
        c.link_prec = p.link_prec[l];
        levels.push_back(c);
    }
    auto T = [&](size_t bytes) { return dalloc(bytes); };
    const size_t zb = sizeof(cpx<double>);
    // ---- persistent: operators and prolongators
    Level& F = levels[0];
    F.U64 = (cpx<double>*)T(zb * 2 * F.nsites);
    F.U32 = (cpx<float>*)T(sizeof(cpx<float>) * 2 * F.nsites);
    if (!F.U64 || !F.U32) return DWF_EINVAL;
    size_t max_setup = 0;   // complex entries of one level's null-vector block
    for (int l = 0; l < p.nlevels; ++l) {
        Level& L = levels[l];
        Level& c = levels[l + 1];
        const size_t n2 = L.field2d_elems() * L.nvec_next;
        max_setup = std::max(max_setup, n2);
        L.V64 = (cpx<double>*)T(zb * n2);
        L.V32 = (cpx<float>*)T(sizeof(cpx<float>) * n2);
        const size_t nl = (size_t)c.nsites * 5 * c.n * c.n;
        c.links64 = (cpx<double>*)T(zb * nl);
        if (!L.V64 || !L.V32 || !c.links64) return DWF_EINVAL;
        if (c.link_prec == P_F64) {
            c.links = c.links64;
        } else {
            const bool frag = coarse_mfma_supported(c.n, c.link_prec);
            c.links = T(cplx_bytes(c.link_prec) * (frag ? links_fragment16_entries(c.nsites, c.n) : nl));
            if (!c.links) return DWF_EINVAL;
        }
    }
    // ---- persistent: reduction partials, flags, FP64 solve vectors, deflation space
    const int lc = (int)levels.size() - 1;
    const size_t nc_el = levels[lc].vec_elems();
    int dnk = 0, dm = 0;
    if (p.coarsest_nev > 0) deflation_dims(p.coarsest_nev, nc_el, dnk, dm);
    rw_.nblk = kRedBlocks;
    rw_.max_q = 40;
    rw_.max_cols = std::max({max_ncol, 64, dnk});
    rw_.partial = (double*)T(sizeof(double) * (size_t)rw_.max_cols * rw_.max_q * rw_.nblk);
    d_flag_ = (int*)T(sizeof(int) * 4);
    d_pub_ctr_ = (unsigned*)T(sizeof(unsigned) * 4);
    if (d_pub_ctr_) zero_at_setup_.emplace_back(d_pub_ctr_, sizeof(unsigned) * 4);
    const size_t nf = F.vec_elems() * max_ncol;
    r64_ = (cpx<double>*)T(zb * nf);
    t64_ = (cpx<double>*)T(zb * nf);
    bp64_ = (cpx<double>*)T(zb * nf);
    if (!rw_.partial || !d_flag_ || !r64_ || !t64_ || !bp64_) return DWF_EINVAL;
    if (p.pv_poly_order > 0) {
        y64_ = (cpx<double>*)T(zb * nf);
        z64_ = (cpx<double>*)T(zb * nf);
        if (!y64_ || !z64_) return DWF_EINVAL;
    }
    if (p.coarsest_nev > 0) {
        const int nev = p.coarsest_nev;
        def_V_ = (cpx<double>*)T(zb * nc_el * nev);
        def_lam_ = (double*)T(sizeof(double) * nev);
        def_C_ = (cpx<double>*)T(zb * (size_t)nev * max_ncol);
        def_part_ = (double*)T(sizeof(double) * 2 * (size_t)nev * max_ncol * kDeflBlocks);
        def_ref_ = (double*)T(sizeof(double) * max_ncol);
        if (!def_V_ || !def_lam_ || !def_C_ || !def_part_ || !def_ref_) return DWF_EINVAL;
    }
    // ---- solve buffers
    const size_t w0 = ws_.off;
    work_.assign(levels.size(), LevelWork{});
    for (int l = 0; l < (int)levels.size(); ++l)
        if (int e = alloc_level_work(l, max_ncol)) return e;
    const size_t w1 = ws_.off;
    // ---- setup temporaries over the solve buffers
    ws_.off = w0;
    int max_nv = 1;
    for (int l = 0; l < p.nlevels; ++l) max_nv = std::max(max_nv, p.nvec[l]);
    stmp_.v = (cpx<double>*)T(zb * max_setup);
    stmp_.r = (cpx<double>*)T(zb * max_setup);
    stmp_.p = (cpx<double>*)T(zb * max_setup);
    stmp_.t = (cpx<double>*)T(zb * max_setup);
    stmp_.q = (cpx<double>*)T(zb * max_setup);
    stmp_.s = (CgScal*)T(sizeof(CgScal) * max_nv);
    if (!stmp_.v || !stmp_.r || !stmp_.p || !stmp_.t || !stmp_.q || !stmp_.s) return DWF_EINVAL;
    const size_t s1 = ws_.off;
    size_t d1 = w0;
    if (p.coarsest_nev > 0) {
        ws_.off = w0;
        DeflTmp& d = dtmp_;
        d.nk = dnk;
        d.m = dm;
        const size_t nb = (size_t)(dm + 1) * nc_el, nkb = (size_t)dnk * nc_el;
        d.Vb = (cpx<double>*)T(zb * nb);
        d.Ub = (cpx<double>*)T(zb * nkb);
        d.HUb = (cpx<double>*)T(zb * nkb);
        d.Xb = (cpx<double>*)T(zb * nkb);
        d.Wb = (cpx<double>*)T(zb * nkb);
        cpx<double>** vecs[] = {&d.P0, &d.P1, &d.P2, &d.Hh, &d.t1, &d.t2};
        for (auto pp : vecs) *pp = (cpx<double>*)T(zb * nc_el);
        d.G = (cpx<double>*)T(zb * (size_t)dm * dm);
        d.Ysd = (cpx<double>*)T(zb * (size_t)dm * dm);
        d.cdev = (cpx<double>*)T(zb * 2 * (size_t)(dm + 1));
        d.lam = (double*)T(sizeof(double) * dm);
        d.E = (double*)T(sizeof(double) * dm);
        d.nrm = (double*)T(sizeof(double) * dnk);
        d.info = (int*)T(sizeof(int) * 4);
        if (!d.Vb || !d.Ub || !d.HUb || !d.Xb || !d.Wb || !d.P0 || !d.P1 || !d.P2 || !d.Hh || !d.t1 || !d.t2 ||
            !d.G || !d.Ysd || !d.cdev || !d.lam || !d.E || !d.nrm || !d.info)
            return DWF_EINVAL;
        d1 = ws_.off;
    }
    ws_.off = std::max({w1, s1, d1});
    return DWF_OK;
}

size_t Hierarchy::workspace_bytes(int Lx, int Ly, int Ls, const dwf_mg_params& p, int max_ncol) {
    Hierarchy h;
    h.prm = p;
    h.ws_.counting = true;
    h.ws_.cap = ~size_t(0) >> 1;
    if (h.plan(Lx, Ly, Ls, max_ncol) != DWF_OK) return 0;
    return h.ws_.off;
}

int Hierarchy::setup(const cpx<double>* U, int Lx, int Ly, int Ls, double m_, double M5_,
                     const dwf_mg_params& p, const void* const* null_starts, int max_ncol, void* ws,
                     size_t ws_bytes, hipStream_t st) {
    prm = p;
    m = m_;
    M5 = M5_;
    if (max_ncol < 1) return DWF_EINVAL;
    const size_t need = workspace_bytes(Lx, Ly, Ls, p, max_ncol);
    if (need == 0) return DWF_EINVAL;
    if (ws) {
        if (ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) return DWF_EINVAL;
    } else {
        std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
        HIPCHK(hipMalloc(&ws_owned_, need));
        ws = ws_owned_;
        ws_bytes = need;
    }
    ws_ = Arena{};
    ws_.base = static_cast<char*>(ws);
    ws_.cap = ws_bytes;
    if (int e = plan(Lx, Ly, Ls, max_ncol)) return e;
    {
        std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
        if (!st_) HIPCHK(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
        if (!ev_in_) HIPCHK(hipEventCreateWithFlags(&ev_in_, hipEventDisableTiming));
        if (!wait_ev_) HIPCHK(hipEventCreateWithFlags(&wait_ev_, hipEventDisableTiming));
        const int hc = std::max(rw_.max_cols, 64);
        // host-coherent: the publishing kernel stores into them directly
        HIPCHK(hipHostMalloc((void**)&h_scal_, sizeof(double) * 4 * hc, hipHostMallocCoherent));
        HIPCHK(hipHostMalloc((void**)&h_int_, sizeof(int) * 4 * hc, hipHostMallocCoherent));
        HIPCHK(hipHostMalloc((void**)&h_cg_, sizeof(CgScal) * hc, hipHostMallocCoherent));
        HIPCHK(hipHostMalloc((void**)&h_seq_, 64, hipHostMallocCoherent));
        void* hp[4] = {h_scal_, h_int_, h_cg_, h_seq_};
        const size_t hb[4] = {sizeof(double) * 4 * hc, sizeof(int) * 4 * hc, sizeof(CgScal) * hc, 64};
        for (int i = 0; i < 4; ++i) {
            void* d = nullptr;
            HIPCHK(hipHostGetDevicePointer(&d, hp[i], 0));
            views_[i] = HostView{(char*)hp[i], (char*)d, hb[i]};
        }
    }
    const char* ng = std::getenv("DWF_NO_GRAPHS");
    use_graphs_ = !(ng && ng[0] == '1');
    for (auto& z : zero_at_setup_) HIPCHK(hipMemsetAsync(z.first, 0, z.second, st));
    // published numbers restart with the device counter
    *h_seq_ = 0;
    pub_ = 0;
    Level& f = levels[0];
    HIPCHK(hipMemcpyAsync(f.U64, U, sizeof(cpx<double>) * 2 * f.nsites, hipMemcpyDeviceToDevice, st));
    HIPCHK((vconvert<double, float>(f.U64, f.U32, 2 * (size_t)f.nsites, st)));
    for (int l = 0; l < p.nlevels; ++l) {
        Level& L = levels[l];
        Level& c = levels[l + 1];
        const int nv = L.nvec_next, bx = L.bx, by = L.by;
        const int nc = L.n / 2;
        const size_t n2 = L.field2d_elems();
        cpx<double>* v = stmp_.v;
        if (int e = null_vectors(l, reinterpret_cast<const cpx<double>*>(null_starts[l]), v, st)) return e;
        HIPCHK(chiral_columns(v, L.V64, L.nsites, nc, nv, st));
        HIPCHK(hipMemsetAsync(d_flag_, 0, sizeof(int), st));
        HIPCHK(block_orthonormalize(L.V64, L.Lx, L.Ly, nc, nv, bx, by, d_flag_, st));
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, d_flag_, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (bad) return DWF_EBREAKDOWN;
        HIPCHK((vconvert<double, float>(L.V64, L.V32, n2 * nv, st)));
        const size_t nl = (size_t)c.nsites * 5 * c.n * c.n;
        if (L.fine) HIPCHK(galerkin_fine(L.U64, L.V64, c.links64, L.Lx, L.Ly, nv, bx, by, st));
        else HIPCHK(galerkin_coarse(L.links64, L.V64, c.links64, L.Lx, L.Ly, nc, nv, bx, by, st));
        if (c.link_prec != P_F64) {
            if (coarse_mfma_supported(c.n, c.link_prec))
                HIPCHK(convert_links_fragment16(c.links64, c.links, c.link_prec, c.nsites, c.n, st));
            else
                HIPCHK(convert_links(c.links64, c.links, c.link_prec, nl, st));
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    if (int e = deflation_setup(st)) return e;
    return DWF_OK;
}

// ------------------------------------------------------------ solve
// Right-hand sides in groups of at most max_ncol columns; the statistics add
// up over the groups (the residual is the worst, the status the worst code).
Task Hierarchy::solve_task(const cpx<double>* b, cpx<double>* x, int ncol, double tol, int flags,
                           dwf_solve_stats* stats, hipStream_t caller) {
    auto t0 = std::chrono::steady_clock::now();
    if (ncol < 1 || max_ncol_ < 1) co_return DWF_EINVAL;
    // run on the context's stream, after everything already queued on the caller's
    CO_HIPCHK(hipEventRecord(ev_in_, caller));
    CO_HIPCHK(hipStreamWaitEvent(st_, ev_in_, 0));
    const size_t n1 = levels[0].vec_elems();
    dwf_solve_stats tot{};
    int worst = DWF_OK;
    for (int c0 = 0; c0 < ncol; c0 += max_ncol_) {
        const int nc = std::min(max_ncol_, ncol - c0);
        dwf_solve_stats g{};
        const int e = co_await solve_group(b + (size_t)c0 * n1, x + (size_t)c0 * n1, nc, tol, flags, &g, st_);
        if (e < 0 && (worst >= 0 || e < worst)) worst = e;
        else if (e > 0 && worst == DWF_OK) worst = e;
        tot.outer_steps += g.outer_steps;
        tot.fine_iters += g.fine_iters;
        tot.fine_applies += g.fine_applies;
        for (int l = 0; l < DWF_MAX_LEVELS; ++l) {
            tot.level_iters[l] += g.level_iters[l];
            tot.level_calls[l] += g.level_calls[l];
        }
        tot.true_rel_residual = std::max(tot.true_rel_residual, g.true_rel_residual);
        tot.escalations += g.escalations;
        if (e < 0) break;
    }
    // the caller's stream continues after the solve
    CO_HIPCHK(hipEventRecord(ev_in_, st_));
    CO_HIPCHK(hipStreamWaitEvent(caller, ev_in_, 0));
    auto t1 = std::chrono::steady_clock::now();
    if (stats) {
        *stats = tot;
        stats->status = worst;
        stats->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    co_return worst;
}

int Hierarchy::solve(const cpx<double>* b, cpx<double>* x, int ncol, double tol, int flags, dwf_solve_stats* stats,
                     hipStream_t caller) {
    return run(solve_task(b, x, ncol, tol, flags, stats, caller));
}

Task Hierarchy::solve_group(const cpx<double>* b_in, cpx<double>* x, int ncol, double tol, int flags,
                           dwf_solve_stats* stats, hipStream_t st) {
    cnt_ = SolveCounters{};
    const Level& L = levels[0];
    LevelWork& w = work_[0];
    const size_t n = L.vec_elems();
    const size_t nt = n * ncol;
    // the system solved: D_DW x = b, or D_DW x = D_PV b (the propagator form)
    const cpx<double>* b = b_in;
    if (flags & DWF_PV_SOURCE) {
        CO_HIPCHK(fine_dw<double>(L.U64, b_in, bp64_, nullptr, L.Lx, L.Ly, L.Ls, ncol, 1.0, M5, false, nullptr, 1, st));
        cnt_.fine_applies += 1;
        b = bp64_;
    }
    // time the coarse operators' launch configurations for this column count
    // before any of their launches is captured in a graph (captures use the choice)
    if (!coarse_tuned_.count(ncol)) {
        for (int l = 1; l < (int)levels.size(); ++l) {
            const Level& Lc = levels[l];
            if (!coarse_mfma_supported(Lc.n, Lc.link_prec)) continue;
            const size_t nc = Lc.vec_elems() * ncol;
            for (int dg = 0; dg < 2; ++dg) {
                if (Lc.vec_prec == P_F32) {
                    CO_HIPCHK(vzero<float>(C<float>(work_[l].rhs), nc, st));
                    CO_HIPCHK(apply_dw<float>(l, C<float>(work_[l].rhs), C<float>(work_[l].tmp2), m, dg == 1, ncol, st));
                } else {
                    CO_HIPCHK(vzero<double>(C<double>(work_[l].rhs), nc, st));
                    CO_HIPCHK(apply_dw<double>(l, C<double>(work_[l].rhs), C<double>(work_[l].tmp2), m, dg == 1, ncol,
                                               st));
                }
            }
            // and the FP64 levels' A with its FP32 intermediate
            if (Lc.vec_prec != P_F32)
                CO_HIPCHK(apply_A<double>(l, C<double>(work_[l].rhs), C<double>(work_[l].tmp2), C<double>(work_[l].tmp),
                                          ncol, st));
        }
        coarse_tuned_.insert(ncol);
    }
    double* d_s = work_[0].gcr.rr;   // scratch for column norms between inner solves
    CO_HIPCHK(norm2<double>(b, n, ncol, d_s, rw_, st));
    CO_HIPCHK(co_await read_back(st, {{h_scal_, d_s, sizeof(double) * ncol}}));
    std::vector<double> bb(h_scal_, h_scal_ + ncol);
    for (int c = 0; c < ncol; ++c)
        if (!std::isfinite(bb[c])) co_return DWF_ENAN;
    CO_HIPCHK(vzero<double>(x, nt, st));
    const double floor_tol = (L.vec_prec == P_F32) ? 1e-5 : 1e-13;
    const double inner_floor = prm.inner_tol > 0 ? prm.inner_tol : floor_tol;
    int status = DWF_NOT_CONVERGED, outer = 0, total_it = 0, escalations = 0;
    double worst = 0.0, prev_worst = 0.0;
    std::vector<double> rel(ncol, 1.0);
    while (true) {
        CO_HIPCHK(fine_dw<double>(L.U64, x, r64_, b, L.Lx, L.Ly, L.Ls, ncol, m, M5, false, nullptr, 1, st));
        cnt_.fine_applies += 1;
        CO_HIPCHK(norm2<double>(r64_, n, ncol, d_s, rw_, st));
        CO_HIPCHK(co_await read_back(st, {{h_scal_, d_s, sizeof(double) * ncol}}));
        bool all = true;
        worst = 0.0;
        for (int c = 0; c < ncol; ++c) {
            const double rr = h_scal_[c];
            if (!std::isfinite(rr)) { status = DWF_ENAN; all = true; worst = rr; break; }
            rel[c] = bb[c] > 0 ? std::sqrt(rr / bb[c]) : 0.0;
            worst = std::max(worst, rel[c]);
            if (rel[c] > tol) all = false;
        }
        if (verbose_solve())
            std::fprintf(stderr, "[dwfmg] outer step %d: worst relative residual %.3e after %d fine iterations\n",
                         outer, worst, total_it);
        if (status == DWF_ENAN) break;
        if (all) { status = DWF_OK; break; }
        if (outer >= prm.max_outer || total_it >= prm.max_iters) { status = DWF_NOT_CONVERGED; break; }
        // stagnation: the last outer step did not cut the worst residual by the ratio.  A
        // 16-bit coarse kernel is then the suspect: promote it to its FP64 links and go on;
        // with nothing left to promote, stop.  Near the target a step only asks the inner
        // solve for the missing factor (itol below), so a ratio around 0.5 there is normal
        // progress and the default threshold sits well above it.
        if (outer > 0 && prm.stagnation_ratio > 0.0 && worst > prm.stagnation_ratio * prev_worst) {
            if (promote_coarse_links()) {
                ++escalations;
                if (verbose_solve()) std::fprintf(stderr, "[dwfmg] stagnation: coarse links promoted to FP64\n");
            } else {
                if (verbose_solve()) std::fprintf(stderr, "[dwfmg] stagnation with FP64 coarse links: stop\n");
                status = DWF_NOT_CONVERGED;
                break;
            }
        }
        prev_worst = worst;
        // inner right-hand side D_PV^dagger r (with the PV polynomial D_PV^dagger p(X) r)
        if (prm.pv_poly_order > 0) {
            CO_HIPCHK(pv_poly<double>(r64_, y64_, z64_, ncol, st));
            CO_HIPCHK(fine_dw<double>(L.U64, y64_, t64_, nullptr, L.Lx, L.Ly, L.Ls, ncol, 1.0, M5, true, nullptr, 1, st));
            cnt_.fine_applies += 1 + 2 * prm.pv_poly_order;
        } else {
            CO_HIPCHK(fine_dw<double>(L.U64, r64_, t64_, nullptr, L.Lx, L.Ly, L.Ls, ncol, 1.0, M5, true, nullptr, 1, st));
            cnt_.fine_applies += 1;
        }
        CO_HIPCHK(norm2<double>(t64_, n, ncol, d_s, rw_, st));
        CO_HIPCHK(co_await read_back(st, {{h_scal_, d_s, sizeof(double) * ncol}}));
        std::vector<double> itol(ncol);
        for (int c = 0; c < ncol; ++c) {
            const double ra = std::sqrt(h_scal_[c]);
            if (rel[c] <= tol || ra == 0.0) { itol[c] = 2.0; continue; }   // column already converged
            double want = 0.5 * tol * std::sqrt(bb[c]) / ra;
            itol[c] = std::min(0.5, std::max(want, inner_floor));
        }
        int it = 0, e;
        const int maxit = prm.max_iters - total_it;
        if (L.vec_prec == P_F32) {
            CO_HIPCHK((vconvert<double, float>(t64_, C<float>(w.rhs), nt, st)));
            e = co_await fgcr<float>(0, C<float>(w.rhs), C<float>(w.x), ncol, itol.data(), maxit,
                            prm.outer_restart, &it, st);
            if (e < 0) { status = e; break; }
            CO_HIPCHK((vadd<float, double>(C<float>(w.x), x, nt, st)));
        } else {
            CO_HIPCHK((vconvert<double, double>(t64_, C<double>(w.rhs), nt, st)));
            e = co_await fgcr<double>(0, C<double>(w.rhs), C<double>(w.x), ncol, itol.data(), maxit,
                             prm.outer_restart, &it, st);
            if (e < 0) { status = e; break; }
            CO_HIPCHK((vadd<double, double>(C<double>(w.x), x, nt, st)));
        }
        total_it += it;
        ++outer;
        if (it == 0) {
            if (verbose_solve()) std::fprintf(stderr, "[dwfmg] inner solve made no iteration: stop\n");
            status = DWF_NOT_CONVERGED;
            break;
        }
    }
    CO_HIPCHK(co_await sync(st));
    if (stats) {
        stats->status = status;
        stats->outer_steps = outer;
        stats->fine_iters = total_it;
        stats->fine_applies = cnt_.fine_applies;
        for (int l = 0; l < DWF_MAX_LEVELS; ++l) {
            stats->level_iters[l] = cnt_.level_iters[l];
            stats->level_calls[l] = cnt_.level_calls[l];
        }
        stats->true_rel_residual = worst;
        stats->escalations = escalations;
    }
    co_return status;
}

// Stagnation response: every coarse level whose kernel is stored in 16 bits (BF16 or
// FP16 matrix-core fragments) switches to the FP64 links it was built from (kept since
// setup) and the VALU coarse kernel.  The captured graphs hold the old launches and are
// dropped (the stream is idle here: the caller has just read a residual back).
bool Hierarchy::promote_coarse_links() {
    bool any = false;
    for (int l = 1; l < (int)levels.size(); ++l) {
        Level& c = levels[l];
        if (c.link_prec != P_BF16 && c.link_prec != P_F16) continue;
        c.link_prec = P_F64;
        c.links = c.links64;
        any = true;
    }
    if (any) clear_graphs();
    return any;
}

// ------------------------------------------------------------ diagnostics
namespace {
template <typename T>
hipError_t to_prec(const cpx<double>* in, void* out, size_t n, hipStream_t st) {
    return vconvert<double, T>(in, C<T>(out), n, st);
}
template <typename T>
hipError_t from_prec(const void* in, cpx<double>* out, size_t n, hipStream_t st) {
    return vconvert<T, double>(C<T>(in), out, n, st);
}
}  // namespace

int Hierarchy::level_op(int level, int op, const cpx<double>* in, cpx<double>* out, int ncol, double mass,
                        hipStream_t st) {
    if (level < 0 || level >= (int)levels.size() || ncol < 1) return DWF_EINVAL;
    const bool transfer = (op == MG_OP_RESTRICT || op == MG_OP_PROLONG || op == MG_OP_KCYCLE);
    if (transfer && level >= (int)levels.size() - 1) return DWF_EINVAL;
    if (int e = check_cols(ncol)) return e;
    const Level& L = levels[level];
    const size_t nl = L.vec_elems() * ncol;
    const size_t n2 = L.field2d_elems() * ncol;
    const int T32 = (L.vec_prec == P_F32);
    // the level's own solve buffers (2-d fields fit: Ls >= 1); transfers use the
    // next level's right-hand side and solution buffers
    LevelWork& w = work_[level];
    void* bin = w.rhs;
    void* bout = w.x;
    void* btmp = w.tmp;
    size_t nn = 0;
    if (transfer) nn = levels[level + 1].vec_elems() * ncol;
    void* bn = transfer ? (op == MG_OP_PROLONG ? work_[level + 1].x : work_[level + 1].rhs) : nullptr;
    int status = DWF_OK;
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        cpx<T>* xi = C<T>(bin);
        cpx<T>* xo = C<T>(bout);
        cpx<T>* xt = C<T>(btmp);
        const int nxt_prec = transfer ? levels[level + 1].vec_prec : 0;
        switch (op) {
            case MG_OP_DW: case MG_OP_DW_DAG: case MG_OP_PV: case MG_OP_PV_DAG: {
                HIPCHK(to_prec<T>(in, bin, nl, st));
                const double ms = (op == MG_OP_PV || op == MG_OP_PV_DAG) ? 1.0 : m;
                const bool dg = (op == MG_OP_DW_DAG || op == MG_OP_PV_DAG);
                HIPCHK(apply_dw<T>(level, xi, xo, ms, dg, ncol, st));
                HIPCHK(from_prec<T>(bout, out, nl, st));
                return DWF_OK;
            }
            case MG_OP_A:
                HIPCHK(to_prec<T>(in, bin, nl, st));
                HIPCHK(apply_A<T>(level, xi, xo, xt, ncol, st));
                HIPCHK(from_prec<T>(bout, out, nl, st));
                return DWF_OK;
            case MG_OP_WILSON: case MG_OP_WILSON_DAG:
                HIPCHK(to_prec<T>(in, bin, n2, st));
                HIPCHK(apply_wilson<T>(level, xi, xo, mass, op == MG_OP_WILSON_DAG, ncol, st));
                HIPCHK(from_prec<T>(bout, out, n2, st));
                return DWF_OK;
            case MG_OP_RESTRICT:
                HIPCHK(to_prec<T>(in, bin, nl, st));
                HIPCHK(restrict_to<T>(level, xi, bn, ncol, st));
                if (nxt_prec == P_F32) HIPCHK(from_prec<float>(bn, out, nn, st));
                else HIPCHK(from_prec<double>(bn, out, nn, st));
                return DWF_OK;
            case MG_OP_PROLONG:
                if (nxt_prec == P_F32) HIPCHK(to_prec<float>(in, bn, nn, st));
                else HIPCHK(to_prec<double>(in, bn, nn, st));
                HIPCHK(prolong_from<T>(level, bn, xo, ncol, st));
                HIPCHK(from_prec<T>(bout, out, nl, st));
                return DWF_OK;
            case MG_OP_KCYCLE: {
                HIPCHK(to_prec<T>(in, bin, nl, st));
                int e = Hierarchy::run(kcycle<T>(level, xi, xo, ncol, st));
                if (e < 0) return e;
                HIPCHK(from_prec<T>(bout, out, nl, st));
                return DWF_OK;
            }
            default:
                return DWF_EINVAL;
        }
    };
    status = T32 ? run(float{}) : run(double{});
    if (hipStreamSynchronize(st) != hipSuccess && status == DWF_OK) status = DWF_EHIP;
    return status;
}

int Hierarchy::time_op(int level, int op, const cpx<double>* in, int ncol, int iters, double* avg_ms,
                       hipStream_t st) {
    if (level < 0 || level >= (int)levels.size() || ncol < 1 || iters < 1 || !avg_ms) return DWF_EINVAL;
    if (op != MG_OP_DW && op != MG_OP_DW_DAG && op != MG_OP_PV && op != MG_OP_PV_DAG && op != MG_OP_A)
        return DWF_EINVAL;
    if (int e = check_cols(ncol)) return e;
    const Level& L = levels[level];
    LevelWork& w = work_[level];
    const size_t nl = L.vec_elems() * ncol;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        cpx<T>* xi = C<T>(w.rhs);
        cpx<T>* xo = C<T>(w.tmp2);
        cpx<T>* xt = C<T>(w.tmp);
        HIPCHK(to_prec<T>(in, w.rhs, nl, st));
        const double ms = (op == MG_OP_PV || op == MG_OP_PV_DAG) ? 1.0 : m;
        const bool dg = (op == MG_OP_DW_DAG || op == MG_OP_PV_DAG);
        auto once = [&]() -> hipError_t {
            if (op == MG_OP_A) return apply_A<T>(level, xi, xo, xt, ncol, st);
            return apply_dw<T>(level, xi, xo, ms, dg, ncol, st);
        };
        HIPCHK(once());   // warm-up
        HIPCHK(hipEventRecord(e0, st));
        for (int i = 0; i < iters; ++i) HIPCHK(once());
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        *avg_ms = (double)t / iters;
        return DWF_OK;
    };
    int status = (L.vec_prec == P_F32) ? run(float{}) : run(double{});
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

int Hierarchy::coarse_config(int level, int ncol, bool dagger, int* tw, int* tpb) const {
    if (level < 1 || level >= (int)levels.size() || ncol < 1) return DWF_EINVAL;
    const Level& L = levels[level];
    CoarseGeom g{L.Lx, L.Ly, L.Ls, L.n};
    return coarse_mfma_config(L.link_prec, L.vec_prec, g, ncol, dagger, tw, tpb) ? DWF_OK : DWF_EUNSUPPORTED;
}

int Hierarchy::update_links(const cpx<double>* U, hipStream_t st) {
    Level& f = levels[0];
    HIPCHK(hipMemcpyAsync(f.U64, U, sizeof(cpx<double>) * 2 * f.nsites, hipMemcpyDeviceToDevice, st));
    HIPCHK((vconvert<double, float>(f.U64, f.U32, 2 * (size_t)f.nsites, st)));
    return DWF_OK;
}

int Hierarchy::export_level(int level, cpx<double>* V, cpx<double>* kernel, hipStream_t st) {
    if (level < 0 || level >= (int)levels.size() - 1) return DWF_EINVAL;
    const Level& L = levels[level];
    const Level& N = levels[level + 1];
    if (V) HIPCHK(hipMemcpyAsync(V, L.V64, sizeof(cpx<double>) * L.field2d_elems() * L.nvec_next,
                                 hipMemcpyDeviceToDevice, st));
    if (kernel) HIPCHK(export_links(N.links64, kernel, N.nsites, N.n, st));
    HIPCHK(hipStreamSynchronize(st));
    return DWF_OK;
}

}  // namespace dwf
