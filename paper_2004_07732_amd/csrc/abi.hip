// C ABI of the library (declared in include/dwfmg.h): argument checks,
// precision dispatch and status codes.  No exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "mg.hpp"

using namespace dwf;

struct dwf_mg {
    Hierarchy h;
    bool ready = false;
};

namespace {

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline int hip_status(hipError_t e) { return e == hipSuccess ? DWF_OK : DWF_EHIP; }

bool dims_ok(int Lx, int Ly, int Ls, int nrhs) {
    return Lx >= 1 && Ly >= 1 && Ls >= 1 && nrhs >= 1 && (long long)Lx * Ly < (1LL << 30) &&
           (long long)Lx * Ly * Ls * nrhs < (1LL << 40);
}

// A library-owned device buffer shared by calls that may come on different
// streams.  acquire() makes the caller's stream wait for the work that the
// previous call queued on the buffer; release() marks the end of the caller's
// queued work.  (Inside a graph capture neither is recorded: the capturing
// caller orders its own work.)
struct SharedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipEvent_t last = nullptr;
    bool pending = false;
};

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone;
}

void* acquire(SharedBuf& b, size_t bytes, hipStream_t st) {
    if (bytes > b.bytes) {
        std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
        if (b.p) { (void)hipDeviceSynchronize(); (void)hipFree(b.p); }
        b.p = nullptr;
        b.bytes = 0;
        b.pending = false;
        if (hipMalloc(&b.p, bytes) != hipSuccess) { b.p = nullptr; return nullptr; }
        b.bytes = bytes;
    }
    if (!b.last && hipEventCreateWithFlags(&b.last, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (b.pending && !capturing(st) && hipStreamWaitEvent(st, b.last, 0) != hipSuccess) return nullptr;
    return b.p;
}

int release(SharedBuf& b, hipStream_t st, int status) {
    if (!capturing(st) && hipEventRecord(b.last, st) == hipSuccess) b.pending = true;
    return status;
}

void drop(SharedBuf& b) {
    std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
    if (b.p) { (void)hipDeviceSynchronize(); (void)hipFree(b.p); }
    b.p = nullptr;
    b.bytes = 0;
    b.pending = false;
}

// the intermediate fields of the product modes of dwf_pv_apply / dwf_pv_poly_apply,
// and the partial sums of dwf_norm2
std::mutex g_scratch_mu;
SharedBuf g_fields, g_partials;

template <typename R>
int pv_apply_t(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, double m,
               double M5, int mode, hipStream_t st) {
    auto u = reinterpret_cast<const cpx<R>*>(U);
    auto in = reinterpret_cast<const cpx<R>*>(psi);
    auto o = reinterpret_cast<cpx<R>*>(out);
    switch (mode) {
        case DWF_PV: return hip_status(fine_dw<R>(u, in, o, nullptr, Lx, Ly, Ls, nrhs, 1.0, M5, false, nullptr, 1, st));
        case DWF_PV_DAG: return hip_status(fine_dw<R>(u, in, o, nullptr, Lx, Ly, Ls, nrhs, 1.0, M5, true, nullptr, 1, st));
        case DWF_PVDAG_DW:
        case DWF_PVDAG_DW_DAG: {
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            const size_t bytes = sizeof(cpx<R>) * 2 * (size_t)Lx * Ly * Ls * nrhs;
            auto t = reinterpret_cast<cpx<R>*>(acquire(g_fields, bytes, st));
            if (!t) return DWF_EHIP;
            const double m1 = (mode == DWF_PVDAG_DW) ? m : 1.0, m2 = (mode == DWF_PVDAG_DW) ? 1.0 : m;
            if (fine_dw<R>(u, in, t, nullptr, Lx, Ly, Ls, nrhs, m1, M5, false, nullptr, 1, st) != hipSuccess)
                return release(g_fields, st, DWF_EHIP);
            return release(g_fields, st,
                           hip_status(fine_dw<R>(u, t, o, nullptr, Lx, Ly, Ls, nrhs, m2, M5, true, nullptr, 1, st)));
        }
        default: return DWF_EINVAL;
    }
}

// out = D_PV^dag p(X) D_DW psi (or D_DW^dag p(X) D_PV psi), X = D_PV D_PV^dag,
// p(X) w by Horner's scheme: y = c_K w, then y = c_k w + X y for k = K-1..0;
// t holds three fields of n complex entries
template <typename R>
int pv_poly_chain(const cpx<R>* u, const cpx<R>* in, cpx<R>* o, cpx<R>* t, size_t n, int Lx, int Ly, int Ls, int nrhs,
                  double m, double M5, const double* c, int order, bool dag, hipStream_t st) {
    cpx<R>* w = t;
    cpx<R>* y = t + n;
    cpx<R>* z = t + 2 * n;
    auto D = [&](const cpx<R>* a, cpx<R>* b, double mass, bool adj) {
        return fine_dw<R>(u, a, b, nullptr, Lx, Ly, Ls, nrhs, mass, M5, adj, nullptr, 1, st);
    };
    if ((dag ? D(in, w, 1.0, false) : D(in, w, m, false)) != hipSuccess) return DWF_EHIP;
    if (vaxpby<R>(c[order], w, 0.0, y, n, st) != hipSuccess) return DWF_EHIP;
    for (int k = order - 1; k >= 0; --k) {
        if (D(y, z, 1.0, true) != hipSuccess || D(z, y, 1.0, false) != hipSuccess) return DWF_EHIP;
        if (vaxpby<R>(c[k], w, 1.0, y, n, st) != hipSuccess) return DWF_EHIP;
    }
    return hip_status(dag ? D(y, o, m, true) : D(y, o, 1.0, true));
}

template <typename R>
int pv_poly_apply_t(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, double m,
                    double M5, const double* c, int order, bool dag, hipStream_t st) {
    auto u = reinterpret_cast<const cpx<R>*>(U);
    auto in = reinterpret_cast<const cpx<R>*>(psi);
    auto o = reinterpret_cast<cpx<R>*>(out);
    const size_t n = (size_t)2 * Lx * Ly * Ls * nrhs;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto t = reinterpret_cast<cpx<R>*>(acquire(g_fields, sizeof(cpx<R>) * 3 * n, st));
    if (!t) return DWF_EHIP;
    const int status = pv_poly_chain<R>(u, in, o, t, n, Lx, Ly, Ls, nrhs, m, M5, c, order, dag, st);
    return release(g_fields, st, status);
}


bool valid_prec(int p, bool link) {
    if (p == DWF_P_F64 || p == DWF_P_F32) return true;
    return link && (p == DWF_P_BF16 || p == DWF_P_F16);
}

}  // namespace

extern "C" {

int dwf_apply(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, double m_f,
              double M5, int flags, void* stream) {
    if (!U || !psi || !out || psi == out || !dims_ok(Lx, Ly, Ls, nrhs)) return DWF_EINVAL;
    if (!std::isfinite(m_f) || !std::isfinite(M5)) return DWF_EINVAL;
    const bool dag = flags & DWF_DAGGER;
    if (flags & DWF_PREC_F32)
        return hip_status(fine_dw<float>((const cpx<float>*)U, (const cpx<float>*)psi, (cpx<float>*)out, nullptr, Lx, Ly,
                                         Ls, nrhs, m_f, M5, dag, nullptr, 1, S(stream)));
    return hip_status(fine_dw<double>((const cpx<double>*)U, (const cpx<double>*)psi, (cpx<double>*)out, nullptr, Lx,
                                      Ly, Ls, nrhs, m_f, M5, dag, nullptr, 1, S(stream)));
}

int dwf_pv_poly_apply(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, double m_f,
                      double M5, const double* c, int order, int flags, void* stream) {
    if (!U || !psi || !out || !c || psi == out || !dims_ok(Lx, Ly, Ls, nrhs)) return DWF_EINVAL;
    if (!std::isfinite(m_f) || !std::isfinite(M5) || order < 0 || order > DWF_PV_POLY_MAX) return DWF_EINVAL;
    for (int k = 0; k <= order; ++k)
        if (!std::isfinite(c[k])) return DWF_EINVAL;
    const bool dag = flags & DWF_DAGGER;
    if (flags & DWF_PREC_F32)
        return pv_poly_apply_t<float>(U, psi, out, Lx, Ly, Ls, nrhs, m_f, M5, c, order, dag, S(stream));
    return pv_poly_apply_t<double>(U, psi, out, Lx, Ly, Ls, nrhs, m_f, M5, c, order, dag, S(stream));
}

int dwf_pv_poly_chebyshev(int order, double lam_min, double lam_max, double* c) {
    if (!c || order < 0 || order > DWF_PV_POLY_MAX) return DWF_EINVAL;
    if (!(lam_min > 0.0) || !(lam_max > lam_min) || !std::isfinite(lam_max)) return DWF_EINVAL;
    // r(x) = 1 - x p(x) = T_n(a + b x) / T_n(a), n = order + 1: power-series
    // coefficients of T_j(a + b x) from T_{j+1} = 2 (a + b x) T_j - T_{j-1}
    const int n = order + 1;
    const double a = (lam_max + lam_min) / (lam_max - lam_min), b = -2.0 / (lam_max - lam_min);
    double t0[DWF_PV_POLY_MAX + 3] = {0.0}, t1[DWF_PV_POLY_MAX + 3] = {0.0};
    t0[0] = 1.0;            // T_0
    t1[0] = a; t1[1] = b;   // T_1
    for (int j = 1; j < n; ++j) {
        double nx[DWF_PV_POLY_MAX + 3] = {0.0};
        for (int i = 0; i <= j; ++i) {
            nx[i] += 2.0 * a * t1[i];
            nx[i + 1] += 2.0 * b * t1[i];
        }
        for (int i = 0; i <= j + 1; ++i) nx[i] -= t0[i];
        for (int i = 0; i <= n; ++i) { t0[i] = t1[i]; t1[i] = nx[i]; }
    }
    // t1 now holds T_n(a + b x); p(x) = -(r_1 + r_2 x + ...) with r = t1 / t1[0]
    for (int k = 0; k <= order; ++k) c[k] = -t1[k + 1] / t1[0];
    return DWF_OK;
}

int dwf_fine_config(int shape, int chunk) { return set_fine_config(shape, chunk) ? DWF_OK : DWF_EINVAL; }

int dwf_fine_a_config(int shape, int chunk) { return set_fine_a_config(shape, chunk) ? DWF_OK : DWF_EINVAL; }

int dwf_fine_a_chosen(int prec, int Lx, int Ly, int Ls, int nrhs, int* shape, int* chunk) {
    if (!shape || !chunk || (prec != 0 && prec != DWF_PREC_F32)) return DWF_EINVAL;
    const int bytes = prec == DWF_PREC_F32 ? (int)sizeof(float) : (int)sizeof(double);
    return fine_a_chosen(bytes, Lx, Ly, Ls, nrhs, shape, chunk) ? DWF_OK : DWF_EINVAL;
}

int dwf_pv_apply(const void* U, const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, double m_f,
                 double M5, int mode, int flags, void* stream) {
    if (!U || !psi || !out || psi == out || !dims_ok(Lx, Ly, Ls, nrhs)) return DWF_EINVAL;
    if (!std::isfinite(m_f) || !std::isfinite(M5) || mode < DWF_PV || mode > DWF_PVINV_DW) return DWF_EINVAL;
    if (mode == DWF_PVINV_DW) {
        if (flags & DWF_PREC_F32) return DWF_EUNSUPPORTED;
        if (Ls < 2) return DWF_EINVAL;
        // D_DW psi into the intermediate field, then D_PV out = D_DW psi per right-hand side
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        const size_t V = 2 * (size_t)Lx * Ly * Ls;
        auto t = reinterpret_cast<cpx<double>*>(acquire(g_fields, sizeof(cpx<double>) * V * nrhs, S(stream)));
        if (!t) return DWF_EHIP;
        const auto u = reinterpret_cast<const cpx<double>*>(U);
        if (fine_dw<double>(u, reinterpret_cast<const cpx<double>*>(psi), t, nullptr, Lx, Ly, Ls, nrhs, m_f, M5, false,
                            nullptr, 1, S(stream)) != hipSuccess)
            return release(g_fields, S(stream), DWF_EHIP);
        int worst = DWF_OK;
        for (int r = 0; r < nrhs; ++r) {
            const int e = krylov_solve(u, t + r * V, reinterpret_cast<cpx<double>*>(out) + r * V, Lx, Ly, Ls, 1.0, M5,
                                       DWF_KRYLOV_CGNR, 0, 1e-12, 10000, nullptr, S(stream));
            if (e < 0) return release(g_fields, S(stream), e);
            if (e > worst) worst = e;
        }
        return release(g_fields, S(stream), worst);
    }
    if (flags & DWF_PREC_F32) return pv_apply_t<float>(U, psi, out, Lx, Ly, Ls, nrhs, m_f, M5, mode, S(stream));
    return pv_apply_t<double>(U, psi, out, Lx, Ly, Ls, nrhs, m_f, M5, mode, S(stream));
}

int dwf_wilson_apply(const void* U, const void* psi, void* out, int Lx, int Ly, int nrhs, double M, int flags,
                     void* stream) {
    if (!U || !psi || !out || psi == out || !dims_ok(Lx, Ly, 1, nrhs) || !std::isfinite(M)) return DWF_EINVAL;
    const bool dag = flags & DWF_DAGGER;
    if (flags & DWF_PREC_F32)
        return hip_status(wilson2d<float>((const cpx<float>*)U, (const cpx<float>*)psi, (cpx<float>*)out, Lx, Ly, nrhs,
                                          M, dag, S(stream)));
    return hip_status(wilson2d<double>((const cpx<double>*)U, (const cpx<double>*)psi, (cpx<double>*)out, Lx, Ly, nrhs,
                                       M, dag, S(stream)));
}

int dwf_gamma5R(const void* psi, void* out, int Lx, int Ly, int Ls, int nrhs, int flags, void* stream) {
    if (!psi || !out || psi == out || !dims_ok(Lx, Ly, Ls, nrhs)) return DWF_EINVAL;
    if (flags & DWF_PREC_F32)
        return hip_status(gamma5R<float>((const cpx<float>*)psi, (cpx<float>*)out, Lx * Ly, Ls, nrhs, S(stream)));
    return hip_status(gamma5R<double>((const cpx<double>*)psi, (cpx<double>*)out, Lx * Ly, Ls, nrhs, S(stream)));
}

int dwf_gauge_transform(const void* U, const void* g, const void* psi, void* Ug, void* psig, int Lx, int Ly, int Ls,
                        int nrhs, void* stream) {
    if (!g || !dims_ok(Lx, Ly, Ls, nrhs)) return DWF_EINVAL;
    if (Ug && !U) return DWF_EINVAL;
    if (psig && !psi) return DWF_EINVAL;
    return hip_status(gauge_transform((const cpx<double>*)U, (const cpx<double>*)g, (const cpx<double>*)psi,
                                      (cpx<double>*)Ug, (cpx<double>*)psig, Lx, Ly, Ls, nrhs, S(stream)));
}

int dwf_pack(const void* in_c128, void* out_c64, size_t n, void* stream) {
    if (!in_c128 || !out_c64) return DWF_EINVAL;
    if (n == 0) return DWF_OK;
    return hip_status(vconvert<double, float>((const cpx<double>*)in_c128, (cpx<float>*)out_c64, n, S(stream)));
}

int dwf_unpack(const void* in_c64, void* out_c128, size_t n, void* stream) {
    if (!in_c64 || !out_c128) return DWF_EINVAL;
    if (n == 0) return DWF_OK;
    return hip_status(vconvert<float, double>((const cpx<float>*)in_c64, (cpx<double>*)out_c128, n, S(stream)));
}

int dwf_force(const void* U, const void* X, const void* Y, double* F, int Lx, int Ly, int Ls, int nrhs, void* stream) {
    if (!U || !X || !Y || !F || !dims_ok(Lx, Ly, Ls, nrhs)) return DWF_EINVAL;
    return hip_status(force((const cpx<double>*)U, (const cpx<double>*)X, (const cpx<double>*)Y, F, Lx, Ly, Ls, nrhs,
                            S(stream)));
}

int dwf_links_from_theta(const double* theta, void* U, int Lx, int Ly, void* stream) {
    if (!theta || !U || !dims_ok(Lx, Ly, 1, 1)) return DWF_EINVAL;
    return hip_status(links_from_theta(theta, (cpx<double>*)U, 2LL * Lx * Ly, S(stream)));
}

int dwf_krylov_solve(const void* U, const void* b, void* x, int Lx, int Ly, int Ls, double m_f, double M5,
                     int method, int ell, double tol, int maxit, dwf_solve_stats* stats, void* stream) {
    if (!U || !b || !x || !dims_ok(Lx, Ly, Ls, 1) || Ls < 2) return DWF_EINVAL;
    if (!std::isfinite(m_f) || !std::isfinite(M5) || !(tol > 0.0) || maxit < 1) return DWF_EINVAL;
    if (method != DWF_KRYLOV_CGNR && method != DWF_KRYLOV_BICGSTAB) return DWF_EINVAL;
    if (method == DWF_KRYLOV_BICGSTAB && (ell < 1 || ell > 16)) return DWF_EINVAL;
    return krylov_solve((const cpx<double>*)U, (const cpx<double>*)b, (cpx<double>*)x, Lx, Ly, Ls, m_f, M5, method,
                        ell, tol, maxit, stats, S(stream));
}

void dwf_mg_default_params(dwf_mg_params* p, int nlevels) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    if (nlevels < 1) nlevels = 1;
    if (nlevels > DWF_MAX_LEVELS) nlevels = DWF_MAX_LEVELS;
    p->nlevels = nlevels;
    for (int l = 0; l < DWF_MAX_LEVELS; ++l) {
        p->nvec[l] = (l == 0) ? 8 : 12;           // Table kcycle
        p->block[l][0] = p->block[l][1] = (l == 0) ? 4 : 2;
        p->Ls_coarse[l] = 4;
        p->link_prec[l] = DWF_P_F64;
        p->vec_prec[l] = DWF_P_F64;
    }
    p->fine_prec = DWF_P_F64;
    p->m_setup = 0.0;
    p->setup_iters = 250;
    p->setup_tol = 1e-4;
    p->outer_restart = 16;
    p->smooth_iters = 8;
    p->smooth_restart = 0;
    p->inter_maxit = 16;
    p->inter_tol = 0.25;
    p->inter_restart = 16;
    p->coarsest_maxit = 1024;
    p->coarsest_tol = 0.05;
    p->inner_tol = 0.0;
    p->max_iters = 10000;
    p->max_outer = 20;
    p->coarsest_nev = 0;
    p->eig_degree = 0;
    p->eig_maxit = 40;
    p->eig_tol = 1e-3;
    p->coarsest_solver = DWF_COARSEST_CGNR;
    p->coarsest_restart = 16;
    p->transfer = DWF_TRANSFER_WALL;
    p->pv_poly_order = 0;
    p->stagnation_ratio = 0.9;
    for (int k = 0; k <= DWF_PV_POLY_MAX; ++k) p->pv_poly[k] = (k == 0) ? 1.0 : 0.0;
}

int mg_deflation_info(const dwf_mg* mg, int* nev, int* iters, double* worst_residual, double* lambdas) {
    if (!mg || !mg->ready) return DWF_ENOSETUP;
    if (nev) *nev = mg->h.def_nev_;
    if (iters) *iters = mg->h.eig_iters_;
    if (worst_residual) *worst_residual = mg->h.eig_worst_;
    if (lambdas)
        for (int i = 0; i < mg->h.def_nev_; ++i) lambdas[i] = mg->h.def_lam_host_[i];
    return DWF_OK;
}

}  // extern "C"

namespace {

// argument checks shared by mg_workspace_bytes and mg_setup
int check_mg_args(int Lx, int Ly, int Ls, double m_f, double M5, const dwf_mg_params* p, int max_nrhs) {
    if (!p) return DWF_EINVAL;
    if (!dims_ok(Lx, Ly, Ls, 1) || Ls < 2 || !std::isfinite(m_f) || !std::isfinite(M5)) return DWF_EINVAL;
    if (max_nrhs < 1 || max_nrhs > 4096) return DWF_EINVAL;
    if (p->nlevels < 1 || p->nlevels > DWF_MAX_LEVELS) return DWF_EINVAL;
    if (p->outer_restart < 1 || p->outer_restart > 16 || p->smooth_iters < 0) return DWF_EINVAL;
    // one smoothing cycle is at most 16 steps; with a restart, up to 64 steps in all
    if (p->smooth_restart < 0 || p->smooth_restart > 16) return DWF_EINVAL;
    if (p->smooth_iters > (p->smooth_restart > 0 ? 64 : 16)) return DWF_EINVAL;
    if (p->nlevels > 1 && (p->inter_restart < 1 || p->inter_restart > 16)) return DWF_EINVAL;
    if (!valid_prec(p->fine_prec, false)) return DWF_EINVAL;
    if (p->coarsest_nev < 0 || (p->coarsest_nev > 0 && (p->eig_maxit < 1 || p->eig_degree < 0 || !(p->eig_tol > 0.0))))
        return DWF_EINVAL;
    if (p->coarsest_nev > 0 && p->vec_prec[p->nlevels - 1] != DWF_P_F64) return DWF_EUNSUPPORTED;
    if (p->coarsest_solver != DWF_COARSEST_CGNR && p->coarsest_solver != DWF_COARSEST_GCR) return DWF_EINVAL;
    if (p->coarsest_solver == DWF_COARSEST_GCR && (p->coarsest_restart < 1 || p->coarsest_restart > 16))
        return DWF_EINVAL;
    if (p->transfer != DWF_TRANSFER_WALL && p->transfer != DWF_TRANSFER_BULK && p->transfer != DWF_TRANSFER_SLICE1)
        return DWF_EINVAL;
    if (p->pv_poly_order < 0 || p->pv_poly_order > DWF_PV_POLY_MAX) return DWF_EINVAL;
    if (!(p->stagnation_ratio >= 0.0) || !(p->stagnation_ratio < 1.0)) return DWF_EINVAL;
    for (int k = 0; k <= p->pv_poly_order; ++k)
        if (!std::isfinite(p->pv_poly[k])) return DWF_EINVAL;
    if (p->transfer == DWF_TRANSFER_BULK)
        for (int l = 0; l < p->nlevels; ++l)
            if (p->Ls_coarse[l] != (l == 0 ? Ls : p->Ls_coarse[l - 1])) return DWF_EINVAL;
    int lx = Lx, ly = Ly, n = 2;
    for (int l = 0; l < p->nlevels; ++l) {
        const int bx = p->block[l][0], by = p->block[l][1], nv = p->nvec[l];
        if (bx < 1 || by < 1 || lx % bx || ly % by || nv < 1) return DWF_EINVAL;
        if (nv > bx * by * (n / 2)) return DWF_EINVAL;
        if (p->Ls_coarse[l] < 2 || p->Ls_coarse[l] > kMaxCoarseLs) return DWF_EINVAL;
        if (!valid_prec(p->link_prec[l], true) || !valid_prec(p->vec_prec[l], false)) return DWF_EINVAL;
        const int nn = 2 * nv;
        if (nn != 4 && nn != 8 && nn != 12 && nn != 16 && nn != 24 && nn != 32 && nn != 48 && nn != 64)
            return DWF_EUNSUPPORTED;
        if ((long long)bx * by * (n / 2) * nv > 4096) return DWF_EUNSUPPORTED;
        lx /= bx;
        ly /= by;
        n = nn;
    }
    return DWF_OK;
}

}  // namespace

extern "C" {

size_t mg_workspace_bytes(int Lx, int Ly, int Ls, int max_nrhs, const dwf_mg_params* p) {
    if (check_mg_args(Lx, Ly, Ls, 0.0, -1.0, p, max_nrhs) != DWF_OK) return 0;
    return Hierarchy::workspace_bytes(Lx, Ly, Ls, *p, max_nrhs);
}

int mg_setup(dwf_mg** out, const void* U, int Lx, int Ly, int Ls, double m_f, double M5, const dwf_mg_params* p,
             const void* const* null_starts, int max_nrhs, void* workspace, size_t ws_bytes, void* stream) {
    if (!out || !U || !p || !null_starts) return DWF_EINVAL;
    *out = nullptr;
    if (int e = check_mg_args(Lx, Ly, Ls, m_f, M5, p, max_nrhs)) return e;
    for (int l = 0; l < p->nlevels; ++l)
        if (!null_starts[l]) return DWF_EINVAL;
    dwf_mg* mg = new (std::nothrow) dwf_mg;
    if (!mg) return DWF_EHIP;
    int e = mg->h.setup((const cpx<double>*)U, Lx, Ly, Ls, m_f, M5, *p, null_starts, max_nrhs, workspace, ws_bytes,
                        S(stream));
    if (e != DWF_OK) {
        delete mg;
        return e;
    }
    mg->ready = true;
    *out = mg;
    return DWF_OK;
}

int mg_solve(dwf_mg* mg, const void* b, void* x, int nrhs, double tol, int flags, dwf_solve_stats* st, void* stream) {
    if (!mg || !mg->ready) return DWF_ENOSETUP;
    if (!b || !x || b == x || nrhs < 1 || !(tol > 0.0) || !std::isfinite(tol)) return DWF_EINVAL;
    if (flags & ~DWF_PV_SOURCE) return DWF_EINVAL;
    if (st) std::memset(st, 0, sizeof(*st));
    int e = mg->h.solve((const cpx<double>*)b, (cpx<double>*)x, nrhs, tol, flags, st, S(stream));
    if (st) st->status = e;
    return e;
}

int mg_level_op(dwf_mg* mg, int level, int op, const void* in, void* out, int ncol, double mass, void* stream) {
    if (!mg || !mg->ready) return DWF_ENOSETUP;
    if (!in || !out || in == out) return DWF_EINVAL;
    return mg->h.level_op(level, op, (const cpx<double>*)in, (cpx<double>*)out, ncol, mass, S(stream));
}

int mg_solve_batch(int nctx, dwf_mg* const* ctx, const void* const* b, void* const* x, const int* nrhs, double tol,
                   int flags, dwf_solve_stats* stats, void* stream) {
    if (nctx < 1 || !ctx || !b || !x || !nrhs || !(tol > 0.0) || !std::isfinite(tol)) return DWF_EINVAL;
    if (flags & ~DWF_PV_SOURCE) return DWF_EINVAL;
    for (int i = 0; i < nctx; ++i) {
        if (!ctx[i] || !ctx[i]->ready) return DWF_ENOSETUP;
        if (!b[i] || !x[i] || b[i] == x[i] || nrhs[i] < 1) return DWF_EINVAL;
        for (int j = 0; j < i; ++j)
            if (ctx[j] == ctx[i]) return DWF_EINVAL;
    }
    // every context starts after the caller's queued work
    if (hipStreamSynchronize(S(stream)) != hipSuccess) return DWF_EHIP;
    // one host thread keeps every solve in flight: each runs on its context's
    // stream until it needs scalars back on the host, and is resumed once that
    // stream has caught up, while the other contexts' work proceeds on the GPU
    std::vector<int> codes(nctx, DWF_OK);
    std::vector<dwf_solve_stats> st(nctx);
    std::vector<Task> tasks(nctx);
    for (int i = 0; i < nctx; ++i) {
        std::memset(&st[i], 0, sizeof(st[i]));
        ctx[i]->h.set_batch(true);
        tasks[i] = ctx[i]->h.solve_task((const cpx<double>*)b[i], (cpx<double>*)x[i], nrhs[i], tol, flags, &st[i],
                                        ctx[i]->h.stream());
        tasks[i].start();
    }
    for (;;) {
        bool all_done = true, progressed = false;
        for (int i = 0; i < nctx; ++i) {
            if (tasks[i].done()) continue;
            all_done = false;
            if (ctx[i]->h.poll()) progressed = true;
        }
        if (all_done) break;
        if (!progressed) std::this_thread::yield();
    }
    for (int i = 0; i < nctx; ++i) {
        ctx[i]->h.set_batch(false);
        codes[i] = tasks[i].result();
        st[i].status = codes[i];
    }
    int worst = DWF_OK;
    for (int i = 0; i < nctx; ++i) {
        if (stats) stats[i] = st[i];
        const int c = codes[i];
        if (c < 0 && (worst >= 0 || c < worst)) worst = c;
        else if (c > 0 && worst == DWF_OK) worst = c;
    }
    return worst;
}

int dwf_copy_bandwidth(const void* src, void* dst, size_t bytes, int iters, double* gb_per_s, void* stream) {
    if (!src || !dst || src == dst || !gb_per_s || iters < 1 || bytes < 16 || (bytes & 15) ||
        (reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
        return DWF_EINVAL;
    hipStream_t st = S(stream);
    const size_t words = bytes / 16;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return DWF_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return DWF_EHIP; }
    int status = DWF_OK;
    float ms = 0.f;
    if (stream_copy(src, dst, words, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess) status = DWF_EHIP;
    for (int i = 0; i < iters && status == DWF_OK; ++i)
        if (stream_copy(src, dst, words, st) != hipSuccess) status = DWF_EHIP;
    if (status == DWF_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        status = DWF_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status == DWF_OK) *gb_per_s = 2.0 * (double)bytes * iters / ((double)ms * 1e-3) / 1e9;
    return status;
}

int dwf_norm2(const void* x, size_t n, int ncol, double* out, void* stream) {
    if (!x || !out || ncol < 1 || n == 0) return DWF_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    RedWork rw;
    rw.nblk = kRedBlocks;
    rw.max_q = 1;
    rw.max_cols = ncol;
    rw.partial = reinterpret_cast<double*>(acquire(g_partials, sizeof(double) * (size_t)rw.nblk * ncol, S(stream)));
    if (!rw.partial) return DWF_EHIP;
    return release(g_partials, S(stream), hip_status(norm2<double>((const cpx<double>*)x, n, ncol, out, rw, S(stream))));
}

int mg_update_links(dwf_mg* mg, const void* U, void* stream) {
    if (!mg || !mg->ready) return DWF_ENOSETUP;
    if (!U) return DWF_EINVAL;
    return mg->h.update_links((const cpx<double>*)U, S(stream));
}

int mg_time_op(dwf_mg* mg, int level, int op, const void* in, int ncol, int iters, double* avg_ms, void* stream) {
    if (!mg || !mg->ready) return DWF_ENOSETUP;
    if (!in || !avg_ms) return DWF_EINVAL;
    return mg->h.time_op(level, op, (const cpx<double>*)in, ncol, iters, avg_ms, S(stream));
}

int mg_export(dwf_mg* mg, int level, void* prolongator, void* coarse_kernel, void* stream) {
    if (!mg || !mg->ready) return DWF_ENOSETUP;
    return mg->h.export_level(level, (cpx<double>*)prolongator, (cpx<double>*)coarse_kernel, S(stream));
}

int mg_coarse_config(const dwf_mg* mg, int level, int ncol, int dagger, int* tile_width, int* tiles_per_block) {
    if (!mg || !mg->ready) return DWF_ENOSETUP;
    if (!tile_width || !tiles_per_block) return DWF_EINVAL;
    return mg->h.coarse_config(level, ncol, dagger != 0, tile_width, tiles_per_block);
}

int mg_level_info(const dwf_mg* mg, int level, int* Lx, int* Ly, int* Ls, int* n, int* nvec) {
    if (!mg || !mg->ready) return DWF_ENOSETUP;
    if (level < 0 || level >= (int)mg->h.levels.size()) return DWF_EINVAL;
    const Level& L = mg->h.levels[level];
    if (Lx) *Lx = L.Lx;
    if (Ly) *Ly = L.Ly;
    if (Ls) *Ls = L.Ls;
    if (n) *n = L.n;
    if (nvec) *nvec = L.nvec_next;
    return DWF_OK;
}

int mg_destroy(dwf_mg* mg) {
    if (!mg) return DWF_EINVAL;
    hipDeviceSynchronize();
    delete mg;
    return DWF_OK;
}

int dwf_release_scratch(void) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    drop(g_fields);
    drop(g_partials);
    return DWF_OK;
}

const char* dwf_strerror(int code) {
    switch (code) {
        case DWF_OK: return "ok";
        case DWF_NOT_CONVERGED: return "not converged: iteration caps reached";
        case DWF_EINVAL: return "invalid argument";
        case DWF_EHIP: return "HIP runtime error";
        case DWF_EBREAKDOWN: return "Krylov or Gram-Schmidt breakdown";
        case DWF_ENAN: return "non-finite value";
        case DWF_ENOSETUP: return "multigrid context missing or not set up";
        case DWF_EUNSUPPORTED: return "unsupported size or option";
        case DWF_ESCRATCH: return "input larger than the static scratch of an allocation-free entry point";
        default: return "unknown status";
    }
}

}  // extern "C"
