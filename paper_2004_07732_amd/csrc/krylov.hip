// Krylov solvers of D_DW x = b without multigrid: the two baselines of the
// paper's solver comparison (Sec. 3, Fig. iterationscompare), counted in
// applications of D_DW, D_DW^dagger and D_PV^dagger as the paper counts them.
//
//   CGNR: CG on D_DW^dagger D_DW x = D_DW^dagger b, keeping r = b - D_DW x and
//         stopping on |r| <= tol |b|.
//   BiCGStab(ell) (Sleijpen & Fokkema 1993) on A x = b' with A = D_PV^dagger
//         D_DW and b' = D_PV^dagger b (the same x; A has its spectrum in the
//         right half-plane, appendix of the paper): ell BiCG steps then one
//         minimal-residual step by modified Gram-Schmidt per cycle, stopping on
//         |r'| <= tol |b'|.  If the true residual of D_DW x = b is then above
//         tol, the method restarts from x with a tolerance ten times smaller.
//
// FP64, one right-hand side.  The host keeps the scalars: every inner product
// is a device reduction read back at once, which is simple and adequate for a
// comparison baseline (the operator applications dominate at the sizes used).
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "mg.hpp"

namespace dwf {

namespace {

using zc = std::complex<double>;

__global__ void k_axpy(cpx<double> a, const cpx<double>* __restrict__ x, cpx<double>* __restrict__ y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const cpx<double> v = x[i];
        cpx<double> w = y[i];
        w.re += a.re * v.re - a.im * v.im;
        w.im += a.re * v.im + a.im * v.re;
        y[i] = w;
    }
}
// y = x + a y
__global__ void k_xpay(const cpx<double>* __restrict__ x, cpx<double> a, cpx<double>* __restrict__ y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const cpx<double> v = y[i], u = x[i];
        y[i] = {u.re + a.re * v.re - a.im * v.im, u.im + a.re * v.im + a.im * v.re};
    }
}

inline unsigned ew_blocks(size_t n) {
    size_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)std::min<size_t>(std::max<size_t>(g, 1), 4096);
}

#define KCHK(...)                                          \
    do {                                                   \
        hipError_t e_ = (__VA_ARGS__);                     \
        if (e_ != hipSuccess) { status = DWF_EHIP; goto done; } \
    } while (0)

struct Work {
    std::vector<void*> bufs;
    double* hres = nullptr;
    ~Work() {
        std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
        for (void* p : bufs) (void)hipFree(p);
        if (hres) (void)hipHostFree(hres);
    }
    template <typename P> bool get(P** p, size_t bytes) {
        std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
        void* q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return false;
        bufs.push_back(q);
        *p = static_cast<P*>(q);
        return true;
    }
};

}  // namespace

int krylov_solve(const cpx<double>* U, const cpx<double>* b, cpx<double>* x, int Lx, int Ly, int Ls, double m,
                 double M5, int method, int ell, double tol, int maxit, dwf_solve_stats* stats, hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = (size_t)Lx * Ly * Ls * 2;   // complex entries of one 5-d field
    Work w;
    RedWork rw{};
    rw.nblk = kRedBlocks;
    rw.max_q = 4;
    rw.max_cols = 1;
    double* dres = nullptr;
    const int nv = (method == DWF_KRYLOV_BICGSTAB) ? 2 * (ell + 1) + 3 : 5;
    std::vector<cpx<double>*> v(nv, nullptr);
    if (!w.get(&rw.partial, sizeof(double) * rw.nblk * rw.max_q) || !w.get(&dres, sizeof(double) * 4))
        return DWF_EHIP;
    for (auto& p : v)
        if (!w.get(&p, sizeof(cpx<double>) * n)) return DWF_EHIP;
    {
        std::lock_guard<std::recursive_mutex> lk(runtime_mutex());
        if (hipHostMalloc((void**)&w.hres, sizeof(double) * 4, hipHostMallocDefault) != hipSuccess) return DWF_EHIP;
    }

    int status = DWF_OK;
    long long applies = 0;
    int iters = 0;
    double true_res = 0.0;
    auto D = [&](const cpx<double>* in, cpx<double>* out, double mass, bool dag) -> hipError_t {
        ++applies;
        return fine_dw<double>(U, in, out, nullptr, Lx, Ly, Ls, 1, mass, M5, dag, nullptr, 1, st);
    };
    auto dot = [&](const cpx<double>* a, const cpx<double>* c, zc* out) -> hipError_t {
        hipError_t e = cdot<double>(a, c, n, 1, dres, rw, st);
        if (e == hipSuccess) e = hipMemcpyAsync(w.hres, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        *out = zc(w.hres[0], w.hres[1]);
        return e;
    };
    auto nrm = [&](const cpx<double>* a, double* out) -> hipError_t {
        hipError_t e = norm2<double>(a, n, 1, dres, rw, st);
        if (e == hipSuccess) e = hipMemcpyAsync(w.hres, dres, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        *out = w.hres[0];
        return e;
    };
    auto axpy = [&](zc a, const cpx<double>* xx, cpx<double>* y) -> hipError_t {
        hipLaunchKernelGGL(k_axpy, dim3(ew_blocks(n)), dim3(kBlock), 0, st, cpx<double>{a.real(), a.imag()}, xx, y, n);
        return hipGetLastError();
    };
    auto xpay = [&](const cpx<double>* xx, zc a, cpx<double>* y) -> hipError_t {
        hipLaunchKernelGGL(k_xpay, dim3(ew_blocks(n)), dim3(kBlock), 0, st, xx, cpx<double>{a.real(), a.imag()}, y, n);
        return hipGetLastError();
    };

    if (method == DWF_KRYLOV_CGNR) {
        cpx<double>*r = v[0], *z = v[1], *p = v[2], *q = v[3];
        double bb = 0, rr = 0, zz = 0, qq = 0, zz_new = 0;
        KCHK(vzero<double>(x, n, st));
        KCHK(vconvert<double, double>(b, r, n, st));
        KCHK(nrm(b, &bb));
        rr = bb;
        KCHK(D(r, z, m, true));
        KCHK(vconvert<double, double>(z, p, n, st));
        KCHK(nrm(z, &zz));
        while (iters < maxit && rr > tol * tol * bb) {
            KCHK(D(p, q, m, false));
            KCHK(nrm(q, &qq));
            if (!(qq > 0.0) || !std::isfinite(qq)) { status = std::isfinite(qq) ? DWF_EBREAKDOWN : DWF_ENAN; goto done; }
            const double alpha = zz / qq;
            KCHK(axpy(alpha, p, x));
            KCHK(axpy(-alpha, q, r));
            KCHK(nrm(r, &rr));
            KCHK(D(r, z, m, true));
            KCHK(nrm(z, &zz_new));
            KCHK(xpay(z, zz_new / zz, p));
            zz = zz_new;
            ++iters;
        }
        if (!std::isfinite(rr)) status = DWF_ENAN;
    } else if (method == DWF_KRYLOV_BICGSTAB) {
        // v: u_0..u_ell, r_0..r_ell, shadow, right-hand side b', scratch
        cpx<double>** u = v.data();
        cpx<double>** r = v.data() + (ell + 1);
        cpx<double>* rt = v[2 * (ell + 1)];
        cpx<double>* bp = v[2 * (ell + 1) + 1];
        cpx<double>* tmp = v[2 * (ell + 1) + 2];
        auto A = [&](const cpx<double>* in, cpx<double>* out) -> hipError_t {
            hipError_t e = D(in, tmp, m, false);
            return e == hipSuccess ? D(tmp, out, 1.0, true) : e;
        };
        double bb = 0.0, rr = 0.0, bpbp = 0.0;
        KCHK(nrm(b, &bb));
        KCHK(D(b, bp, 1.0, true));                 // b' = D_PV^dagger b
        KCHK(nrm(bp, &bpbp));
        KCHK(vzero<double>(x, n, st));
        double tol_in = tol;
        bool first = true;
        while (true) {
            // (re)start: r_0 = b' - A x, shadow = r_0, u_0 = 0
            if (first) {
                KCHK(vconvert<double, double>(bp, r[0], n, st));
            } else {
                KCHK(A(x, r[1]));
                KCHK(vsub<double>(bp, r[1], r[0], n, st));
            }
            KCHK(vconvert<double, double>(r[0], rt, n, st));
            KCHK(vzero<double>(u[0], n, st));
            KCHK(nrm(r[0], &rr));
            zc rho0(1.0, 0.0), alpha(0.0, 0.0), omega(1.0, 0.0);
            while (iters < maxit && rr > tol_in * tol_in * bpbp) {
                rho0 = -omega * rho0;
                for (int j = 0; j < ell; ++j) {
                    zc rho1, gam;
                    KCHK(dot(rt, r[j], &rho1));
                    const zc beta = alpha * rho1 / rho0;
                    rho0 = rho1;
                    for (int i = 0; i <= j; ++i) KCHK(xpay(r[i], -beta, u[i]));
                    KCHK(A(u[j], u[j + 1]));
                    KCHK(dot(rt, u[j + 1], &gam));
                    if (!(std::abs(gam) > 0.0) || !std::isfinite(std::abs(gam))) {
                        status = std::isfinite(std::abs(gam)) ? DWF_EBREAKDOWN : DWF_ENAN;
                        goto done;
                    }
                    alpha = rho0 / gam;
                    for (int i = 0; i <= j; ++i) KCHK(axpy(-alpha, u[i + 1], r[i]));
                    KCHK(A(r[j], r[j + 1]));
                    KCHK(axpy(alpha, u[0], x));
                }
                // minimal-residual step: modified Gram-Schmidt on r_1..r_ell
                std::vector<zc> tau((size_t)(ell + 1) * (ell + 1)), gp(ell + 1), g(ell + 1), gpp(ell + 1);
                std::vector<double> sigma(ell + 1, 0.0);
                for (int j = 1; j <= ell; ++j) {
                    for (int i = 1; i < j; ++i) {
                        zc t;
                        KCHK(dot(r[i], r[j], &t));
                        t /= sigma[i];
                        tau[(size_t)i * (ell + 1) + j] = t;
                        KCHK(axpy(-t, r[i], r[j]));
                    }
                    KCHK(nrm(r[j], &sigma[j]));
                    if (!(sigma[j] > 0.0)) { status = DWF_EBREAKDOWN; goto done; }
                    zc t;
                    KCHK(dot(r[j], r[0], &t));
                    gp[j] = t / sigma[j];
                }
                g[ell] = gp[ell];
                omega = g[ell];
                for (int j = ell - 1; j >= 1; --j) {
                    zc s = 0.0;
                    for (int i = j + 1; i <= ell; ++i) s += tau[(size_t)j * (ell + 1) + i] * g[i];
                    g[j] = gp[j] - s;
                }
                for (int j = 1; j < ell; ++j) {
                    zc s = 0.0;
                    for (int i = j + 1; i < ell; ++i) s += tau[(size_t)j * (ell + 1) + i] * g[i + 1];
                    gpp[j] = g[j + 1] + s;
                }
                KCHK(axpy(g[1], r[0], x));
                KCHK(axpy(-gp[ell], r[ell], r[0]));
                KCHK(axpy(-g[ell], u[ell], u[0]));
                for (int j = 1; j < ell; ++j) {
                    KCHK(axpy(-g[j], u[j], u[0]));
                    KCHK(axpy(gpp[j], r[j], x));
                    KCHK(axpy(-gp[j], r[j], r[0]));
                }
                KCHK(nrm(r[0], &rr));
                if (!std::isfinite(rr)) { status = DWF_ENAN; goto done; }
                ++iters;
            }
            // true residual of D_DW x = b
            KCHK(D(x, tmp, m, false));
            KCHK(vsub<double>(b, tmp, r[1], n, st));
            KCHK(nrm(r[1], &rr));
            if (rr <= tol * tol * bb || iters >= maxit || tol_in < 1e-3 * tol) break;
            tol_in *= 0.1;
            first = false;
        }
    } else {
        return DWF_EINVAL;
    }
done:
    if (status == DWF_OK || status == DWF_NOT_CONVERGED) {
        double bb = 0.0, rr = 0.0;
        cpx<double>* tmp = v[nv - 1];
        cpx<double>* res = v[nv - 2];
        if (D(x, tmp, m, false) == hipSuccess && vsub<double>(b, tmp, res, n, st) == hipSuccess &&
            nrm(res, &rr) == hipSuccess && nrm(b, &bb) == hipSuccess) {
            --applies;   // the check is not part of the method's count
            true_res = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
            if (!(true_res <= tol)) status = std::isfinite(true_res) ? DWF_NOT_CONVERGED : DWF_ENAN;
        } else {
            status = DWF_EHIP;
        }
    }
    if (stats) {
        *stats = dwf_solve_stats{};
        stats->status = status;
        stats->fine_iters = iters;
        stats->fine_applies = applies;
        stats->true_rel_residual = true_res;
        stats->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // namespace dwf
