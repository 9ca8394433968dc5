// Coarsest-level deflation (Sec. 3, Table 1: the coarsest level deflated
// with 128 of its lowest eigenvectors, making a four-level algorithm).
//
// The coarsest solve is CGNR on H = A^dag A with A = hat-D_PV^dag hat-D_DW.
// Setup: the nev lowest eigenpairs of H come from a thick-restart Lanczos
// process (Wu & Simon 2000) run on p(H) = T_d((2H - a - b)/(b - a)), a
// Chebyshev polynomial that is bounded by 1 on the unwanted part [a, b] of
// the spectrum and grows fast below a, so that the lowest eigenvalues of H
// become the best separated largest ones of p(H).  b comes from a power
// iteration; a starts high and is lowered to the largest kept Ritz value of
// H, an upper bound of lambda_nk.  Every cycle ends with a Rayleigh-Ritz step
// for H itself on the kept vectors, which gives the eigenpairs and their true
// residuals.  Full reorthogonalisation (two Gram-Schmidt passes) and the
// dense steps use rocBLAS / rocSOLVER; H is applied by the coarse kernels.
// Solve: every coarsest CGNR starts from the deflated guess
// e0 = V Lambda^{-1} V^dag (A^dag r), which removes the slowest directions;
// the stopping rule stays relative to |A^dag r| as without deflation.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mg.hpp"

namespace dwf {

namespace {

#define HIPCHK(...)                                   \
    do {                                              \
        hipError_t e_ = (__VA_ARGS__);                \
        if (e_ != hipSuccess) return DWF_EHIP;        \
    } while (0)
#define RBCHK(...)                                                    \
    do {                                                              \
        rocblas_status s_ = (__VA_ARGS__);                            \
        if (s_ != rocblas_status_success) return DWF_EHIP;            \
    } while (0)

// SplitMix64 (Steele, Lea, Flood 2014) and Box-Muller: Gaussian entries
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__global__ void k_randn(cpx<double>* v, size_t n, uint64_t seed) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64(seed ^ (2 * i)), b = splitmix64(seed ^ (2 * i + 1));
        const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
        const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
        const double r = sqrt(-2.0 * log(u1)), t = 6.283185307179586 * u2;
        v[i] = {r * cos(t), r * sin(t)};
    }
}

// y2 = alpha (h1 - c y1) + beta y0
__global__ void k_cheb(cpx<double>* y2, const cpx<double>* h1, const cpx<double>* y1, const cpx<double>* y0,
                       size_t n, double alpha, double c, double beta) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const cpx<double> a = h1[i], b = y1[i];
        cpx<double> r = {alpha * (a.re - c * b.re), alpha * (a.im - c * b.im)};
        if (y0) { r.re += beta * y0[i].re; r.im += beta * y0[i].im; }
        y2[i] = r;
    }
}

// per column j of an n x ncol block: out_j = w_j - theta_j v_j
__global__ void k_resid(cpx<double>* out, const cpx<double>* w, const cpx<double>* v, const double* theta, size_t n,
                        int ncol) {
    const size_t total = n * ncol;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const double th = theta[i / n];
        out[i] = {w[i].re - th * v[i].re, w[i].im - th * v[i].im};
    }
}

// ---- deflated start of a coarsest solve, e0 = V Lambda^{-1} V^dag z (per column of z)
// Column tiles of the projection kernels: each wave reads an element of V once
// for up to kDeflTile right-hand sides.
constexpr int kDeflTile = 8;

// part[c][i][b] = sum over block b's slice of conj(V_i) z_c, for the columns
// c0 .. c0 + nc of the tile (blockIdx.y); wave w of the block takes i = w, w + 4, ...
template <int NC>
__global__ __launch_bounds__(256) void k_defl_dots(const cpx<double>* __restrict__ V, const cpx<double>* __restrict__ z,
                                                   double* __restrict__ part, size_t n, int nev, int ncol) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.x, c0 = blockIdx.y * NC;
    const int nc = min(NC, ncol - c0);
    const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const size_t lo = (size_t)b * chunk, hi = min(n, lo + chunk);
    for (int i = wave; i < nev; i += 4) {
        double ar[NC], ai[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) ar[c] = ai[c] = 0.0;
        const cpx<double>* vi = V + (size_t)i * n;
        for (size_t e = lo + lane; e < hi; e += 64) {
            const cpx<double> v = vi[e];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (c < nc) {
                    const cpx<double> w = z[(size_t)(c0 + c) * n + e];
                    ar[c] += v.re * w.re + v.im * w.im;
                    ai[c] += v.re * w.im - v.im * w.re;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double r = ar[c], m = ai[c];
            for (int off = 32; off > 0; off >>= 1) {
                r += __shfl_down(r, off);
                m += __shfl_down(m, off);
            }
            if (lane == 0 && c < nc) {
                const size_t o = (((size_t)(c0 + c) * nev + i) * gridDim.x + b) * 2;
                part[o] = r;
                part[o + 1] = m;
            }
        }
    }
}

// C[c][i] = (sum_b part[c][i][b]) / lambda_i, in block order
__global__ void k_defl_coef(const double* __restrict__ part, const double* __restrict__ lam, cpx<double>* C, int nev,
                            int ncol, int nblk) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nev * ncol) return;
    const int i = t % nev;
    const double* p = part + (size_t)t * nblk * 2;
    double r = 0.0, m = 0.0;
    for (int b = 0; b < nblk; ++b) {
        r += p[2 * b];
        m += p[2 * b + 1];
    }
    C[t] = {r / lam[i], m / lam[i]};
}

// x_c[e] = sum_i V_i[e] C[c][i] for the columns of the tile (blockIdx.y)
template <int NC>
__global__ __launch_bounds__(256) void k_defl_expand(const cpx<double>* __restrict__ V, const cpx<double>* __restrict__ C,
                                                     cpx<double>* __restrict__ x, size_t n, int nev, int ncol) {
    const int c0 = blockIdx.y * NC;
    const int nc = min(NC, ncol - c0);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double ar[NC], ai[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) ar[c] = ai[c] = 0.0;
        for (int i = 0; i < nev; ++i) {
            const cpx<double> v = V[(size_t)i * n + e];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (c < nc) {
                    const cpx<double> k = C[(size_t)(c0 + c) * nev + i];
                    ar[c] += v.re * k.re - v.im * k.im;
                    ai[c] += v.re * k.im + v.im * k.re;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < nc) x[(size_t)(c0 + c) * n + e] = {ar[c], ai[c]};
    }
}

inline unsigned grid1(size_t n) {
    size_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)std::min<size_t>(std::max<size_t>(g, 1), 8192);
}

}  // namespace

// reference norm for the deflated CGNR: s.zz0 = ref[c], done re-evaluated
__global__ void k_cg_set_ref(CgScal* s, const double* ref, int ncol) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    CgScal v = s[c];
    v.zz0 = ref[c];
    if (v.done != 4) v.done = (v.zz <= v.tol2 * v.zz0) ? 1 : 0;
    s[c] = v;
}

int Hierarchy::deflation_setup(hipStream_t st) {
    const int nev = prm.coarsest_nev;
    if (nev <= 0) return DWF_OK;
    const int l = (int)levels.size() - 1;
    const Level& L = levels[l];
    if (L.vec_prec != P_F64) return DWF_EUNSUPPORTED;
    const size_t n = L.vec_elems();
    if ((size_t)nev >= n) return DWF_EINVAL;
    // nk Ritz vectors are kept at a thick restart, the Lanczos basis holds m (+1)
    int nk = 0, m = 0;
    deflation_dims(nev, n, nk, m);
    const bool verbose = std::getenv("DWF_VERBOSE") != nullptr;
    if (!blas_) {
        if (rocblas_create_handle(&blas_) != rocblas_status_success) return DWF_EHIP;
    }
    RBCHK(rocblas_set_stream(blas_, st));
    RBCHK(rocblas_set_pointer_mode(blas_, rocblas_pointer_mode_host));
    // the temporaries were laid out with the hierarchy (over the solve buffers)
    DeflTmp& D = dtmp_;
    if (D.nk != nk || D.m != m || !D.Vb) return DWF_EINVAL;
    using zc = std::complex<double>;
    const size_t nkb = (size_t)nk * n;
    cpx<double>* Vb = D.Vb;
    cpx<double> *Ub = D.Ub, *HUb = D.HUb, *Xb = D.Xb, *Wb = D.Wb;
    cpx<double> *P0 = D.P0, *P1 = D.P1, *P2 = D.P2, *Hh = D.Hh, *t1 = D.t1, *t2 = D.t2;
    cpx<double> *G = D.G, *Ysd = D.Ysd, *cdev = D.cdev;
    double *lam = D.lam, *E = D.E, *nrm = D.nrm;
    rocblas_int* info = reinterpret_cast<rocblas_int*>(D.info);
    const size_t zb = sizeof(cpx<double>);
    auto cleanup = [&]() { (void)hipStreamSynchronize(st); };

    int status = DWF_OK;
    const auto t_start = std::chrono::steady_clock::now();
    auto secs = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0}, mone = {-1.0, 0.0};
    auto rb = [](cpx<double>* p) { return reinterpret_cast<rocblas_double_complex*>(p); };
    long long matvecs = 0;
    auto applyH = [&](const cpx<double>* in, cpx<double>* out, cpx<double>* s1, cpx<double>* s2, int ncol) -> int {
        HIPCHK(apply_A<double>(l, in, s1, s2, ncol, st));
        HIPCHK(apply_Adag<double>(l, s1, out, s2, ncol, st));
        matvecs += ncol;
        return DWF_OK;
    };
    auto col = [&](int j) { return Vb + (size_t)j * n; };
    auto nrm2 = [&](const cpx<double>* v, double* out) -> int {
        RBCHK(rocblas_dznrm2(blas_, (rocblas_int)n, reinterpret_cast<const rocblas_double_complex*>(v), 1, out));
        return DWF_OK;
    };
    // w <- w - V[:, 0..k) (V^dag w), twice (classical Gram-Schmidt with one
    // reorthogonalisation); the projections are added into c (host)
    auto orth = [&](cpx<double>* w, int k, zc* c) -> int {
        for (int pass = 0; pass < 2; ++pass) {
            RBCHK(rocblas_zgemv(blas_, rocblas_operation_conjugate_transpose, (rocblas_int)n, k, &one, rb(Vb),
                                (rocblas_int)n, rb(w), 1, &zero, rb(cdev), 1));
            RBCHK(rocblas_zgemv(blas_, rocblas_operation_none, (rocblas_int)n, k, &mone, rb(Vb), (rocblas_int)n,
                                rb(cdev), 1, &one, rb(w), 1));
            if (c) {
                std::vector<zc> h(k);
                HIPCHK(hipMemcpyAsync(h.data(), cdev, zb * k, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                for (int i = 0; i < k; ++i) c[i] += h[i];
            }
        }
        return DWF_OK;
    };
    // unit vector at column k of the basis, random and orthogonal to columns 0..k
    uint64_t seed = 0x5eedull + (uint64_t)l;
    auto random_col = [&](int k) -> int {
        hipLaunchKernelGGL(k_randn, dim3(grid1(n)), dim3(kBlock), 0, st, col(k), n, seed++);
        if (k > 0) if (int e = orth(col(k), k, nullptr)) return e;
        double nr = 0.0;
        if (int e = nrm2(col(k), &nr)) return e;
        RBCHK(rocblas_zdscal(blas_, (rocblas_int)n, &(nr = 1.0 / nr), rb(col(k)), 1));
        return DWF_OK;
    };

    do {
        // ---- upper bound of the spectrum of H: power iteration, with a margin
        double lam_max = 0.0;
        if ((status = random_col(0))) break;
        HIPCHK(vconvert<double, double>(col(0), P0, n, st));
        for (int it = 0; it < 40; ++it) {
            if ((status = applyH(P0, P1, t1, t2, 1))) break;
            double a2 = 0.0, b2 = 0.0;
            if ((status = nrm2(P1, &a2)) || (status = nrm2(P0, &b2))) break;
            lam_max = a2 / b2;
            hipLaunchKernelGGL(k_cheb, dim3(grid1(n)), dim3(kBlock), 0, st, P0, P1, P1, (const cpx<double>*)nullptr, n,
                               1.0 / a2, 0.0, 0.0);
        }
        if (status) break;
        const double b = 1.15 * lam_max;
        // lower edge of the damped interval [a, b]; the polynomial T_d((2H - a - b)/(b - a))
        // is at most 1 in modulus on [a, b] and grows monotonically below a
        double a = 1e-4 * b;
        bool bounded = false;
        int d = 0;
        auto pick_degree = [&]() {
            if (prm.eig_degree > 0) { d = prm.eig_degree; }
            else {
                // target p(0) = cosh(2): enough separation, moderate dynamic range
                const double s0 = std::acosh(1.0 + 2.0 * a / (b - a));
                d = (int)std::ceil(2.0 / std::max(s0, 1e-12));
            }
            d = std::max(2, std::min(d, 4096));
            d += d & 1;   // even: p > 1 everywhere below a
        };
        pick_degree();
        std::vector<zc> T((size_t)(m + 1) * (m + 1));
        auto Tij = [&](int i, int j) -> zc& { return T[(size_t)i + (size_t)j * (m + 1)]; };
        int j0 = 0;          // first Lanczos step of the cycle
        int cycle = 0, steps = 0;
        double worst = 1e300;
        bool done = false;
        std::vector<double> th(m), lh(nk), rr(nk);
        std::vector<zc> Y((size_t)m * m), Ysel((size_t)m * nk);
        while (!done && cycle < prm.eig_maxit && status == DWF_OK) {
            ++cycle;
            // ---- Lanczos steps j0 .. m-1 on p(H)
            const double e = 0.5 * (b - a), c = 0.5 * (b + a);
            bool exhausted = false;
            for (int j = j0; j < m; ++j) {
                // w = p(H) v_j by the three-term Chebyshev recurrence
                cpx<double>* y0 = P0; cpx<double>* y1 = P1; cpx<double>* y2 = P2;
                HIPCHK(vconvert<double, double>(col(j), y0, n, st));
                if ((status = applyH(y0, Hh, t1, t2, 1))) break;
                hipLaunchKernelGGL(k_cheb, dim3(grid1(n)), dim3(kBlock), 0, st, y1, Hh, y0, (const cpx<double>*)nullptr,
                                   n, 1.0 / e, c, 0.0);
                for (int k = 2; k <= d && status == DWF_OK; ++k) {
                    if ((status = applyH(y1, Hh, t1, t2, 1))) break;
                    hipLaunchKernelGGL(k_cheb, dim3(grid1(n)), dim3(kBlock), 0, st, y2, Hh, y1, y0, n, 2.0 / e, c, -1.0);
                    cpx<double>* tmp = y0; y0 = y1; y1 = y2; y2 = tmp;
                }
                if (status) break;
                double w0 = 0.0, beta = 0.0;
                if ((status = nrm2(y1, &w0))) break;
                std::vector<zc> cj(j + 1, zc(0.0, 0.0));
                if ((status = orth(y1, j + 1, cj.data()))) break;
                if ((status = nrm2(y1, &beta))) break;
                for (int i = 0; i <= j; ++i) Tij(i, j) = cj[i];
                ++steps;
                if (j + 1 == (int)n) { Tij(j + 1, j) = 0.0; exhausted = true; break; }
                if (beta <= 1e-12 * w0) {        // invariant subspace: continue with a fresh direction
                    Tij(j + 1, j) = 0.0;
                    if ((status = random_col(j + 1))) break;
                } else {
                    Tij(j + 1, j) = beta;
                    HIPCHK(vconvert<double, double>(y1, col(j + 1), n, st));
                    double inv = 1.0 / beta;
                    RBCHK(rocblas_zdscal(blas_, (rocblas_int)n, &inv, rb(col(j + 1)), 1));
                }
            }
            if (status) break;
            // ---- Rayleigh-Ritz for p(H) on the m-dimensional basis
            {
                std::vector<zc> Ts((size_t)m * m);
                for (int jj = 0; jj < m; ++jj)
                    for (int i = 0; i < m; ++i)
                        Ts[(size_t)i + (size_t)jj * m] = 0.5 * (Tij(i, jj) + std::conj(Tij(jj, i)));
                HIPCHK(hipMemcpyAsync(G, Ts.data(), zb * m * m, hipMemcpyHostToDevice, st));
                RBCHK(rocsolver_zheevd(blas_, rocblas_evect_original, rocblas_fill_upper, m, rb(G), m, lam, E, info));
                HIPCHK(hipMemcpyAsync(Y.data(), G, zb * m * m, hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemcpyAsync(th.data(), lam, sizeof(double) * m, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
            }
            // the nk largest Ritz values of p(H) belong to the lowest eigenvalues of H
            for (int i = 0; i < nk; ++i)
                for (int r = 0; r < m; ++r) Ysel[(size_t)r + (size_t)i * m] = Y[(size_t)r + (size_t)(m - 1 - i) * m];
            const zc beta_m = exhausted ? zc(0.0) : Tij(m, m - 1);
            int above = 0;
            for (int i = 0; i < nk; ++i)
                if (th[m - 1 - i] > 1.0) ++above;
            HIPCHK(hipMemcpyAsync(Ysd, Ysel.data(), zb * m * nk, hipMemcpyHostToDevice, st));
            RBCHK(rocblas_zgemm(blas_, rocblas_operation_none, rocblas_operation_none, (rocblas_int)n, nk, m, &one,
                                rb(Vb), (rocblas_int)n, rb(Ysd), m, &zero, rb(Ub), (rocblas_int)n));
            // ---- Rayleigh-Ritz for H on span(U): eigenpairs, residuals, convergence
            if ((status = applyH(Ub, HUb, Xb, Wb, nk))) break;
            RBCHK(rocblas_zgemm(blas_, rocblas_operation_conjugate_transpose, rocblas_operation_none, nk, nk,
                                (rocblas_int)n, &one, rb(Ub), (rocblas_int)n, rb(HUb), (rocblas_int)n, &zero, rb(G), nk));
            RBCHK(rocsolver_zheevd(blas_, rocblas_evect_original, rocblas_fill_upper, nk, rb(G), nk, lam, E, info));
            RBCHK(rocblas_zgemm(blas_, rocblas_operation_none, rocblas_operation_none, (rocblas_int)n, nk, nk, &one,
                                rb(Ub), (rocblas_int)n, rb(G), nk, &zero, rb(Xb), (rocblas_int)n));
            RBCHK(rocblas_zgemm(blas_, rocblas_operation_none, rocblas_operation_none, (rocblas_int)n, nk, nk, &one,
                                rb(HUb), (rocblas_int)n, rb(G), nk, &zero, rb(Wb), (rocblas_int)n));
            hipLaunchKernelGGL(k_resid, dim3(grid1(n * nk)), dim3(kBlock), 0, st, Wb, Wb, Xb, lam, n, nk);
            HIPCHK(norm2<double>(Wb, n, nk, nrm, rw_, st));
            HIPCHK(hipMemcpyAsync(lh.data(), lam, sizeof(double) * nk, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(rr.data(), nrm, sizeof(double) * nk, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            worst = 0.0;
            int conv = 0;
            for (int i = 0; i < nev; ++i) {
                const double r = std::sqrt(rr[i]) / std::max(lh[i], 1e-300);
                worst = std::max(worst, r);
                if (r <= prm.eig_tol) ++conv;
            }
            // converged pairs count only when the nev largest p-Ritz values exceed 1: then they
            // come from the monotone branch below a and are the lowest eigenvalues seen
            int above_nev = 0;
            for (int i = 0; i < nev; ++i)
                if (th[m - 1 - i] > 1.0) ++above_nev;
            done = (conv == nev) && (above_nev == nev);
            if (verbose)
                std::fprintf(stderr, "[dwfmg] lanczos cycle %d: a %.3e b %.3e degree %d steps %d H-applies %lld | "
                             "lambda[0] %.4e lambda[nev-1] %.4e lambda[nk-1] %.4e | p-Ritz above 1: %d/%d | "
                             "worst %.2e converged %d/%d (%.2f s)\n", cycle, a, b, d, steps, matvecs, lh[0],
                             lh[nev - 1], lh[nk - 1], above, nk, worst, conv, nev, secs());
            if (done) break;
            // ---- next cycle: adapt the damped interval, or thick restart
            const double a_new = lh[nk - 1];      // nk-th Ritz value of H: an upper bound of lambda_nk
            const bool raise = !bounded && above < nk && a < 0.9 * b;
            if (raise || a_new < 0.25 * a) {
                // fewer than nk eigenvalues below a were seen (a too low), or a far too high:
                // move a, change the polynomial and restart from the sum of the Ritz vectors.
                // Once a comes from the bound it is never raised again.
                if (raise) {
                    a = std::min(8.0 * a, 0.9 * b);
                } else {
                    a = a_new;
                    bounded = true;
                }
                pick_degree();
                std::vector<zc> ones(nk, zc(1.0, 0.0));
                HIPCHK(hipMemcpyAsync(cdev, ones.data(), zb * nk, hipMemcpyHostToDevice, st));
                RBCHK(rocblas_zgemv(blas_, rocblas_operation_none, (rocblas_int)n, nk, &one, rb(Xb), (rocblas_int)n,
                                    rb(cdev), 1, &zero, rb(col(0)), 1));
                double nr = 0.0;
                if ((status = nrm2(col(0), &nr))) break;
                nr = 1.0 / nr;
                RBCHK(rocblas_zdscal(blas_, (rocblas_int)n, &nr, rb(col(0)), 1));
                std::fill(T.begin(), T.end(), zc(0.0));
                j0 = 0;
                continue;
            }
            // thick restart: basis = [kept p-Ritz vectors, v_m], projected matrix = diag + arrow
            HIPCHK(hipMemcpyAsync(col(0), Ub, zb * nkb, hipMemcpyDeviceToDevice, st));
            std::fill(T.begin(), T.end(), zc(0.0));
            for (int i = 0; i < nk; ++i) Tij(i, i) = th[m - 1 - i];
            if (std::abs(beta_m) > 0.0) {
                HIPCHK(hipMemcpyAsync(col(nk), col(m), zb * n, hipMemcpyDeviceToDevice, st));
                for (int i = 0; i < nk; ++i) {
                    const zc v = beta_m * Ysel[(size_t)(m - 1) + (size_t)i * m];
                    Tij(nk, i) = v;
                    Tij(i, nk) = std::conj(v);
                }
            } else if ((status = random_col(nk))) {
                break;
            }
            j0 = nk;
        }
        if (status) break;
        eig_iters_ = steps;
        eig_worst_ = worst;
        // keep the nev lowest eigenpairs of H (columns 0..nev of X, ascending)
        if (!def_V_ || !def_lam_ || !def_C_ || !def_part_) { status = DWF_EINVAL; break; }
        HIPCHK(hipMemcpyAsync(def_V_, Xb, zb * n * nev, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(def_lam_, lam, sizeof(double) * nev, hipMemcpyDeviceToDevice, st));
        def_lam_host_.assign(lh.begin(), lh.begin() + nev);
        HIPCHK(hipStreamSynchronize(st));
        def_nev_ = nev;
        if (verbose)
            std::fprintf(stderr, "[dwfmg] deflation space: %d vectors, %d Lanczos steps, %lld H applications, "
                         "%.2f s\n", nev, steps, matvecs, secs());
    } while (false);
    cleanup();
    return status;
}

// e0 = V Lambda^{-1} V^dag z for ncol columns of z (n each), written to x
int Hierarchy::deflate_guess(int l, const cpx<double>* z, cpx<double>* x, int ncol, hipStream_t st) {
    const size_t n = levels[l].vec_elems();
    const int nev = def_nev_;
    if (ncol > max_ncol_) return DWF_EINVAL;
    const dim3 gd(kDeflBlocks, (ncol + kDeflTile - 1) / kDeflTile);
    hipLaunchKernelGGL(k_defl_dots<kDeflTile>, gd, dim3(256), 0, st, def_V_, z, def_part_, n, nev, ncol);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_defl_coef, dim3((nev * ncol + 255) / 256), dim3(256), 0, st, def_part_, def_lam_, def_C_, nev,
                       ncol, kDeflBlocks);
    HIPCHK(hipGetLastError());
    const dim3 ge(grid1(n), (ncol + kDeflTile - 1) / kDeflTile);
    hipLaunchKernelGGL(k_defl_expand<kDeflTile>, ge, dim3(kBlock), 0, st, def_V_, def_C_, x, n, nev, ncol);
    HIPCHK(hipGetLastError());
    return DWF_OK;
}

hipError_t cg_set_ref(CgScal* s, const double* ref, int ncol, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_set_ref, dim3((ncol + 63) / 64), dim3(64), 0, st, s, ref, ncol);
    return hipGetLastError();
}

void Hierarchy::destroy_blas() {
    if (blas_) (void)rocblas_destroy_handle(blas_);
    blas_ = nullptr;
}

}  // namespace dwf
