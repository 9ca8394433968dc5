// Layout and gauge utilities (bit-exact) and the fermion force.
#include "kernels.hpp"

// Gauge transforms must agree bit for bit with a reference that rounds every
// product and sum on its own: no contraction into fused multiply-adds here.
#pragma clang fp contract(off)

namespace dwf {

// out = gamma_5 R psi: slice s <- slice Ls-1-s, spin 1 negated (Sec. 2.1)
template <typename R>
__global__ void k_gamma5R(const spinor<R>* in, spinor<R>* out, int V, int Ls, long long total) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int site = (int)(t % V);
    const int s = (int)((t / V) % Ls);
    const long long col = t / ((long long)V * Ls);
    spinor<R> v = in[((size_t)col * Ls + (Ls - 1 - s)) * V + site];
    v.c1.re = -v.c1.re;
    v.c1.im = -v.c1.im;
    out[t] = v;
}

template <typename R>
hipError_t gamma5R(const cpx<R>* in, cpx<R>* out, int V, int Ls, int ncol, hipStream_t st) {
    const long long total = (long long)V * Ls * ncol;
    hipLaunchKernelGGL(k_gamma5R<R>, dim3(grid_for(total)), dim3(kBlock), 0, st,
                       reinterpret_cast<const spinor<R>*>(in), reinterpret_cast<spinor<R>*>(out), V, Ls, total);
    return hipGetLastError();
}
template hipError_t gamma5R<float>(const cpx<float>*, cpx<float>*, int, int, int, hipStream_t);
template hipError_t gamma5R<double>(const cpx<double>*, cpx<double>*, int, int, int, hipStream_t);

// complex product, each real product and sum rounded on its own (this file is
// compiled without floating-point contraction)
__device__ __forceinline__ cpx<double> mul_rn(cpx<double> a, cpx<double> b) {
    const double rr = a.re * b.re, ii = a.im * b.im;
    const double ri = a.re * b.im, ir = a.im * b.re;
    return {rr - ii, ri + ir};
}

__global__ void k_gauge_links(const cpx<double>* U, const cpx<double>* g, cpx<double>* Ug, int Lx, int Ly) {
    const int V = Lx * Ly;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * V) return;
    const int mu = t / V, site = t % V;
    const int x = site % Lx, y = site / Lx;
    const int nb = (mu == 0) ? y * Lx + ((x + 1 == Lx) ? 0 : x + 1) : ((y + 1 == Ly) ? 0 : y + 1) * Lx + x;
    const cpx<double> gn = {g[nb].re, -g[nb].im};
    Ug[t] = mul_rn(mul_rn(g[site], U[t]), gn);
}

__global__ void k_gauge_field(const cpx<double>* g, const cpx<double>* psi, cpx<double>* out, int V, long long total) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int site = (int)((t / 2) % V);
    out[t] = mul_rn(g[site], psi[t]);
}

hipError_t gauge_transform(const cpx<double>* U, const cpx<double>* g, const cpx<double>* psi,
                           cpx<double>* Ug, cpx<double>* psig, int Lx, int Ly, int Ls, int ncol,
                           hipStream_t st) {
    const int V = Lx * Ly;
    if (Ug) hipLaunchKernelGGL(k_gauge_links, dim3(grid_for(2LL * V)), dim3(kBlock), 0, st, U, g, Ug, Lx, Ly);
    if (psig) {
        const long long total = (long long)ncol * Ls * V * 2;
        hipLaunchKernelGGL(k_gauge_field, dim3(grid_for(total)), dim3(kBlock), 0, st, g, psi, psig, V, total);
    }
    return hipGetLastError();
}

// F_mu(x) = 2 Re sum [ i U Y(x)^dag (1-g_mu)/2 X(x+mu) - i U^* Y(x+mu)^dag (1+g_mu)/2 X(x) ]
//         = -2 Im( U t1 - U^* t2 )
__global__ void k_force(const cpx<double>* U, const spinor<double>* X, const spinor<double>* Y, double* F,
                        int Lx, int Ly, int Ls, int ncol) {
    const int V = Lx * Ly;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * V) return;
    const int mu = t / V, site = t % V;
    const int x = site % Lx, y = site / Lx;
    const int nb = (mu == 0) ? y * Lx + ((x + 1 == Lx) ? 0 : x + 1) : ((y + 1 == Ly) ? 0 : y + 1) * Lx + x;
    cpx<double> t1 = {0.0, 0.0}, t2 = {0.0, 0.0};
    for (int col = 0; col < ncol; ++col)
        for (int s = 0; s < Ls; ++s) {
            const size_t base = ((size_t)col * Ls + s) * V;
            const spinor<double> yx = Y[base + site], xn = X[base + nb];
            const spinor<double> yn = Y[base + nb], xx = X[base + site];
            cpx<double> pm, pp, ya, yb;
            if (mu == 0) {
                // (1 - s1)/2 X = (X0 - X1)/2 (1, -1);  (1 + s1)/2 X = (X0 + X1)/2 (1, 1)
                pm = 0.5 * (xn.c0 - xn.c1);
                ya = conj(yx.c0) - conj(yx.c1);
                pp = 0.5 * (xx.c0 + xx.c1);
                yb = conj(yn.c0) + conj(yn.c1);
            } else {
                // (1 - s2)/2 X = (X0 + i X1)/2 (1, -i);  (1 + s2)/2 X = (X0 - i X1)/2 (1, i)
                pm = 0.5 * (xn.c0 + mul_i(xn.c1));
                ya = conj(yx.c0) - mul_i(conj(yx.c1));
                pp = 0.5 * (xx.c0 - mul_i(xx.c1));
                yb = conj(yn.c0) + mul_i(conj(yn.c1));
            }
            t1 = t1 + cmul(ya, pm);
            t2 = t2 + cmul(yb, pp);
        }
    const cpx<double> u = U[t];
    const cpx<double> a = cmul(u, t1) - cmul(conj(u), t2);
    F[t] = -2.0 * a.im;
}

// U_mu(x) = exp(i theta_mu(x)) = cos theta + i sin theta (the compact U(1) links)
__global__ void k_links_from_theta(const double* theta, cpx<double>* U, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double sv, cv;
    sincos(theta[t], &sv, &cv);
    U[t] = {cv, sv};
}

hipError_t links_from_theta(const double* theta, cpx<double>* U, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_links_from_theta, dim3(grid_for(n)), dim3(kBlock), 0, st, theta, U, n);
    return hipGetLastError();
}

// Scalar read-back without a copy engine or a stream synchronisation: one
// wavefront copies the listed device words into host-coherent memory and then
// stores the sequence number with release ordering at system scope, so that a
// host that reads the number also reads the words.
__global__ void __launch_bounds__(64) k_publish(PublishArgs a) {
#pragma unroll
    for (int k = 0; k < kPublishItems; ++k)
        for (int i = threadIdx.x; i < a.words[k]; i += 64) a.dst[k][i] = a.src[k][i];
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned v = *a.ctr + 1u;
        *a.ctr = v;
        __hip_atomic_store(a.seq, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

hipError_t publish_to_host(const PublishArgs& a, hipStream_t st) {
    if (!a.seq || !a.ctr) return hipErrorInvalidValue;
    for (int k = 0; k < kPublishItems; ++k)
        if (a.words[k] < 0 || (a.words[k] > 0 && (!a.src[k] || !a.dst[k]))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t force(const cpx<double>* U, const cpx<double>* X, const cpx<double>* Y, double* F,
                 int Lx, int Ly, int Ls, int ncol, hipStream_t st) {
    const int V = Lx * Ly;
    hipLaunchKernelGGL(k_force, dim3(grid_for(2LL * V)), dim3(kBlock), 0, st, U,
                       reinterpret_cast<const spinor<double>*>(X), reinterpret_cast<const spinor<double>*>(Y), F,
                       Lx, Ly, Ls, ncol);
    return hipGetLastError();
}

}  // namespace dwf
