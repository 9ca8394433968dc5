// Coarse-level operator: the Galerkin kernel hat-D_W = P^dagger D_W P in
// stencil form (Sec. 2.3) and the coarse domain-wall operator of
// eq. coarsenDW built on it:
//   hat-D_DW(m) psi_s = (hat-D_W(M5) + 1) psi_s + hatP_- psi_{s+1} + hatP_+ psi_{s-1}
// with hatP_pm = (1 pm sigma_3)/2 and the -m corners, and
//   hat-D_W psi(x) = X(x) psi(x) + sum_h Y_h(x) psi(x + h)   (X includes M5 via a shift).
// The adjoint uses sigma_3-hermiticity of the Galerkin kernel
// (gamma_5 P = P sigma_3): hat-D_W^dagger = sigma_3 hat-D_W sigma_3.
//
// VALU kernel: one wavefront per (coarse site, column).  The five neighbour
// vectors of all coarse slices are staged in LDS (converted to the arithmetic
// type, sigma_3 applied for the adjoint); lane i owns output row i and a
// stride of the 5n inner index, reading links blk[k][i] that are contiguous
// across lanes.  Each link element is read once per pass of eight coarse
// slices (once per apply for L-hat_s <= 8) and used for every slice of it.  Links may be stored in FP64, FP32, BF16 or FP16; the latter
// three are multiplied in FP32.
#include "kernels.hpp"

namespace dwf {

template <typename L, typename T, int N, bool DAG, bool WIL>
__global__ void __launch_bounds__(256)
coarse_kernel(const L* __restrict__ links, const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
              const int* __restrict__ skip, int skip_stride, int Lx, int Ly, int Ls, int nsites,
              typename acc_of<L>::type cdiag, typename acc_of<L>::type mwrap) {
    using A = typename acc_of<L>::type;
    constexpr int P = (N <= 64) ? (64 / N) : 1;   // partitions of the inner index
    constexpr int MAXS = 8;                       // slices accumulated per pass
    constexpr int H = N / 2;
    extern __shared__ unsigned char smem_raw[];
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int site = (int)xcd_block(blockIdx.x, gridDim.x) * wpb + wave;
    const int col = blockIdx.y;
    // per wave: the five staged neighbour vectors; the partition sums of a pass (P > 1)
    // follow them, or with a single pass overwrite them
    cpx<A>* my = reinterpret_cast<cpx<A>*>(smem_raw) + (size_t)wave * coarse_lds_per_wave(N, Ls);
    cpx<A>* scr = (Ls <= MAXS) ? my : my + (size_t)5 * N * Ls;
    const bool valid = (site < nsites) && !(skip && skip[(size_t)col * skip_stride]);

    int nb[5] = {0, 0, 0, 0, 0};
    const cpx<T>* src = in + (size_t)col * Ls * nsites * N;
    cpx<T>* dst = out + (size_t)col * Ls * nsites * N;
    if (valid) {
        const int x = site % Lx, y = site / Lx;
        const int xp = (x + 1 == Lx) ? 0 : x + 1, xm = (x == 0) ? Lx - 1 : x - 1;
        const int yp = (y + 1 == Ly) ? 0 : y + 1, ym = (y == 0) ? Ly - 1 : y - 1;
        nb[0] = site; nb[1] = y * Lx + xp; nb[2] = y * Lx + xm; nb[3] = yp * Lx + x; nb[4] = ym * Lx + x;
        for (int e = lane; e < 5 * Ls * N; e += 64) {
            const int d = e / (Ls * N), rem = e - d * Ls * N;
            const int s = rem / N, k = rem - s * N;
            cpx<T> v = src[((size_t)s * nsites + nb[d]) * N + k];
            A re = (A)v.re, im = (A)v.im;
            if (DAG && k >= H) { re = -re; im = -im; }
            my[e] = {re, im};
        }
    }
    __syncthreads();

    const int i = lane % N;
    const int part = lane / N;
    const L* lk = links + (size_t)site * 5 * N * N;
    // slices in passes of MAXS (the accumulators stay in registers); every wave
    // takes every pass, so the barriers are uniform
    for (int s0 = 0; s0 < Ls; s0 += MAXS) {
        cpx<A> acc[MAXS];
#pragma unroll
        for (int s = 0; s < MAXS; ++s) acc[s] = {A(0), A(0)};
        if (valid && part < P) {
            for (int kk = part; kk < 5 * N; kk += P) {
                const int d = kk / N, k = kk - d * N;
                const cpx<A> l = load_link(lk, (size_t)kk * N + i);
                const cpx<A>* pv = my + (size_t)d * Ls * N + (size_t)s0 * N + k;
#pragma unroll
                for (int s = 0; s < MAXS; ++s)
                    if (s0 + s < Ls) cfma(acc[s], l, pv[(size_t)s * N]);
            }
        }
        // partition sums in a fixed order
        if (P > 1) {
            if (Ls <= MAXS) __syncthreads();   // (they overwrite the staged vectors)
            if (valid && part < P) {
#pragma unroll
                for (int s = 0; s < MAXS; ++s)
                    if (s0 + s < Ls) scr[(size_t)s * 64 + part * N + i] = acc[s];
            }
            __syncthreads();
        }
        if (valid && part == 0) {
#pragma unroll
            for (int s1 = 0; s1 < MAXS; ++s1) {
                const int s = s0 + s1;
                if (s >= Ls) break;
                cpx<A> v = {A(0), A(0)};
                if (P > 1) {
                    for (int p = 0; p < P; ++p) v = v + scr[(size_t)s1 * 64 + p * N + i];
                } else {
                    v = acc[s1];
                }
                if (DAG && i >= H) { v.re = -v.re; v.im = -v.im; }
                const cpx<T> c = src[((size_t)s * nsites + site) * N + i];
                v.re += cdiag * (A)c.re;
                v.im += cdiag * (A)c.im;
                if (!WIL) {
                    const bool minus = (i >= H);
                    // non-adjoint: hatP_- psi_{s+1} + hatP_+ psi_{s-1}; adjoint swaps
                    const bool from_up = DAG ? !minus : minus;
                    int so;
                    A f = A(1);
                    if (from_up) {
                        so = s + 1;
                        if (so == Ls) { so = 0; f = mwrap; }
                    } else {
                        so = s - 1;
                        if (so < 0) { so = Ls - 1; f = mwrap; }
                    }
                    const cpx<T> h = src[((size_t)so * nsites + site) * N + i];
                    v.re += f * (A)h.re;
                    v.im += f * (A)h.im;
                }
                dst[((size_t)s * nsites + site) * N + i] = {(T)v.re, (T)v.im};
            }
        }
        if (P > 1) __syncthreads();   // scr is rewritten by the next pass
    }
}

namespace {

template <typename L, typename T, int N>
hipError_t launch_n(const void* links, const cpx<T>* in, cpx<T>* out, const CoarseGeom& g, int ncol,
                    double m, double M5, bool dagger, bool wil, double wmass, const int* skip, int sks, hipStream_t st) {
    using A = typename acc_of<L>::type;
    const int nsites = g.Lx * g.Ly;
    size_t per_wave_bytes = (size_t)coarse_lds_per_wave(N, g.Ls) * sizeof(cpx<A>);
    int wpb = 4;
    while (wpb > 1 && per_wave_bytes * wpb > 64 * 1024) wpb >>= 1;
    if (per_wave_bytes * wpb > 160 * 1024) return hipErrorInvalidValue;
    dim3 grid((nsites + wpb - 1) / wpb, ncol), block(64 * wpb);
    const size_t shm = per_wave_bytes * wpb;
    const L* lk = reinterpret_cast<const L*>(links);
    const A cd = wil ? (A)wmass : (A)(M5 + 1.0);
    const A mw = (A)(-m);
    if (wil) {
        if (dagger) hipLaunchKernelGGL((coarse_kernel<L, T, N, true, true>), grid, block, shm, st, lk, in, out, skip, sks, g.Lx, g.Ly, g.Ls, nsites, cd, mw);
        else        hipLaunchKernelGGL((coarse_kernel<L, T, N, false, true>), grid, block, shm, st, lk, in, out, skip, sks, g.Lx, g.Ly, g.Ls, nsites, cd, mw);
    } else {
        if (dagger) hipLaunchKernelGGL((coarse_kernel<L, T, N, true, false>), grid, block, shm, st, lk, in, out, skip, sks, g.Lx, g.Ly, g.Ls, nsites, cd, mw);
        else        hipLaunchKernelGGL((coarse_kernel<L, T, N, false, false>), grid, block, shm, st, lk, in, out, skip, sks, g.Lx, g.Ly, g.Ls, nsites, cd, mw);
    }
    return hipGetLastError();
}

template <typename L, typename T>
hipError_t launch_l(const void* links, const cpx<T>* in, cpx<T>* out, const CoarseGeom& g, int ncol,
                    double m, double M5, bool dagger, bool wil, double wmass, const int* skip, int sks, hipStream_t st) {
    switch (g.n) {
        case 4:  return launch_n<L, T, 4>(links, in, out, g, ncol, m, M5, dagger, wil, wmass, skip, sks, st);
        case 8:  return launch_n<L, T, 8>(links, in, out, g, ncol, m, M5, dagger, wil, wmass, skip, sks, st);
        case 12: return launch_n<L, T, 12>(links, in, out, g, ncol, m, M5, dagger, wil, wmass, skip, sks, st);
        case 16: return launch_n<L, T, 16>(links, in, out, g, ncol, m, M5, dagger, wil, wmass, skip, sks, st);
        case 24: return launch_n<L, T, 24>(links, in, out, g, ncol, m, M5, dagger, wil, wmass, skip, sks, st);
        case 32: return launch_n<L, T, 32>(links, in, out, g, ncol, m, M5, dagger, wil, wmass, skip, sks, st);
        case 48: return launch_n<L, T, 48>(links, in, out, g, ncol, m, M5, dagger, wil, wmass, skip, sks, st);
        case 64: return launch_n<L, T, 64>(links, in, out, g, ncol, m, M5, dagger, wil, wmass, skip, sks, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename T>
hipError_t coarse_apply(const void* links, int link_prec, const cpx<T>* in, cpx<T>* out,
                        const CoarseGeom& g, int ncol, double m, double M5, bool dagger,
                        bool wilson_mode, double wilson_mass, const int* skip, int sks, hipStream_t st) {
    if (g.Ls < 1 || g.Ls > kMaxCoarseLs) return hipErrorInvalidValue;
    if (!wilson_mode && coarse_mfma_supported(g.n, link_prec))
        return coarse_apply_mfma<T>(links, link_prec, in, out, g, ncol, m, M5, dagger, skip, sks, st);
    switch (link_prec) {
        case P_F64: return launch_l<cpx<double>, T>(links, in, out, g, ncol, m, M5, dagger, wilson_mode, wilson_mass, skip, sks, st);
        case P_F32: return launch_l<cpx<float>, T>(links, in, out, g, ncol, m, M5, dagger, wilson_mode, wilson_mass, skip, sks, st);
        case P_BF16: return launch_l<cbf16, T>(links, in, out, g, ncol, m, M5, dagger, wilson_mode, wilson_mass, skip, sks, st);
        case P_F16: return launch_l<cf16, T>(links, in, out, g, ncol, m, M5, dagger, wilson_mode, wilson_mass, skip, sks, st);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t coarse_apply<float>(const void*, int, const cpx<float>*, cpx<float>*, const CoarseGeom&, int, double, double, bool, bool, double, const int*, int, hipStream_t);
template hipError_t coarse_apply<double>(const void*, int, const cpx<double>*, cpx<double>*, const CoarseGeom&, int, double, double, bool, bool, double, const int*, int, hipStream_t);

}  // namespace dwf
