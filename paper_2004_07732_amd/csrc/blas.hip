// BLAS-1 kernels and the device-resident Krylov scalar algebra.
//
// Reductions are deterministic and fence-free: the partial kernel reduces each
// block with wavefront shuffles (64 lanes) and a fixed-order sum over its four
// waves and writes one partial per quantity; a one-block-per-column finaliser
// (the next launch, so the kernel boundary orders the two) adds the partials
// in block order and turns the sums into Krylov coefficients.  No cross-block
// fence is needed inside a kernel, which matters on a part whose L2 caches are
// private to each XCD.  The host never has to read a scalar back to continue:
// CG, CGNR and GCR coefficients live on the device and a per-column `done` /
// `stop` flag turns later updates into no-ops.  Accumulation is FP64 for both
// FP32 and FP64 vectors.
#include <utility>

#include <algorithm>

#include "kernels.hpp"

namespace dwf {

namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kMaxQ = 40;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

// Reduce per-thread values v[0..nq) over the block; totals end in tot[0..nq)
// (shared) and are visible to every thread of the block afterwards.
template <int NQ>
__device__ __forceinline__ void block_reduce(double (&v)[NQ], int nq, double* sh, double* tot) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (q < nq) {
            double s = wave_sum(v[q]);
            if (lane == 0) sh[q * kWaves + wid] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x < nq) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += sh[threadIdx.x * kWaves + w];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
}

template <int NQ>
__device__ __forceinline__ void write_partials(double (&v)[NQ], int nq, const RedWork& rw, int col, double* sh,
                                               double* tot) {
    block_reduce<NQ>(v, nq, sh, tot);
    double* part = rw.partial + (size_t)col * rw.max_q * rw.nblk;
    if (threadIdx.x < nq) part[(size_t)threadIdx.x * rw.nblk + blockIdx.x] = tot[threadIdx.x];
}

// finaliser side: column `col` (= blockIdx.x), nb partials per quantity
template <int NQ>
__device__ __forceinline__ void sum_partials(int nq, int nb, const RedWork& rw, int col, double* sh, double* tot) {
    const double* part = rw.partial + (size_t)col * rw.max_q * rw.nblk;
    double w[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        w[q] = 0.0;
        if (q < nq)
            for (int b = threadIdx.x; b < nb; b += blockDim.x) w[q] += part[(size_t)q * rw.nblk + b];
    }
    block_reduce<NQ>(w, nq, sh, tot);
}

// at least two entries per thread: a block's partial sums cost about as much as
// streaming a few thousand entries, so small vectors take fewer, fuller blocks
inline dim3 red_grid(size_t n, int ncol, const RedWork& rw) {
    long long nb = (long long)((n + 2 * kBlock - 1) / (2 * kBlock));
    if (nb > rw.nblk) nb = rw.nblk;
    if (nb < 1) nb = 1;
    return dim3((unsigned)nb, (unsigned)ncol);
}

inline dim3 ew_grid(size_t n, int ncol) {
    long long nb = (long long)((n + kBlock - 1) / kBlock);
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    return dim3((unsigned)nb, (unsigned)ncol);
}

#define GRID_STRIDE(i, n) \
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

#define SHARED_RED __shared__ double sh[kMaxQ * kWaves], tot[kMaxQ]

// calls f(std::integral_constant<int, j>) for a run-time j in Js...
template <typename F, int... Js>
void with_j(int j, F&& f, std::integer_sequence<int, Js...>) {
    ((j == Js ? (f(std::integral_constant<int, Js>{}), 0) : 0), ...);
}


template <typename T>
__device__ __forceinline__ cpx<double> up(cpx<T> a) { return {(double)a.re, (double)a.im}; }

__device__ __forceinline__ bool finite(double x) { return !(isnan(x) || isinf(x)); }

}  // namespace

// ------------------------------------------------------------ elementwise
template <typename T>
__global__ void k_zero(cpx<T>* x, size_t n) {
    GRID_STRIDE(i, n) x[i] = {T(0), T(0)};
}
template <typename Ti, typename To>
__global__ void k_convert(const cpx<Ti>* in, cpx<To>* out, size_t n) {
    GRID_STRIDE(i, n) out[i] = {(To)in[i].re, (To)in[i].im};
}
template <typename Tx, typename Ty>
__global__ void k_add(const cpx<Tx>* x, cpx<Ty>* y, size_t n) {
    GRID_STRIDE(i, n) {
        cpx<Ty> a = y[i];
        y[i] = {a.re + (Ty)x[i].re, a.im + (Ty)x[i].im};
    }
}
template <typename T>
__global__ void k_sub(const cpx<T>* a, const cpx<T>* b, cpx<T>* out, size_t n) {
    GRID_STRIDE(i, n) out[i] = a[i] - b[i];
}

// y = a x + b y (b == 0: y = a x, whatever y held)
template <typename T>
__global__ void k_axpby(double a, const cpx<T>* x, double b, cpx<T>* y, size_t n) {
    const T ta = (T)a, tb = (T)b;
    if (b == 0.0) {
        GRID_STRIDE(i, n) y[i] = ta * x[i];
    } else {
        GRID_STRIDE(i, n) y[i] = ta * x[i] + tb * y[i];
    }
}
template <typename T> hipError_t vaxpby(double a, const cpx<T>* x, double b, cpx<T>* y, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby<T>, ew_grid(n, 1), dim3(kBlock), 0, st, a, x, b, y, n);
    return hipGetLastError();
}
template hipError_t vaxpby<float>(double, const cpx<float>*, double, cpx<float>*, size_t, hipStream_t);
template hipError_t vaxpby<double>(double, const cpx<double>*, double, cpx<double>*, size_t, hipStream_t);

template <typename T> hipError_t vzero(cpx<T>* x, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero<T>, ew_grid(n, 1), dim3(kBlock), 0, st, x, n);
    return hipGetLastError();
}
template <typename Ti, typename To>
hipError_t vconvert(const cpx<Ti>* in, cpx<To>* out, size_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_convert<Ti, To>), ew_grid(n, 1), dim3(kBlock), 0, st, in, out, n);
    return hipGetLastError();
}
template <typename Tx, typename Ty>
hipError_t vadd(const cpx<Tx>* x, cpx<Ty>* y, size_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_add<Tx, Ty>), ew_grid(n, 1), dim3(kBlock), 0, st, x, y, n);
    return hipGetLastError();
}
template <typename T>
hipError_t vsub(const cpx<T>* a, const cpx<T>* b, cpx<T>* out, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_sub<T>, ew_grid(n, 1), dim3(kBlock), 0, st, a, b, out, n);
    return hipGetLastError();
}

// ------------------------------------------------------------ streaming copy (bandwidth reference)
// dst = src in 16-byte words: each workgroup copies one contiguous chunk of
// 1024 words (16 KB), every thread issuing its four loads before its four
// nontemporal stores.  Of the copy forms measured on the MI355X (grid-stride
// loops with 1 k - 8 k workgroups, chunks of 1 k - 16 k words with 4 - 16 loads
// in flight, with and without nontemporal loads and stores, hipMemcpyAsync),
// this one moved the most bytes per second over 2 GiB.
typedef unsigned int sc_u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyChunk = 1024;
__global__ void __launch_bounds__(kBlock) k_stream_copy(const sc_u32x4* __restrict__ src, sc_u32x4* __restrict__ dst,
                                                        size_t n) {
    const size_t base = (size_t)blockIdx.x * kCopyChunk;
    if (base + kCopyChunk <= n) {
        sc_u32x4 v[kCopyChunk / kBlock];
#pragma unroll
        for (int u = 0; u < kCopyChunk / kBlock; ++u) v[u] = src[base + u * kBlock + threadIdx.x];
#pragma unroll
        for (int u = 0; u < kCopyChunk / kBlock; ++u)
            __builtin_nontemporal_store(v[u], dst + base + u * kBlock + threadIdx.x);
    } else {
        for (size_t i = base + threadIdx.x; i < n; i += kBlock) dst[i] = src[i];
    }
}

hipError_t stream_copy(const void* src, void* dst, size_t words, hipStream_t st) {
    const size_t blocks = (words + kCopyChunk - 1) / kCopyChunk;
    if (blocks == 0 || blocks > 0x7fffffffULL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                       reinterpret_cast<const sc_u32x4*>(src), reinterpret_cast<sc_u32x4*>(dst), words);
    return hipGetLastError();
}

// ------------------------------------------------------------ finalisers (one block per column)
// out[col * stride + q] = total q
__global__ void __launch_bounds__(kBlock) k_fin_store(RedWork rw, int nq, int nb, double* out, size_t stride) {
    SHARED_RED;
    const int col = blockIdx.x;
    sum_partials<kMaxQ>(nq, nb, rw, col, sh, tot);
    if (threadIdx.x < nq) out[(size_t)col * stride + threadIdx.x] = tot[threadIdx.x];
}

// the same sums with one block per (quantity, column): for many quantities
// the same with one wavefront per (quantity, column): no barrier, all loads in flight
__global__ void __launch_bounds__(64) k_fin_store_q1(RedWork rw, int nb, double* out, size_t stride) {
    const int q = blockIdx.x, col = blockIdx.y;
    const double* part = rw.partial + (size_t)col * rw.max_q * rw.nblk + (size_t)q * rw.nblk;
    double s = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nb; b += 64) s += part[b];
    s = wave_sum(s);
    if (threadIdx.x == 0) out[(size_t)col * stride + q] = s;
}

__global__ void __launch_bounds__(kBlock) k_fin_store_q(RedWork rw, int nb, double* out, size_t stride) {
    __shared__ double sh[kWaves];
    const int q = blockIdx.x, col = blockIdx.y;
    const double* part = rw.partial + (size_t)col * rw.max_q * rw.nblk + (size_t)q * rw.nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += sh[w];
        out[(size_t)col * stride + q] = t;
    }
}

__global__ void __launch_bounds__(kBlock) k_fin_cg_init(RedWork rw, int nb, CgScal* s, double tol2) {
    SHARED_RED;
    const int col = blockIdx.x;
    sum_partials<1>(1, nb, rw, col, sh, tot);
    if (threadIdx.x == 0) {
        CgScal c;
        c.zz = tot[0];
        c.zz0 = tot[0];
        c.alpha = 0.0;
        c.beta = 0.0;
        c.tol2 = tol2;
        c.iters = 0;
        c.done = (tot[0] == 0.0) ? 1 : (finite(tot[0]) ? 0 : 4);
        s[col] = c;
    }
}

__global__ void __launch_bounds__(kBlock) k_fin_cg_alpha(RedWork rw, int nb, CgScal* s) {
    SHARED_RED;
    const int col = blockIdx.x;
    if (s[col].done) return;
    sum_partials<1>(1, nb, rw, col, sh, tot);
    if (threadIdx.x == 0) {
        const double ww = tot[0];
        if (!(ww > 0.0) || !finite(ww)) {
            s[col].alpha = 0.0;
            s[col].done = finite(ww) ? 2 : 4;   // breakdown / non-finite
        } else {
            s[col].alpha = s[col].zz / ww;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_fin_cg_beta(RedWork rw, int nb, CgScal* s, int maxit) {
    SHARED_RED;
    const int col = blockIdx.x;
    if (s[col].done) return;
    sum_partials<1>(1, nb, rw, col, sh, tot);
    if (threadIdx.x == 0) {
        CgScal c = s[col];
        const double znew = tot[0];
        c.iters += 1;
        if (!finite(znew)) {
            c.done = 4;
        } else {
            c.beta = znew / c.zz;
            c.zz = znew;
            if (znew <= c.tol2 * c.zz0) c.done = 1;
            else if (c.iters >= maxit) c.done = 3;
        }
        s[col] = c;
    }
}

// ------------------------------------------------------------ reductions: partial kernels
template <typename T>
__global__ void __launch_bounds__(kBlock) k_norm2_part(const cpx<T>* x, size_t n, RedWork rw, const int* skip, int sks) {
    SHARED_RED;
    const int col = blockIdx.y;
    if (skip && skip[(size_t)col * sks]) return;
    const cpx<T>* xc = x + (size_t)col * n;
    double v[1] = {0.0};
    GRID_STRIDE(i, n) {
        cpx<double> a = up(xc[i]);
        v[0] += a.re * a.re + a.im * a.im;
    }
    write_partials<1>(v, 1, rw, col, sh, tot);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_cdot_part(const cpx<T>* a, const cpx<T>* b, size_t n, RedWork rw) {
    SHARED_RED;
    const int col = blockIdx.y;
    const cpx<T>* ac = a + (size_t)col * n;
    const cpx<T>* bc = b + (size_t)col * n;
    double v[2] = {0.0, 0.0};
    GRID_STRIDE(i, n) {
        cpx<double> p = cjmul(up(ac[i]), up(bc[i]));
        v[0] += p.re;
        v[1] += p.im;
    }
    write_partials<2>(v, 2, rw, col, sh, tot);
}

namespace {
const int kCgSkipStride = (int)(sizeof(CgScal) / sizeof(int));
}

template <typename T>
hipError_t norm2(const cpx<T>* x, size_t n, int ncol, double* out, const RedWork& rw, hipStream_t st) {
    dim3 g = red_grid(n, ncol, rw);
    hipLaunchKernelGGL(k_norm2_part<T>, g, dim3(kBlock), 0, st, x, n, rw, (const int*)nullptr, 1);
    hipLaunchKernelGGL(k_fin_store, dim3(ncol), dim3(kBlock), 0, st, rw, 1, (int)g.x, out, (size_t)1);
    return hipGetLastError();
}
template <typename T>
hipError_t cdot(const cpx<T>* a, const cpx<T>* b, size_t n, int ncol, double* out2, const RedWork& rw, hipStream_t st) {
    dim3 g = red_grid(n, ncol, rw);
    hipLaunchKernelGGL(k_cdot_part<T>, g, dim3(kBlock), 0, st, a, b, n, rw);
    hipLaunchKernelGGL(k_fin_store, dim3(ncol), dim3(kBlock), 0, st, rw, 2, (int)g.x, out2, (size_t)2);
    return hipGetLastError();
}

// ------------------------------------------------------------ CG family
template <typename T>
hipError_t cg_init(const cpx<T>* v, size_t n, int ncol, CgScal* s, double tol, const RedWork& rw, hipStream_t st) {
    dim3 g = red_grid(n, ncol, rw);
    hipLaunchKernelGGL(k_norm2_part<T>, g, dim3(kBlock), 0, st, v, n, rw, (const int*)nullptr, 1);
    hipLaunchKernelGGL(k_fin_cg_init, dim3(ncol), dim3(kBlock), 0, st, rw, (int)g.x, s, tol * tol);
    return hipGetLastError();
}
template <typename T>
hipError_t cg_alpha(const cpx<T>* w, size_t n, int ncol, CgScal* s, const RedWork& rw, hipStream_t st) {
    dim3 g = red_grid(n, ncol, rw);
    hipLaunchKernelGGL(k_norm2_part<T>, g, dim3(kBlock), 0, st, w, n, rw, &s[0].done, kCgSkipStride);
    hipLaunchKernelGGL(k_fin_cg_alpha, dim3(ncol), dim3(kBlock), 0, st, rw, (int)g.x, s);
    return hipGetLastError();
}

template <typename T>
__global__ void k_cg_update_xr(cpx<T>* x, cpx<T>* r, const cpx<T>* p, const cpx<T>* w, size_t n, const CgScal* s) {
    const int col = blockIdx.y;
    if (s[col].done) return;
    const T a = (T)s[col].alpha;
    const size_t o = (size_t)col * n;
    GRID_STRIDE(i, n) {
        cpx<T> pi = p[o + i], wi = w[o + i], xi = x[o + i], ri = r[o + i];
        x[o + i] = {xi.re + a * pi.re, xi.im + a * pi.im};
        r[o + i] = {ri.re - a * wi.re, ri.im - a * wi.im};
    }
}

template <typename T>
__global__ void k_cg_update_p(cpx<T>* p, const cpx<T>* z, size_t n, const CgScal* s) {
    const int col = blockIdx.y;
    if (s[col].done) return;
    const T b = (T)s[col].beta;
    const size_t o = (size_t)col * n;
    GRID_STRIDE(i, n) {
        cpx<T> pi = p[o + i], zi = z[o + i];
        p[o + i] = {zi.re + b * pi.re, zi.im + b * pi.im};
    }
}

template <typename T>
hipError_t cg_update_xr(cpx<T>* x, cpx<T>* r, const cpx<T>* p, const cpx<T>* w, size_t n, int ncol,
                        const CgScal* s, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_update_xr<T>, ew_grid(n, ncol), dim3(kBlock), 0, st, x, r, p, w, n, s);
    return hipGetLastError();
}
template <typename T>
hipError_t cg_beta(const cpx<T>* z, size_t n, int ncol, CgScal* s, int maxit, const RedWork& rw, hipStream_t st) {
    dim3 g = red_grid(n, ncol, rw);
    hipLaunchKernelGGL(k_norm2_part<T>, g, dim3(kBlock), 0, st, z, n, rw, &s[0].done, kCgSkipStride);
    hipLaunchKernelGGL(k_fin_cg_beta, dim3(ncol), dim3(kBlock), 0, st, rw, (int)g.x, s, maxit);
    return hipGetLastError();
}
template <typename T>
hipError_t cg_update_p(cpx<T>* p, const cpx<T>* z, size_t n, int ncol, const CgScal* s, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_update_p<T>, ew_grid(n, ncol), dim3(kBlock), 0, st, p, z, n, s);
    return hipGetLastError();
}

// ------------------------------------------------------------ GCR
namespace {
__device__ __forceinline__ cpx<double> ld2(const double* p) { return {p[0], p[1]}; }
// entries per thread whose loads the fused GCR kernels issue together (bounded by
// the registers of U (j + 2) loaded vectors)
template <typename T>
constexpr int gcr_unroll(int j) {
    return sizeof(T) == 4 ? (j <= 6 ? 4 : 2) : (j <= 6 ? 2 : 1);
}

__device__ __forceinline__ cpx<double> cdiv_real(cpx<double> a, double d) {
    return d > 0.0 ? cpx<double>{a.re / d, a.im / d} : cpx<double>{0.0, 0.0};
}
}  // namespace

template <typename T, int j>   // (j: directions, a template argument so that every load is unconditional)
__global__ void __launch_bounds__(kBlock)
k_gcr_multidot(const cpx<T>* W, size_t wstride, const cpx<T>* w, size_t n, GcrDev g, RedWork rw) {
    SHARED_RED;
    const int col = blockIdx.y;
    const size_t o = (size_t)col * n;
    const bool stop = g.stop[col] != 0;
    double v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] = 0.0;
    if (!stop) GRID_STRIDE(e, n) {
        const cpx<double> we = up(w[o + e]);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i < j) {
                cpx<double> p = cjmul(up(W[(size_t)i * wstride + o + e]), we);
                v[2 * i] += p.re;
                v[2 * i + 1] += p.im;
            }
        }
    }
    write_partials<32>(v, 2 * j, rw, col, sh, tot);
}

template <typename T, int j>
__global__ void __launch_bounds__(kBlock)
k_gcr_orth(const cpx<T>* W, size_t wstride, cpx<T>* w, const cpx<T>* r, size_t n, GcrDev g, RedWork rw) {
    SHARED_RED;
    const int col = blockIdx.y;
    const bool stop = g.stop[col] != 0;
    const size_t o = (size_t)col * n;
    cpx<T> c[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        c[i] = {T(0), T(0)};
        if (i < j && !stop) {
            cpx<double> d = ld2(&g.D[(((size_t)col * g.kmax + j) * g.kmax + i) * 2]);
            cpx<double> ci = cdiv_real(d, g.nn[(size_t)col * g.kmax + i]);
            c[i] = {(T)ci.re, (T)ci.im};
        }
    }
    double v[3] = {0.0, 0.0, 0.0};
    GRID_STRIDE(e, n) {
        cpx<T> we = w[o + e];
        if (!stop && j > 0) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < j) {
                    cpx<T> Wi = W[(size_t)i * wstride + o + e];
                    we.re -= c[i].re * Wi.re - c[i].im * Wi.im;
                    we.im -= c[i].re * Wi.im + c[i].im * Wi.re;
                }
            w[o + e] = we;
        }
        const cpx<double> wd = up(we), rd = up(r[o + e]);
        v[0] += wd.re * wd.re + wd.im * wd.im;
        cpx<double> p = cjmul(wd, rd);
        v[1] += p.re;
        v[2] += p.im;
    }
    write_partials<3>(v, 3, rw, col, sh, tot);
}

__global__ void __launch_bounds__(kBlock) k_fin_gcr_orth(RedWork rw, int nb, GcrDev g, int j) {
    SHARED_RED;
    const int col = blockIdx.x;
    sum_partials<3>(3, nb, rw, col, sh, tot);
    if (threadIdx.x == 0) {
        const size_t s = (size_t)col * g.kmax + j;
        if (g.stop[col]) {
            g.nn[s] = 0.0;
            g.wr[2 * s] = 0.0;
            g.wr[2 * s + 1] = 0.0;
        } else {
            g.nn[s] = tot[0];
            g.wr[2 * s] = tot[1];
            g.wr[2 * s + 1] = tot[2];
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_gcr_rupdate(const cpx<T>* w, cpx<T>* r, cpx<T>* copy, int j, size_t n, int want_norm, GcrDev g, RedWork rw) {
    SHARED_RED;
    const int col = blockIdx.y;
    const size_t s = (size_t)col * g.kmax + j;
    const cpx<double> ad = cdiv_real(ld2(&g.wr[2 * s]), g.nn[s]);
    const cpx<T> a = {(T)ad.re, (T)ad.im};
    const size_t o = (size_t)col * n;
    double v[1] = {0.0};
    GRID_STRIDE(e, n) {
        cpx<T> re = r[o + e];
        const cpx<T> we = w[o + e];
        re.re -= a.re * we.re - a.im * we.im;
        re.im -= a.re * we.im + a.im * we.re;
        r[o + e] = re;
        if (copy) copy[o + e] = re;
        const cpx<double> rd = up(re);
        v[0] += rd.re * rd.re + rd.im * rd.im;
    }
    if (want_norm) write_partials<1>(v, 1, rw, col, sh, tot);
}

// ---- fused GCR iteration (see kernels.hpp); the direction count j is a template
// argument, so that every load of an iteration is unconditional and in flight at once
template <typename T, int j>
__global__ void __launch_bounds__(kBlock)
k_gcr_dots(const cpx<T>* W, size_t wstride, const cpx<T>* w, const cpx<T>* r, size_t n, const int* stop,
           RedWork rw) {
    SHARED_RED;
    const int col = blockIdx.y;
    const size_t o = (size_t)col * n;
    // the vectors are read whatever the stop flag says, so that no load waits for it;
    // a stopped column's sums (possibly of unwritten directions) are replaced by zeros.
    // The flag is read by a vector load (an offset the compiler cannot see is zero), which
    // completes in order with the vectors' loads instead of holding them back.
    int zoff;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zoff));
    const int sflag = stop[col + zoff];
    // layout (static indices, so the accumulators stay in registers):
    // [|w|^2, Re <w, r>, Im <w, r>, Re <W_0, w>, Im <W_0, w>, ...]
    double v[35];
#pragma unroll
    for (int q = 0; q < 35; ++q) v[q] = 0.0;
    // the entries of a thread are added in grid-stride order; U of them are loaded
    // together, so that a thread keeps U (j + 2) loads in flight (same sums, same order)
    constexpr int U = gcr_unroll<T>(j);
    auto add = [&](const cpx<T>& wt, const cpx<T>& rt, const cpx<T>* Wt) {
        const cpx<double> we = up(wt), re = up(rt);
#pragma unroll
        for (int i = 0; i < j; ++i) {
            const cpx<double> p = cjmul(up(Wt[i]), we);
            v[3 + 2 * i] += p.re;
            v[4 + 2 * i] += p.im;
        }
        v[0] += we.re * we.re + we.im * we.im;
        const cpx<double> p = cjmul(we, re);
        v[1] += p.re;
        v[2] += p.im;
    };
    {
        const size_t stride = (size_t)gridDim.x * blockDim.x;
        size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
        for (; e + (U - 1) * stride < n; e += U * stride) {
            cpx<T> wv[U], rv[U], Wv[U][j > 0 ? j : 1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                wv[u] = w[o + e + u * stride];
                rv[u] = r[o + e + u * stride];
#pragma unroll
                for (int i = 0; i < j; ++i) Wv[u][i] = W[(size_t)i * wstride + o + e + u * stride];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) add(wv[u], rv[u], Wv[u]);
        }
        for (; e < n; e += stride) {
            cpx<T> Wt[j > 0 ? j : 1];
#pragma unroll
            for (int i = 0; i < j; ++i) Wt[i] = W[(size_t)i * wstride + o + e];
            add(w[o + e], r[o + e], Wt);
        }
    }
#pragma unroll
    for (int q = 0; q < 35; ++q) v[q] = sflag != 0 ? 0.0 : v[q];
    write_partials<35>(v, 2 * j + 3, rw, col, sh, tot);
}

template <typename T, int j>
__global__ void __launch_bounds__(kBlock)
k_gcr_fused_update(const cpx<T>* W, size_t wstride, cpx<T>* w, cpx<T>* r, cpx<T>* copy, size_t n,
                   double tol2, const int* stop_in, int* stop_out, GcrDev g) {
    const int col = blockIdx.y;
    const bool stopped = stop_in[col] != 0;
    const double* t = g.tot + (size_t)col * kGcrTot;
    const size_t kb = (size_t)col * g.kmax;
    cpx<double> c[16];
    double nnj = t[0];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        c[i] = {0.0, 0.0};
        if (i < j) {
            const cpx<double> d = {t[3 + 2 * i], t[4 + 2 * i]};
            const double nni = g.nn[kb + i];
            if (nni > 0.0) {
                c[i] = {d.re / nni, d.im / nni};
                nnj -= (d.re * d.re + d.im * d.im) / nni;
            }
        }
    }
    const cpx<double> wr = {t[1], t[2]};
    const bool live = !stopped && nnj > 0.0;
    const cpx<double> a = live ? cpx<double>{wr.re / nnj, wr.im / nnj} : cpx<double>{0.0, 0.0};
    const size_t o = (size_t)col * n;
    if (!stopped) {
        cpx<T> cc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) cc[i] = {(T)c[i].re, (T)c[i].im};
        const cpx<T> at = {(T)a.re, (T)a.im};
        // one entry: w' = w - sum c_i W_i, r -= a w', copy = r (U entries' loads issued together)
        auto step = [&](size_t i0, cpx<T> we, cpx<T> re, const cpx<T>* Wt) {
#pragma unroll
            for (int i = 0; i < j; ++i) {
                we.re -= cc[i].re * Wt[i].re - cc[i].im * Wt[i].im;
                we.im -= cc[i].re * Wt[i].im + cc[i].im * Wt[i].re;
            }
            w[i0] = we;
            re.re -= at.re * we.re - at.im * we.im;
            re.im -= at.re * we.im + at.im * we.re;
            r[i0] = re;
            if (copy) copy[i0] = re;
        };
        constexpr int U = gcr_unroll<T>(j);
        const size_t stride = (size_t)gridDim.x * blockDim.x;
        size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
        for (; e + (U - 1) * stride < n; e += U * stride) {
            cpx<T> wv[U], rv[U], Wv[U][j > 0 ? j : 1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                wv[u] = w[o + e + u * stride];
                rv[u] = r[o + e + u * stride];
#pragma unroll
                for (int i = 0; i < j; ++i) Wv[u][i] = W[(size_t)i * wstride + o + e + u * stride];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) step(o + e + u * stride, wv[u], rv[u], Wv[u]);
        }
        for (; e < n; e += stride) {
            cpx<T> Wt[j > 0 ? j : 1];
#pragma unroll
            for (int i = 0; i < j; ++i) Wt[i] = W[(size_t)i * wstride + o + e];
            step(o + e, w[o + e], r[o + e], Wt);
        }
    } else if (copy) {
        // a column that stopped earlier in the cycle: its later directions are zero.  The
        // solution update weights them by zero coefficients, which must not meet whatever
        // the unwritten buffer holds (a non-finite word would turn 0 x into NaN), and a
        // zero direction keeps the stencil of that column finite for its tile neighbours.
        GRID_STRIDE(e, n) copy[o + e] = cpx<T>{(T)0, (T)0};
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const size_t s = kb + j;
        g.nn[s] = live ? nnj : 0.0;
        g.wr[2 * s] = live ? wr.re : 0.0;
        g.wr[2 * s + 1] = live ? wr.im : 0.0;
        for (int i = 0; i < j; ++i) {   // <W_i, w> for the back substitution
            g.D[((kb + j) * g.kmax + i) * 2] = stopped ? 0.0 : t[3 + 2 * i];
            g.D[((kb + j) * g.kmax + i) * 2 + 1] = stopped ? 0.0 : t[4 + 2 * i];
        }
        int sflag = stop_in[col];
        if (!stopped) {
            double rr = g.rr[col] - (live ? (wr.re * wr.re + wr.im * wr.im) / nnj : 0.0);
            if (rr < 0.0) rr = 0.0;
            g.rr[col] = rr;
            g.it[col] += 1;
            if (!finite(rr) || !finite(nnj)) sflag = 2;
            else if (rr <= tol2 * g.bb[col]) sflag = 1;
        }
        stop_out[col] = sflag;
    }
}

// ---- Gram-form GCR step (short restart cycles: the smoother's and the coarsest solve's).
// With w_i = A p_i kept as computed (not orthogonalised) and r0 the cycle's starting
// residual, step j's minimal residual over span(p_0..p_j) is r_{j+1} = r0 - sum_{i<=j} y_i w_i
// with G y = b, G_il = <w_i, w_l>, b_i = <w_i, r0> (the normal equations of the same
// least-squares problem GCR solves by orthogonalising).  The multi-dot of step j gives G's
// new row and b_j.  Its finaliser is one workgroup per column: wave q adds the partials of
// quantity q, then one thread solves the (j+1)-square system by Cholesky in FP64 registers
// (a pivot that is not positive drops that direction: its y is zero) and stores G's row,
// b_j, y, the new residual norm and the stop flag.  A streaming pass then writes
// r_{j+1}, the next direction (k_gcr_gram_step), or at the cycle's last step adds the
// correction to x and leaves r_{j+1} in P_0 (k_gcr_gram_last); no orthogonalised direction
// and no running residual is written.
constexpr int kGramPartials = 1024;   // multi-dot blocks per column (partials per finaliser wave)
template <int j>
__global__ void __launch_bounds__(64 * (2 * kGramMax + 1)) k_fin_gram(RedWork rw, int nb, const int* stop_in,
                                                                     int* stop_out, GcrDev g, double tol2, int last) {
    constexpr int m = j + 1;
    constexpr int NQ = 2 * j + 3;
    static_assert(64 * NQ <= 1024, "one wave per inner product in one workgroup");
    // G's rows and b of the cycle's earlier steps, one value per thread: D's j x j block
    // (only the lower triangle is used), |w_i|^2, <w_i, r0>
    constexpr int ND = 2 * j * j;
    constexpr int NOLD = ND + 3 * j;
    static_assert(NOLD <= 64 * NQ, "one earlier value per thread");
    __shared__ double tq[NQ];
    __shared__ double old[NOLD > 0 ? NOLD : 1];
    const int col = blockIdx.x;
    const int t = threadIdx.x;
    const int lane = t & 63, q = t >> 6;   // one wave per quantity
    const size_t kb = (size_t)col * g.kmax;
    // every load is issued before the first wait: the stop flag, the partials (added
    // whether or not the column has stopped: a stopped column's sums go unused) and the
    // earlier rows.  The flag and the column's scalars are read by vector loads (an offset
    // the compiler cannot see is zero), which complete in order with the partials' loads
    // instead of holding them back in a wait shared with the kernel arguments.
    int zoff;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zoff));
    const int sflag = stop_in[col + zoff];
    const double rr0 = g.rr[col + zoff];
    const int it0 = g.it[col + zoff];
    double ov = 0.0;
    if (t < NOLD) {   // (the address by selects: one load, no branches between the loads)
        const double* src = t < ND ? g.D + ((kb + t / (2 * j)) * g.kmax + (t % (2 * j)) / 2) * 2 + (t & 1)
                                   : (t < ND + j ? g.nn + kb + (t - ND) : g.wr + 2 * kb + (t - ND - j));
        ov = *src;
    }
    {
        const double* part = rw.partial + (size_t)col * rw.max_q * rw.nblk + (size_t)q * rw.nblk;
        double sq = 0.0;
#pragma unroll 8
        for (int b = lane; b < nb; b += 64) sq += part[b];
        sq = wave_sum(sq);
        if (lane == 0) tq[q] = sq;
    }
    if (t < NOLD) old[t] = ov;
    __syncthreads();
    if (t != 0) return;
    if (sflag != 0) {
        for (int l = 0; l < j; ++l) {
            g.D[((kb + j) * g.kmax + l) * 2] = 0.0;
            g.D[((kb + j) * g.kmax + l) * 2 + 1] = 0.0;
        }
        g.nn[kb + j] = 0.0;
        g.wr[2 * (kb + j)] = 0.0;
        g.wr[2 * (kb + j) + 1] = 0.0;
        // the coefficients of the step the column stopped at stay (a stopped step's own is
        // zero), so that the cycle's solution update adds that step's minimal residual correction
        g.gam[2 * (kb + j)] = 0.0;
        g.gam[2 * (kb + j) + 1] = 0.0;
        stop_out[col] = sflag;
        return;
    }
    // G (lower triangle: G_il = conj <w_l, w_i>, l < i) and b
    cpx<double> G[m][m], b[m];
#pragma unroll
    for (int i = 0; i < j; ++i) {
#pragma unroll
        for (int l = 0; l < i; ++l) G[i][l] = {old[i * 2 * j + 2 * l], -old[i * 2 * j + 2 * l + 1]};
        G[i][i] = {old[ND + i], 0.0};
        b[i] = {old[ND + j + 2 * i], old[ND + j + 2 * i + 1]};
    }
#pragma unroll
    for (int l = 0; l < j; ++l) G[j][l] = {tq[3 + 2 * l], -tq[4 + 2 * l]};
    G[j][j] = {tq[0], 0.0};
    b[j] = {tq[1], tq[2]};
    // Cholesky G = L L^H in place (lower triangle), inv[i] = 1 / L_ii or 0 for a dropped direction
    double inv[m];
#pragma unroll
    for (int i = 0; i < m; ++i) {
#pragma unroll
        for (int l = 0; l <= i; ++l) {
            cpx<double> acc = G[i][l];
#pragma unroll
            for (int qq = 0; qq < l; ++qq) {   // - L_iq conj(L_lq)
                acc.re -= G[i][qq].re * G[l][qq].re + G[i][qq].im * G[l][qq].im;
                acc.im -= G[i][qq].im * G[l][qq].re - G[i][qq].re * G[l][qq].im;
            }
            if (l == i) {
                const bool ok = acc.re > 0.0 && finite(acc.re);
                inv[i] = ok ? 1.0 / sqrt(acc.re) : 0.0;
                G[i][i] = {ok ? sqrt(acc.re) : 0.0, 0.0};
            } else {
                G[i][l] = {acc.re * inv[l], acc.im * inv[l]};
            }
        }
    }
    cpx<double> u[m], y[m];
#pragma unroll
    for (int i = 0; i < m; ++i) {   // L u = b
        cpx<double> acc = b[i];
#pragma unroll
        for (int qq = 0; qq < i; ++qq) {
            acc.re -= G[i][qq].re * u[qq].re - G[i][qq].im * u[qq].im;
            acc.im -= G[i][qq].re * u[qq].im + G[i][qq].im * u[qq].re;
        }
        u[i] = {acc.re * inv[i], acc.im * inv[i]};
    }
#pragma unroll
    for (int i = m - 1; i >= 0; --i) {   // L^H y = u, (L^H)_iq = conj(L_qi)
        cpx<double> acc = u[i];
#pragma unroll
        for (int qq = i + 1; qq < m; ++qq) {
            acc.re -= G[qq][i].re * y[qq].re + G[qq][i].im * y[qq].im;
            acc.im -= G[qq][i].re * y[qq].im - G[qq][i].im * y[qq].re;
        }
        y[i] = {acc.re * inv[i], acc.im * inv[i]};
    }
#pragma unroll
    for (int l = 0; l < j; ++l) {
        g.D[((kb + j) * g.kmax + l) * 2] = tq[3 + 2 * l];
        g.D[((kb + j) * g.kmax + l) * 2 + 1] = tq[4 + 2 * l];
    }
    g.nn[kb + j] = tq[0];
    g.wr[2 * (kb + j)] = tq[1];
    g.wr[2 * (kb + j) + 1] = tq[2];
    // |r_{j+1}|^2 = |r0|^2 - Re <b, y> (the minimal residual), the cycle's |r0|^2 in g.rr
    double by = 0.0;
#pragma unroll
    for (int i = 0; i < m; ++i) {
        g.gam[2 * (kb + i)] = y[i].re;
        g.gam[2 * (kb + i) + 1] = y[i].im;
        by += b[i].re * y[i].re + b[i].im * y[i].im;
    }
    double rr = rr0 - by;
    if (rr < 0.0) rr = 0.0;
    if (last) g.rr[col] = rr;
    g.it[col] = it0 + 1;
    int f = 0;
    if (!(finite(tq[0]) && finite(tq[1]) && finite(tq[2]) && finite(rr))) f = 2;
    else if (rr <= tol2 * g.bb[col]) f = 1;
    stop_out[col] = f;
}

template <typename T, int j>
__global__ void __launch_bounds__(kBlock)
k_gcr_gram_step(const cpx<T>* W, size_t wstride, const cpx<T>* r0, cpx<T>* out, size_t n, const int* stop_in,
                GcrDev g) {
    constexpr int m = j + 1;
    const int col = blockIdx.y;
    const size_t o = (size_t)col * n;
    // the coefficients are loaded with the stop flag, one wait for both (the empty asm
    // statements take them before the branch; the compiler would otherwise move the
    // coefficient loads below it, a second round trip)
    const double* gam = g.gam + 2 * (size_t)col * g.kmax;
    double gv[2 * m];
#pragma unroll
    for (int i = 0; i < 2 * m; ++i) gv[i] = gam[i];
    const int sflag = stop_in[col];
#pragma unroll
    for (int i = 0; i < 2 * m; ++i) asm volatile("" ::"s"(gv[i]));
    cpx<T> c[m];
#pragma unroll
    for (int i = 0; i < m; ++i) c[i] = {(T)gv[2 * i], (T)gv[2 * i + 1]};
    if (sflag != 0) {   // (block-uniform) a stopped column's later directions are zero; r0 is kept
        if (out != r0) GRID_STRIDE(e, n) out[o + e] = cpx<T>{(T)0, (T)0};
        return;
    }
    constexpr int U = gcr_unroll<T>(j);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    auto step = [&](size_t i0, cpx<T> re, const cpx<T>* Wt) {
#pragma unroll
        for (int i = 0; i < m; ++i) {
            re.re -= c[i].re * Wt[i].re - c[i].im * Wt[i].im;
            re.im -= c[i].re * Wt[i].im + c[i].im * Wt[i].re;
        }
        out[i0] = re;
    };
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e + (U - 1) * stride < n; e += U * stride) {
        cpx<T> rv[U], Wv[U][m];
#pragma unroll
        for (int u2 = 0; u2 < U; ++u2) {
            rv[u2] = r0[o + e + u2 * stride];
#pragma unroll
            for (int i = 0; i < m; ++i) Wv[u2][i] = W[(size_t)i * wstride + o + e + u2 * stride];
        }
#pragma unroll
        for (int u2 = 0; u2 < U; ++u2) step(o + e + u2 * stride, rv[u2], Wv[u2]);
    }
    for (; e < n; e += stride) {
        cpx<T> Wt[m];
#pragma unroll
        for (int i = 0; i < m; ++i) Wt[i] = W[(size_t)i * wstride + o + e];
        step(o + e, r0[o + e], Wt);
    }
}

// The last Gram-form step of a cycle together with the cycle's solution update: with
// P_0 = r0 (the cycle's starting residual, the first direction), x += sum_{i<K} y_i P_i and
// P_0 = r0 - sum_{i<K} y_i W_i (the next cycle's starting residual) in one pass, element
// by element in place.
template <typename T, int K>
__global__ void __launch_bounds__(kBlock)
k_gcr_gram_last(cpx<T>* P, const cpx<T>* W, size_t stride_v, cpx<T>* x, size_t n, const int* stop_src, GcrDev g,
                int ncol) {
    const int col = blockIdx.y;
    const size_t o = (size_t)col * n;
    if (stop_src != g.stop && blockIdx.x == 0 && blockIdx.y == 0)
        for (int cc = threadIdx.x; cc < ncol; cc += blockDim.x) g.stop[cc] = stop_src[cc];
    const double* gam = g.gam + 2 * (size_t)col * g.kmax;
    cpx<double> c[K];
#pragma unroll
    for (int i = 0; i < K; ++i) c[i] = {gam[2 * i], gam[2 * i + 1]};
    GRID_STRIDE(e, n) {
        cpx<double> acc = {(double)x[o + e].re, (double)x[o + e].im};
        cpx<T> rn = P[o + e];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const cpx<double> p = up(P[(size_t)i * stride_v + o + e]);
            acc.re += c[i].re * p.re - c[i].im * p.im;
            acc.im += c[i].re * p.im + c[i].im * p.re;
            const cpx<T> wv = W[(size_t)i * stride_v + o + e];
            const cpx<T> ci = {(T)c[i].re, (T)c[i].im};
            rn.re -= ci.re * wv.re - ci.im * wv.im;
            rn.im -= ci.re * wv.im + ci.im * wv.re;
        }
        x[o + e] = {(T)acc.re, (T)acc.im};
        P[o + e] = rn;
    }
}

// restart of the device-driven GCR on the recursive residual: the next first
// direction is r, and the stop flags of the last step move to g.stop
template <typename T>
__global__ void k_gcr_restart(const cpx<T>* r, cpx<T>* P0, size_t n, const int* stop_src, int* stop, int ncol) {
    if (blockIdx.x == 0 && stop_src != stop)
        for (int c = threadIdx.x; c < ncol; c += blockDim.x) stop[c] = stop_src[c];
    GRID_STRIDE(i, n) P0[i] = r[i];
}

__global__ void k_gcr_dev_init(int ncol, GcrDev g) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    const double b = g.rr[c];
    g.bb[c] = b;
    g.it[c] = 0;
    g.stop[c] = finite(b) ? (b == 0.0 ? 1 : 0) : 2;
}

// back substitution gam_j = (wr_j - sum_{l>j} D[l][j] gam_l) / nn_j, from arrays laid out
// as in GcrDev (row stride ds of D); shared by the one-thread kernel and the x-update
__device__ __forceinline__ void gcr_back_substitute(int k, const double* wr, const double* nn, const double* D,
                                                    size_t ds, double* gam) {
    for (int j = k - 1; j >= 0; --j) {
        cpx<double> gj = cdiv_real(ld2(&wr[2 * j]), nn[j]);
        for (int l = j + 1; l < k; ++l) {
            // beta_{j l} = <w_j, A p_l> / |w_j|^2
            cpx<double> bjl = cdiv_real(ld2(&D[(l * ds + j) * 2]), nn[j]);
            cpx<double> gl = ld2(&gam[2 * l]);
            cpx<double> t = cmul(bjl, gl);
            gj.re -= t.re;
            gj.im -= t.im;
        }
        gam[2 * j] = gj.re;
        gam[2 * j + 1] = gj.im;
    }
}

__global__ void k_gcr_solve(int k, int ncol, GcrDev g) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncol) return;
    const size_t b = (size_t)col * g.kmax;
    gcr_back_substitute(k, g.wr + 2 * b, g.nn + b, g.D + b * g.kmax * 2, (size_t)g.kmax, g.gam + 2 * b);
}

// (the direction count K is a template argument, as in the fused GCR kernels: with a
// run-time count every direction's load sat behind its own branch and waited there)
template <typename T, typename Tx, int K>
__global__ void k_gcr_xupdate(const cpx<T>* P, size_t pstride, cpx<Tx>* x, size_t n, int accumulate, GcrDev g,
                              int solve, const cpx<T>* rsrc, cpx<T>* p0dst, const int* stop_src, int ncol) {
    constexpr int k = K;
    const int col = blockIdx.y;
    const size_t o = (size_t)col * n;
    const double* gam = g.gam + 2 * (size_t)col * g.kmax;
    __shared__ double sD[16 * 16 * 2], snn[16], swr[32], sgam[32];
    if (solve) {
        // every block solves the small triangular system itself (the same arithmetic in
        // the same order as the one-thread kernel): the entries are loaded in parallel
        // into LDS, one thread substitutes, block 0 stores gam
        const size_t b = (size_t)col * g.kmax;
        for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
            const int l = t / k, j = t - l * k;
            sD[(l * 16 + j) * 2] = g.D[((b + l) * g.kmax + j) * 2];
            sD[(l * 16 + j) * 2 + 1] = g.D[((b + l) * g.kmax + j) * 2 + 1];
        }
        if (threadIdx.x < k) {
            snn[threadIdx.x] = g.nn[b + threadIdx.x];
            swr[2 * threadIdx.x] = g.wr[2 * (b + threadIdx.x)];
            swr[2 * threadIdx.x + 1] = g.wr[2 * (b + threadIdx.x) + 1];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            gcr_back_substitute(k, swr, snn, sD, 16, sgam);
            if (blockIdx.x == 0)
                for (int i = 0; i < 2 * k; ++i) g.gam[2 * b + i] = sgam[i];
        }
        __syncthreads();
        gam = sgam;
    }
    cpx<double> c[K > 0 ? K : 1];
#pragma unroll
    for (int i = 0; i < K; ++i) c[i] = cpx<double>{gam[2 * i], gam[2 * i + 1]};
    if (stop_src && stop_src != g.stop && blockIdx.x == 0 && blockIdx.y == 0)
        for (int cc = threadIdx.x; cc < ncol; cc += blockDim.x) g.stop[cc] = stop_src[cc];
    GRID_STRIDE(e, n) {
        cpx<double> acc = {0.0, 0.0};
        if (accumulate) acc = {(double)x[o + e].re, (double)x[o + e].im};
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const cpx<double> p = up(P[(size_t)i * pstride + o + e]);
            acc.re += c[i].re * p.re - c[i].im * p.im;
            acc.im += c[i].re * p.im + c[i].im * p.re;
        }
        x[o + e] = {(Tx)acc.re, (Tx)acc.im};
        // restart: the residual becomes the first direction (after P_0 was read above)
        if (p0dst) p0dst[o + e] = rsrc[o + e];
    }
}

template <typename T>
hipError_t gcr_multidot(const cpx<T>* W, size_t wstride, int j, const cpx<T>* w, size_t n, int ncol,
                        const GcrDev& g, const RedWork& rw, hipStream_t st) {
    if (j <= 0) return hipSuccess;
    if (j > 16) return hipErrorInvalidValue;
    dim3 grid = red_grid(n, ncol, rw);
    with_j(j, [&](auto jc) {
        hipLaunchKernelGGL((k_gcr_multidot<T, decltype(jc)::value>), grid, dim3(kBlock), 0, st, W, wstride, w, n, g, rw);
    }, std::make_integer_sequence<int, 17>{});
    hipLaunchKernelGGL(k_fin_store_q, dim3(2 * j, ncol), dim3(kBlock), 0, st, rw, (int)grid.x,
                       g.D + (size_t)j * g.kmax * 2, (size_t)g.kmax * g.kmax * 2);
    return hipGetLastError();
}
template <typename T>
hipError_t gcr_orth(const cpx<T>* W, size_t wstride, int j, cpx<T>* w, const cpx<T>* r, size_t n,
                    int ncol, const GcrDev& g, const RedWork& rw, hipStream_t st) {
    if (j > 16) return hipErrorInvalidValue;
    if (j < 0) return hipErrorInvalidValue;
    dim3 grid = red_grid(n, ncol, rw);
    with_j(j, [&](auto jc) {
        hipLaunchKernelGGL((k_gcr_orth<T, decltype(jc)::value>), grid, dim3(kBlock), 0, st, W, wstride, w, r, n, g, rw);
    }, std::make_integer_sequence<int, 17>{});
    hipLaunchKernelGGL(k_fin_gcr_orth, dim3(ncol), dim3(kBlock), 0, st, rw, (int)grid.x, g, j);
    return hipGetLastError();
}
template <typename T>
hipError_t gcr_rupdate(const cpx<T>* w, cpx<T>* r, cpx<T>* copy, int j, size_t n, int ncol,
                       bool want_norm, const GcrDev& g, const RedWork& rw, hipStream_t st) {
    dim3 grid = want_norm ? red_grid(n, ncol, rw) : ew_grid(n, ncol);
    hipLaunchKernelGGL(k_gcr_rupdate<T>, grid, dim3(kBlock), 0, st, w, r, copy, j, n, want_norm ? 1 : 0, g, rw);
    if (want_norm)
        hipLaunchKernelGGL(k_fin_store, dim3(ncol), dim3(kBlock), 0, st, rw, 1, (int)grid.x, g.rr, (size_t)1);
    return hipGetLastError();
}
template <typename T>
hipError_t gcr_fused_step(const cpx<T>* W, size_t wstride, int j, cpx<T>* w, cpx<T>* r, cpx<T>* copy, size_t n,
                          int ncol, double tol2, const int* stop_in, int* stop_out, const GcrDev& g,
                          const RedWork& rw, hipStream_t st) {
    if (j < 0 || j > 15 || 2 * j + 3 > kGcrTot || 2 * j + 3 > rw.max_q) return hipErrorInvalidValue;
    const dim3 grid = red_grid(n, ncol, rw);
    auto launch = [&](auto jc) {
        constexpr int J = decltype(jc)::value;
        hipLaunchKernelGGL((k_gcr_dots<T, J>), grid, dim3(kBlock), 0, st, W, wstride, w, r, n, stop_in, rw);
        hipLaunchKernelGGL(k_fin_store_q1, dim3(2 * J + 3, ncol), dim3(64), 0, st, rw, (int)grid.x, g.tot,
                           (size_t)kGcrTot);
        hipLaunchKernelGGL((k_gcr_fused_update<T, J>), ew_grid(n, ncol), dim3(kBlock), 0, st, W, wstride, w, r,
                           copy, n, tol2, stop_in, stop_out, g);
    };
    with_j(j, launch, std::make_integer_sequence<int, 16>{});
    return hipGetLastError();
}
template <typename T>
hipError_t gcr_gram_step(const cpx<T>* W, size_t wstride, int j, const cpx<T>* r0, cpx<T>* out, size_t n, int ncol,
                         double tol2, const int* stop_in, int* stop_out, const GcrDev& g, const RedWork& rw,
                         hipStream_t st) {
    if (j < 0 || j >= kGramMax || 2 * j + 3 > kGcrTot || 2 * j + 3 > rw.max_q || j >= g.kmax) return hipErrorInvalidValue;
    // at most kGramPartials multi-dot blocks: the finaliser's waves each add that many partials
    dim3 grid = red_grid(n, ncol, rw);
    grid.x = std::min(grid.x, (unsigned)kGramPartials);
    auto launch = [&](auto jc) {
        constexpr int J = decltype(jc)::value;
        hipLaunchKernelGGL((k_gcr_dots<T, J>), grid, dim3(kBlock), 0, st, W, wstride, W + (size_t)J * wstride, r0, n,
                           stop_in, rw);
        hipLaunchKernelGGL(k_fin_gram<J>, dim3(ncol), dim3(64 * (2 * J + 3)), 0, st, rw, (int)grid.x, stop_in, stop_out,
                           g, tol2, 0);
        hipLaunchKernelGGL((k_gcr_gram_step<T, J>), ew_grid(n, ncol), dim3(kBlock), 0, st, W, wstride, r0, out, n,
                           stop_in, g);
    };
    with_j(j, launch, std::make_integer_sequence<int, kGramMax>{});
    return hipGetLastError();
}
template <typename T>
hipError_t gcr_gram_last(cpx<T>* P, const cpx<T>* W, size_t stride_v, int k, cpx<T>* x, size_t n, int ncol,
                         double tol2, const int* stop_in, int* stop_out, const GcrDev& g, const RedWork& rw,
                         hipStream_t st) {
    const int j = k - 1;
    if (j < 0 || j >= kGramMax || 2 * j + 3 > kGcrTot || 2 * j + 3 > rw.max_q || j >= g.kmax) return hipErrorInvalidValue;
    dim3 grid = red_grid(n, ncol, rw);
    grid.x = std::min(grid.x, (unsigned)kGramPartials);
    auto launch = [&](auto jc) {
        constexpr int J = decltype(jc)::value;
        hipLaunchKernelGGL((k_gcr_dots<T, J>), grid, dim3(kBlock), 0, st, W, stride_v, W + (size_t)J * stride_v, P, n,
                           stop_in, rw);
        hipLaunchKernelGGL(k_fin_gram<J>, dim3(ncol), dim3(64 * (2 * J + 3)), 0, st, rw, (int)grid.x, stop_in, stop_out,
                           g, tol2, 1);
        hipLaunchKernelGGL((k_gcr_gram_last<T, J + 1>), ew_grid(n, ncol), dim3(kBlock), 0, st, P, W, stride_v, x, n,
                           stop_out, g, ncol);
    };
    with_j(j, launch, std::make_integer_sequence<int, kGramMax>{});
    return hipGetLastError();
}
template <typename T>
hipError_t gcr_restart(const cpx<T>* r, cpx<T>* P0, size_t n, int ncol, const int* stop_src, const GcrDev& g,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_gcr_restart<T>, ew_grid(n * ncol, 1), dim3(kBlock), 0, st, r, P0, n * ncol, stop_src, g.stop,
                       ncol);
    return hipGetLastError();
}
hipError_t gcr_dev_init(int ncol, const GcrDev& g, hipStream_t st) {
    hipLaunchKernelGGL(k_gcr_dev_init, dim3(grid_for(ncol, 64)), dim3(64), 0, st, ncol, g);
    return hipGetLastError();
}
hipError_t gcr_solve(int k, int ncol, const GcrDev& g, hipStream_t st) {
    hipLaunchKernelGGL(k_gcr_solve, dim3(grid_for(ncol, 64)), dim3(64), 0, st, k, ncol, g);
    return hipGetLastError();
}
template <typename T, typename Tx>
void launch_xupdate(const cpx<T>* P, size_t pstride, int k, cpx<Tx>* x, size_t n, int ncol, bool accumulate,
                    const GcrDev& g, int solve, const cpx<T>* rsrc, cpx<T>* p0dst, const int* stop_src,
                    hipStream_t st) {
    with_j(k, [&](auto kc) {
        hipLaunchKernelGGL((k_gcr_xupdate<T, Tx, decltype(kc)::value>), ew_grid(n, ncol), dim3(kBlock), 0, st, P,
                           pstride, x, n, accumulate ? 1 : 0, g, solve, rsrc, p0dst, stop_src, ncol);
    }, std::make_integer_sequence<int, 17>{});
}
template <typename T, typename Tx>
hipError_t gcr_xupdate(const cpx<T>* P, size_t pstride, int k, cpx<Tx>* x, size_t n, int ncol,
                       bool accumulate, const GcrDev& g, hipStream_t st) {
    if (k < 0 || k > 16) return hipErrorInvalidValue;
    launch_xupdate<T, Tx>(P, pstride, k, x, n, ncol, accumulate, g, 0, nullptr, nullptr, nullptr, st);
    return hipGetLastError();
}
template <typename T, typename Tx>
hipError_t gcr_solve_xupdate(const cpx<T>* P, size_t pstride, int k, cpx<Tx>* x, size_t n, int ncol,
                             bool accumulate, const GcrDev& g, hipStream_t st) {
    if (k < 0 || k > 16) return hipErrorInvalidValue;
    // (the substitution is serial in every block: beyond 8 directions the separate
    // one-thread kernel is cheaper, measured with 16)
    if (k > 8) {
        if (hipError_t e = gcr_solve(k, ncol, g, st)) return e;
        return gcr_xupdate<T, Tx>(P, pstride, k, x, n, ncol, accumulate, g, st);
    }
    launch_xupdate<T, Tx>(P, pstride, k, x, n, ncol, accumulate, g, 1, nullptr, nullptr, nullptr, st);
    return hipGetLastError();
}
template <typename T>
hipError_t gcr_solve_xupdate_restart(cpx<T>* P, size_t pstride, int k, cpx<T>* x, size_t n, int ncol, const cpx<T>* r,
                                     const int* stop_src, const GcrDev& g, hipStream_t st) {
    if (k < 0 || k > 16) return hipErrorInvalidValue;
    if (k > 8) {
        if (hipError_t e = gcr_solve_xupdate<T, T>(P, pstride, k, x, n, ncol, true, g, st)) return e;
        return gcr_restart<T>(r, P, n, ncol, stop_src, g, st);
    }
    launch_xupdate<T, T>(P, pstride, k, x, n, ncol, true, g, 1, r, P, stop_src, st);
    return hipGetLastError();
}

// ------------------------------------------------------------ finiteness check
template <typename T>
__global__ void k_check_finite(const cpx<T>* x, size_t n, int* flag) {
    bool bad = false;
    GRID_STRIDE(i, n) {
        cpx<T> a = x[i];
        if (isnan(a.re) || isnan(a.im) || isinf(a.re) || isinf(a.im)) bad = true;
    }
    if (bad) flag[0] = 1;
}
template <typename T>
hipError_t check_finite(const cpx<T>* x, size_t n, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_check_finite<T>, ew_grid(n, 1), dim3(kBlock), 0, st, x, n, flag);
    return hipGetLastError();
}

// ------------------------------------------------------------ instantiations
#define INST_T(T)                                                                                       \
    template hipError_t vzero<T>(cpx<T>*, size_t, hipStream_t);                                         \
    template hipError_t vsub<T>(const cpx<T>*, const cpx<T>*, cpx<T>*, size_t, hipStream_t);            \
    template hipError_t norm2<T>(const cpx<T>*, size_t, int, double*, const RedWork&, hipStream_t);     \
    template hipError_t cdot<T>(const cpx<T>*, const cpx<T>*, size_t, int, double*, const RedWork&, hipStream_t); \
    template hipError_t cg_init<T>(const cpx<T>*, size_t, int, CgScal*, double, const RedWork&, hipStream_t); \
    template hipError_t cg_alpha<T>(const cpx<T>*, size_t, int, CgScal*, const RedWork&, hipStream_t); \
    template hipError_t cg_update_xr<T>(cpx<T>*, cpx<T>*, const cpx<T>*, const cpx<T>*, size_t, int, const CgScal*, hipStream_t); \
    template hipError_t cg_beta<T>(const cpx<T>*, size_t, int, CgScal*, int, const RedWork&, hipStream_t); \
    template hipError_t cg_update_p<T>(cpx<T>*, const cpx<T>*, size_t, int, const CgScal*, hipStream_t); \
    template hipError_t gcr_multidot<T>(const cpx<T>*, size_t, int, const cpx<T>*, size_t, int, const GcrDev&, const RedWork&, hipStream_t); \
    template hipError_t gcr_orth<T>(const cpx<T>*, size_t, int, cpx<T>*, const cpx<T>*, size_t, int, const GcrDev&, const RedWork&, hipStream_t); \
    template hipError_t gcr_rupdate<T>(const cpx<T>*, cpx<T>*, cpx<T>*, int, size_t, int, bool, const GcrDev&, const RedWork&, hipStream_t); \
    template hipError_t gcr_fused_step<T>(const cpx<T>*, size_t, int, cpx<T>*, cpx<T>*, cpx<T>*, size_t, int, double, const int*, int*, const GcrDev&, const RedWork&, hipStream_t); \
    template hipError_t gcr_restart<T>(const cpx<T>*, cpx<T>*, size_t, int, const int*, const GcrDev&, hipStream_t); \
    template hipError_t check_finite<T>(const cpx<T>*, size_t, int*, hipStream_t);

INST_T(float)
INST_T(double)

template hipError_t vconvert<double, float>(const cpx<double>*, cpx<float>*, size_t, hipStream_t);
template hipError_t vconvert<float, double>(const cpx<float>*, cpx<double>*, size_t, hipStream_t);
template hipError_t vconvert<double, double>(const cpx<double>*, cpx<double>*, size_t, hipStream_t);
template hipError_t vconvert<float, float>(const cpx<float>*, cpx<float>*, size_t, hipStream_t);
template hipError_t vadd<float, double>(const cpx<float>*, cpx<double>*, size_t, hipStream_t);
template hipError_t vadd<double, double>(const cpx<double>*, cpx<double>*, size_t, hipStream_t);
template hipError_t vadd<float, float>(const cpx<float>*, cpx<float>*, size_t, hipStream_t);
template hipError_t gcr_xupdate<float, float>(const cpx<float>*, size_t, int, cpx<float>*, size_t, int, bool, const GcrDev&, hipStream_t);
template hipError_t gcr_xupdate<double, double>(const cpx<double>*, size_t, int, cpx<double>*, size_t, int, bool, const GcrDev&, hipStream_t);
template hipError_t gcr_xupdate<float, double>(const cpx<float>*, size_t, int, cpx<double>*, size_t, int, bool, const GcrDev&, hipStream_t);
template hipError_t gcr_solve_xupdate<float, float>(const cpx<float>*, size_t, int, cpx<float>*, size_t, int, bool, const GcrDev&, hipStream_t);
template hipError_t gcr_solve_xupdate<double, double>(const cpx<double>*, size_t, int, cpx<double>*, size_t, int, bool, const GcrDev&, hipStream_t);
template hipError_t gcr_gram_step<float>(const cpx<float>*, size_t, int, const cpx<float>*, cpx<float>*, size_t, int, double, const int*, int*, const GcrDev&, const RedWork&, hipStream_t);
template hipError_t gcr_gram_step<double>(const cpx<double>*, size_t, int, const cpx<double>*, cpx<double>*, size_t, int, double, const int*, int*, const GcrDev&, const RedWork&, hipStream_t);
template hipError_t gcr_gram_last<float>(cpx<float>*, const cpx<float>*, size_t, int, cpx<float>*, size_t, int, double, const int*, int*, const GcrDev&, const RedWork&, hipStream_t);
template hipError_t gcr_gram_last<double>(cpx<double>*, const cpx<double>*, size_t, int, cpx<double>*, size_t, int, double, const int*, int*, const GcrDev&, const RedWork&, hipStream_t);
template hipError_t gcr_solve_xupdate_restart<float>(cpx<float>*, size_t, int, cpx<float>*, size_t, int, const cpx<float>*, const int*, const GcrDev&, hipStream_t);
template hipError_t gcr_solve_xupdate_restart<double>(cpx<double>*, size_t, int, cpx<double>*, size_t, int, const cpx<double>*, const int*, const GcrDev&, hipStream_t);

}  // namespace dwf
