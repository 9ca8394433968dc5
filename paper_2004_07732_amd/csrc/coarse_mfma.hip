// Coarse domain-wall operator on the matrix cores (BF16 links, FP32 accumulation).
//
// Per coarse site the Galerkin stencil is a dense block contraction
//   out[i][c] = sum_{d,k} Y_d[i][k] psi_d[k][c]        (d: site and 4 neighbours,
//                                                       c: coarse slice x right-hand side)
// with complex entries.  In real arithmetic, with the inner index split as
// (k, re/im), the link rows are used as stored (interleaved complex) and the
// vector side is rebuilt on the fly:
//   [Re out | Im out] = [Yr Yi] . [[ psi_r, psi_i], [-psi_i, psi_r]],
// so one v_mfma_f32_16x16x32_bf16 covers 16 rows x 8 complex columns x 16
// complex inner entries.  The vector is split into two BF16 parts (hi + lo)
// and multiplied twice, so the operator applied is the BF16-rounded link
// matrix acting on a vector carried to about 16 mantissa bits; products are
// exact in FP32 and accumulate in FP32.  One wavefront owns one coarse site
// and up to 64 complex columns; each link element is read once per apply.
//
// Links layout for this kernel: per site, row-major [i][d*n + k] complex BF16.
// The site-local terms (the M5 + 1 shift and the fifth-dimension hops through
// hatP_pm with the -m corners, eq. coarsenDW) and sigma_3 for the adjoint
// (hat-D_W^dagger = sigma_3 hat-D_W sigma_3) are applied in the epilogue.
#include "kernels.hpp"

namespace dwf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

template <typename T>
__device__ __forceinline__ void load4(const cpx<T>* p, float (&re)[4], float (&im)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const cpx<T> v = p[e];
        re[e] = (float)v.re;
        im[e] = (float)v.im;
    }
}

__device__ __forceinline__ void split(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

}  // namespace

template <typename T, int N, int NTMAX, bool DAG>
__global__ void __launch_bounds__(256)
coarse_mfma_kernel(const bf16x8* __restrict__ links, const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                   const int* __restrict__ skip, int sks, int Lx, int Ly, int Ls, int nsites, int ncol,
                   float cdiag, float mwrap) {
    constexpr int MT = N / 16;          // row tiles
    constexpr int KS = 5 * N / 16;      // inner steps of 16 complex entries
    constexpr int H = N / 2;            // chirality boundary (sigma_3)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int site = blockIdx.x * 4 + wave;
    if (site >= nsites) return;         // no block-level synchronisation in this kernel
    const int C = Ls * ncol;            // complex columns
    const int c0 = blockIdx.y * 8 * NTMAX;
    const int q = lane & 15, kg = lane >> 4;

    const int x = site % Lx, y = site / Lx;
    const int xp = (x + 1 == Lx) ? 0 : x + 1, xm = (x == 0) ? Lx - 1 : x - 1;
    const int yp = (y + 1 == Ly) ? 0 : y + 1, ym = (y == 0) ? Ly - 1 : y - 1;
    const int nb[5] = {site, y * Lx + xp, y * Lx + xm, yp * Lx + x, ym * Lx + x};

    // column owned by this lane in tile t (B operand and epilogue)
    auto col_of = [&](int t) { return c0 + 8 * t + (q & 7); };
    auto col_ok = [&](int c) {
        if (c >= C) return false;
        return !(skip && skip[(size_t)(c / Ls) * sks]);
    };

    f32x4 acc[MT][NTMAX];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTMAX; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    // link rows of this site: row i starts at (site*N + i) * 5N complex = (site*N + i) * 5N/4 chunks
    const bf16x8* lrow = links + ((size_t)site * N + q) * (5 * N / 4);

#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int d = (ks * 16) / N;
        const int kd = (ks * 16) % N + 4 * kg;     // first of this lane's 4 complex inner entries
        bf16x8 a[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) a[m] = lrow[(size_t)m * 16 * (5 * N / 4) + ks * 4 + kg];
        const int nbs = nb[d];
        const bool neg = DAG && (kd >= H);
#pragma unroll
        for (int t = 0; t < NTMAX; ++t) {
            const int c = col_of(t);
            bf16x8 bh, bl;
            if (col_ok(c)) {
                float re[4], im[4];
                load4<T>(in + ((size_t)c * nsites + nbs) * N + kd, re, im);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (neg) { re[e] = -re[e]; im[e] = -im[e]; }
                    __bf16 rh, rl, ih, il, nih, nil;
                    split(re[e], rh, rl);
                    split(im[e], ih, il);
                    split(-im[e], nih, nil);
                    if (q < 8) {   // real part of the output: [re, -im] per inner entry
                        bh[2 * e] = rh; bh[2 * e + 1] = nih;
                        bl[2 * e] = rl; bl[2 * e + 1] = nil;
                    } else {       // imaginary part: [im, re]
                        bh[2 * e] = ih; bh[2 * e + 1] = rh;
                        bl[2 * e] = il; bl[2 * e + 1] = rl;
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) { bh[e] = (__bf16)0.f; bl[e] = (__bf16)0.f; }
            }
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bh, acc[m][t], 0, 0, 0);
                acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bl, acc[m][t], 0, 0, 0);
            }
        }
    }

    // epilogue: lanes q and q^8 hold the real and imaginary parts of the same outputs
#pragma unroll
    for (int t = 0; t < NTMAX; ++t) {
        const int c = col_of(t);
        const bool ok = (q < 8) && col_ok(c);
        const int rhs = c / Ls, s = c - rhs * Ls;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            f32x4 v = acc[m][t], p;
#pragma unroll
            for (int e = 0; e < 4; ++e) p[e] = __shfl_xor(v[e], 8, 64);
            if (!ok) continue;
            const int i0 = 16 * m + 4 * kg;
            const bool minus = (i0 >= H);
            // fifth-dimension neighbour slice for these rows
            const bool from_up = DAG ? !minus : minus;
            int so;
            float f = 1.f;
            if (from_up) { so = s + 1; if (so == Ls) { so = 0; f = mwrap; } }
            else         { so = s - 1; if (so < 0) { so = Ls - 1; f = mwrap; } }
            float cr[4], ci[4], hr[4], hi[4];
            load4<T>(in + ((size_t)c * nsites + site) * N + i0, cr, ci);
            load4<T>(in + ((size_t)(rhs * Ls + so) * nsites + site) * N + i0, hr, hi);
            cpx<T>* dst = out + ((size_t)c * nsites + site) * N + i0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float re = v[e], im = p[e];
                if (DAG && minus) { re = -re; im = -im; }
                re += cdiag * cr[e] + f * hr[e];
                im += cdiag * ci[e] + f * hi[e];
                dst[e] = {(T)re, (T)im};
            }
        }
    }
}

namespace {

template <typename T, int N, int NTMAX>
hipError_t launch_nt(const void* links, const cpx<T>* in, cpx<T>* out, const CoarseGeom& g, int ncol, double m,
                     double M5, bool dagger, const int* skip, int sks, hipStream_t st) {
    const int nsites = g.Lx * g.Ly;
    const int C = g.Ls * ncol;
    dim3 grid((nsites + 3) / 4, (C + 8 * NTMAX - 1) / (8 * NTMAX)), block(256);
    const bf16x8* lk = reinterpret_cast<const bf16x8*>(links);
    const float cd = (float)(M5 + 1.0), mw = (float)(-m);
    if (dagger) hipLaunchKernelGGL((coarse_mfma_kernel<T, N, NTMAX, true>), grid, block, 0, st, lk, in, out, skip, sks, g.Lx, g.Ly, g.Ls, nsites, ncol, cd, mw);
    else        hipLaunchKernelGGL((coarse_mfma_kernel<T, N, NTMAX, false>), grid, block, 0, st, lk, in, out, skip, sks, g.Lx, g.Ly, g.Ls, nsites, ncol, cd, mw);
    return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_n(const void* links, const cpx<T>* in, cpx<T>* out, const CoarseGeom& g, int ncol, double m,
                    double M5, bool dagger, const int* skip, int sks, hipStream_t st) {
    const int tiles = (g.Ls * ncol + 7) / 8;
    if (tiles <= 1) return launch_nt<T, N, 1>(links, in, out, g, ncol, m, M5, dagger, skip, sks, st);
    if (tiles <= 2) return launch_nt<T, N, 2>(links, in, out, g, ncol, m, M5, dagger, skip, sks, st);
    if (tiles <= 4) return launch_nt<T, N, 4>(links, in, out, g, ncol, m, M5, dagger, skip, sks, st);
    return launch_nt<T, N, 8>(links, in, out, g, ncol, m, M5, dagger, skip, sks, st);
}

}  // namespace

bool coarse_mfma_supported(int n, int link_prec) { return link_prec == P_BF16 && (n % 16) == 0 && n <= 64; }

template <typename T>
hipError_t coarse_apply_mfma(const void* links, const cpx<T>* in, cpx<T>* out, const CoarseGeom& g, int ncol,
                             double m, double M5, bool dagger, const int* skip, int sks, hipStream_t st) {
    switch (g.n) {
        case 16: return launch_n<T, 16>(links, in, out, g, ncol, m, M5, dagger, skip, sks, st);
        case 32: return launch_n<T, 32>(links, in, out, g, ncol, m, M5, dagger, skip, sks, st);
        case 48: return launch_n<T, 48>(links, in, out, g, ncol, m, M5, dagger, skip, sks, st);
        case 64: return launch_n<T, 64>(links, in, out, g, ncol, m, M5, dagger, skip, sks, st);
        default: return hipErrorInvalidValue;
    }
}

// FP64 column layout blk[k][i] -> row-major [i][d*n + k] complex BF16 (round to nearest even)
__global__ void k_links_rowmajor_bf16(const cpx<double>* in, cbf16* out, int nsites, int n) {
    const long long total = (long long)nsites * 5 * n * n;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    // output index t = ((site*n + i)*5 + d)*n + k
    const int k = (int)(t % n);
    const int d = (int)((t / n) % 5);
    const int i = (int)((t / (5LL * n)) % n);
    const int site = (int)(t / (5LL * n * n));
    const cpx<double> v = in[(((size_t)site * 5 + d) * n + k) * n + i];
    const uint32_t re = f32_to_bf16_bits((float)v.re), im = f32_to_bf16_bits((float)v.im);
    out[t].v = re | (im << 16);
}

hipError_t convert_links_rowmajor_bf16(const cpx<double>* in, void* out, int nsites, int n, hipStream_t st) {
    const long long total = (long long)nsites * 5 * n * n;
    hipLaunchKernelGGL(k_links_rowmajor_bf16, dim3(grid_for(total)), dim3(kBlock), 0, st, in, (cbf16*)out, nsites, n);
    return hipGetLastError();
}

template hipError_t coarse_apply_mfma<float>(const void*, const cpx<float>*, cpx<float>*, const CoarseGeom&, int, double, double, bool, const int*, int, hipStream_t);
template hipError_t coarse_apply_mfma<double>(const void*, const cpx<double>*, cpx<double>*, const CoarseGeom&, int, double, double, bool, const int*, int, hipStream_t);

}  // namespace dwf
