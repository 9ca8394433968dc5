// Coarse domain-wall operator on the matrix cores (BF16 or FP16 links, FP32
// accumulation).
//
// Per coarse site the Galerkin stencil is a dense block contraction
//   out[i][c] = sum_{d,k} Y_d[i][k] psi_d[k][c]        (d: site and 4 neighbours,
//                                                       c: coarse slice x right-hand side)
// with complex entries.  In real arithmetic, with the inner index split as
// (k, re/im), the link rows are used as stored (interleaved complex) and the
// vector side takes the two forms
//   [Re out | Im out] = [Yr Yi] . [[ psi_r, psi_i], [-psi_i, psi_r]],
// so one 16x16x32 matrix instruction covers 16 rows x 8 complex columns x 16
// complex inner entries.  The vector is split into two 16-bit parts (hi + lo)
// and multiplied twice, so the operator applied is the rounded link matrix
// acting on a vector carried to about twice the 16-bit mantissa; products are
// exact in FP32 and accumulate in FP32.  With FP16 the staged vector of each
// (site, column tile) is first scaled by a power of two that brings its
// largest entry near 1 (exact, undone in the epilogue), which keeps FP16 in
// range whatever the magnitude of the Krylov vectors.
//
// Work split: one wavefront per (coarse site, 16-row tile), one workgroup per
// site.  A wave loads all of its link fragments up front (a site's own link
// elements are read once per apply, the backward hops' from the neighbours'
// forward links, mostly in L2; all loads in flight together) and keeps them in
// registers while
// it walks the column tiles (8 columns, or 4 or 2 when there are at most that
// many).  The
// five neighbour vectors of a column tile are staged once per site in LDS,
// already split and in both forms above (each entry converted by one thread,
// instead of every reading lane rearranging its fragments), and read back as
// 16-byte fragments; the staging loads are branch-free (dead columns read a
// valid address and are zeroed) so that the compiler keeps them all in flight.
//
// Links layout for this kernel: only the site term and the two forward hops are
// stored.  The Galerkin operator of a gamma_5-hermitian fine operator with a
// chirally doubled prolongator is sigma_3-hermitian link by link: the hop from
// x back to x - mu is sigma_3 Y_{x-mu,+mu}^dagger sigma_3 (every fine hop across
// the face between the two aggregates appears in both, reversed).  The
// backward hops are therefore read from the neighbour's forward links,
// transposed by the load pattern, conjugated and signed on the bits, which cuts
// the link bytes of a launch from 5 n^2 to 3 n^2 per site (a neighbour's links
// are usually still in L2 from the wave that read them as its own).
// Stored in fragment order, so that every own-link load of a wave reads 1 KB
// contiguous: [site][row tile m][inner step ks][lane][4] with lane = q + 16 kg
// holding row 16 m + q, inner entries j = 16 ks + 4 kg + e of the row
// [h*n + k] (h: 0 site term, 1 hop +x, 2 hop +y; k: column of that hop's
// block), each a complex 16-bit pair (re low, im high).  The site-local terms
// (the M5 + 1 shift and the fifth-dimension hops through hatP_pm with the -m
// corners, eq. coarsenDW) and sigma_3 for the adjoint (hat-D_W^dagger =
// sigma_3 hat-D_W sigma_3) are applied in the epilogue.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <type_traits>

#include "kernels.hpp"

namespace dwf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

template <bool F16> struct Half;
template <> struct Half<false> {   // bfloat16
    // round to nearest even by the hardware conversion (branch-free)
    static __device__ __forceinline__ uint32_t bits(float x) {
        return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)x);
    }
    static __device__ __forceinline__ float value(uint32_t b) { return __uint_as_float(b << 16); }
    static __device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                       0, 0, 0);
    }
};
template <> struct Half<true> {    // binary16
    static __device__ __forceinline__ uint32_t bits(float x) {
        return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)x);
    }
    static __device__ __forceinline__ float value(uint32_t b) {
        return (float)__builtin_bit_cast(_Float16, (unsigned short)(b & 0xffffu));
    }
    static __device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    }
};

template <typename T>
__device__ __forceinline__ void load4(const cpx<T>* p, float (&re)[4], float (&im)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const cpx<T> v = p[e];
        re[e] = (float)v.re;
        im[e] = (float)v.im;
    }
}

}  // namespace

template <bool F16, typename TI, typename TO, int N, bool DAG, int TW>
__global__ void __launch_bounds__(256)
coarse_mfma_kernel(const u32x4* __restrict__ links, const cpx<TI>* __restrict__ in, cpx<TO>* __restrict__ out,
                   const int* __restrict__ skip, int sks, int Lx, int Ly, int Ls, int nsites, int ncol,
                   float cdiag, float mwrap, int tpb) {
    using HF = Half<F16>;
    constexpr int MT = N / 16;                    // row tiles = waves per site
    constexpr int SPB = 1;                        // sites per block (measured: one is best)
    constexpr int KS = 5 * N / 16;                // inner steps of 16 complex entries
    constexpr int KS3 = 3 * N / 16;               // stored inner steps (site term, +x, +y)
    constexpr int H = N / 2;                      // chirality boundary (sigma_3)
    static_assert(H % 4 == 0, "the four output rows of a lane share their chirality");
    constexpr int SLAB = 5 * TW * N;              // LDS entries per site, part and form (d, c8, k)
    constexpr int PER = (SLAB + MT * 64 - 1) / (MT * 64);   // staged entries per thread (the last may be partial)
    // staged vectors as B fragments, [site][hi/lo][form][(d*TW + c8)*N + k], each entry a
    // complex 16-bit pair in the order the matrix instruction takes it: form 0 feeds the
    // real-output columns ([re, -im]), form 1 the imaginary-output columns ([im, re]), so
    // the lanes read their operands ready-made
    // (padded to PER * MT * 64 entries: the last round of staging writes needs no guard)
    // Per wave, sT: the neighbours' forward-hop fragments of its backward hops, as
    // 16 x 16 matrices of complex 16-bit pairs with row stride 20 words (the
    // transposed reads of a wavefront then fall in distinct banks).  With several
    // column tiles the transpose is done once before the tile loop and sT shares
    // its memory with sB; with one tile both are live across the same barrier.
    constexpr int SBW = SPB * 2 * 2 * PER * MT * 64;   // words of sB
    constexpr int TS = 16 * 20;
    constexpr int STW = SPB * MT * 2 * MT * TS;       // words of sT
    constexpr bool SHARE = (TW == 8);
    __shared__ __attribute__((aligned(16))) uint32_t smem[SHARE ? (SBW > STW ? SBW : STW) : SBW + STW];
    auto& sB = *reinterpret_cast<uint32_t (*)[SPB][2][2][PER * MT * 64]>(smem);
    auto& sT = *reinterpret_cast<uint32_t (*)[SPB * MT][2][MT][TS]>(smem + (SHARE ? 0 : SBW));
    __shared__ float smax[SPB][MT];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = wave / MT, m = wave - sl * MT;
    const int site = (int)xcd_block(blockIdx.x, gridDim.x) * SPB + sl;
    const bool valid_site = site < nsites;
    const int C = Ls * ncol;
    const int q = lane & 15, kg = lane >> 4;
    const bool imag_col = q >= 8;
    const int form = imag_col ? 1 : 0;

    int nb[5] = {0, 0, 0, 0, 0};
    if (valid_site) {
        const int x = site % Lx, y = site / Lx;
        const int xp = (x + 1 == Lx) ? 0 : x + 1, xm = (x == 0) ? Lx - 1 : x - 1;
        const int yp = (y + 1 == Ly) ? 0 : y + 1, ym = (y == 0) ? Ly - 1 : y - 1;
        nb[0] = site; nb[1] = y * Lx + xp; nb[2] = y * Lx + xm; nb[3] = yp * Lx + x; nb[4] = ym * Lx + x;
    }

    // all link fragments of this wave's 16 rows, loaded once (32-bit offsets from
    // the uniform base pointers: the launcher keeps every array under 4 GiB; a site
    // past the end reads site 0 and computes nothing that is stored).
    // Hop order d: 0 site, 1 +x, 2 -x, 3 +y, 4 -y; inner step ks = d * MT + kb.
    u32x4 a[KS];
    auto load_links = [&]() {
        const uint32_t own = ((uint32_t)nb[0] * MT + m) * KS3 * 64 + lane;
#pragma unroll
        for (int kb = 0; kb < MT; ++kb) {
            a[0 * MT + kb] = links[own + (0 * MT + kb) * 64];
            a[1 * MT + kb] = links[own + (1 * MT + kb) * 64];
            a[3 * MT + kb] = links[own + (2 * MT + kb) * 64];
        }
        // backward hop entry [i][k] = s_i s_k conj(Y_fwd(neighbour)[k][i]), i = 16 m + q,
        // k = 16 kb + 4 kg + e.  The neighbour's fragments (row tile kb, inner step of
        // the forward hop's column block m) are loaded as stored, 1 KB contiguous per
        // wave load, and transposed through LDS below.  The conjugation and s_k are
        // folded into the staged vector forms and s_i into the epilogue, so that the
        // transposed words feed the matrix instruction unchanged.
#pragma unroll
        for (int kb = 0; kb < MT; ++kb) {
            a[2 * MT + kb] = links[(((uint32_t)nb[2] * MT + kb) * KS3 + 1 * MT + m) * 64 + lane];
            a[4 * MT + kb] = links[(((uint32_t)nb[4] * MT + kb) * KS3 + 2 * MT + m) * 64 + lane];
        }
    };
    // transpose of the backward-hop fragments: each lane writes its stored row piece
    // (row q, entries 4 kg..4 kg+3 of the 16 x 16 block) and, after the block barrier
    // that follows, reads entries [4 kg + e][q], e = 0..3 (row k, column i)
    auto put_bwd = [&]() {
#pragma unroll
        for (int kb = 0; kb < MT; ++kb) {
            *reinterpret_cast<u32x4*>(&sT[wave][0][kb][q * 20 + 4 * kg]) = a[2 * MT + kb];
            *reinterpret_cast<u32x4*>(&sT[wave][1][kb][q * 20 + 4 * kg]) = a[4 * MT + kb];
        }
    };
    auto get_bwd = [&]() {
#pragma unroll
        for (int kb = 0; kb < MT; ++kb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                a[2 * MT + kb][e] = sT[wave][0][kb][(4 * kg + e) * 20 + q];
                a[4 * MT + kb][e] = sT[wave][1][kb][(4 * kg + e) * 20 + q];
            }
    };
    // Memory counters complete in issue order, so a wait for one load is a wait for
    // every older one.  With several column tiles the links come first (every tile
    // needs them); with one tile they are issued after the flag and staging loads,
    // so that the waits before the LDS writes leave them in flight.
    if (TW == 8) {
        load_links();
        put_bwd();
        __syncthreads();
        get_bwd();
        __syncthreads();   // sT is sB from here on
    }

    // the launcher takes tiles of 2 or 4 columns only when they hold every column:
    // then the tile loop is straight-line code (a loop would make the compiler wait
    // for the link loads at its head, before the first staging load is issued)
    const int ntile = (TW < 8) ? 1 : (C + TW - 1) / TW;
    // tiles tpb * blockIdx.y .. of this workgroup (with TW < 8 the one tile)
    const int t_lo = (TW < 8) ? 0 : (int)blockIdx.y * tpb;
    const int t_hi = (TW < 8) ? 1 : min(ntile, t_lo + tpb);
    const int tid_in_site = threadIdx.x - sl * MT * 64;
    for (int t = t_lo; t < t_hi; ++t) {
        const int cbase = TW * t;
        // live columns of the tile: lanes c8 < TW read one flag each, a ballot
        // makes the mask (the same for the whole wavefront).  Issued first, so
        // that waiting for it does not wait for the loads below.  Every lane loads
        // (straight-line code): lanes past TW or past the end read a valid repeat,
        // and without flags a word of the input is read and ignored.
        const int cf = (lane < TW && cbase + lane < C) ? cbase + lane : 0;
        const int* fp = skip ? skip + (uint32_t)(cf / Ls) * sks : reinterpret_cast<const int*>(in);
        const int flag = *fp & (skip ? -1 : 0);
        const bool lane_live = lane < TW && cbase + lane < C && flag == 0;
        // the site-local terms of this lane's outputs: column cbase + q % 8 (a column
        // past the end reads column 0 and is not written), rows i0..i0+3, slice s and
        // its fifth-dimension neighbour so
        const int cl = (cbase + (q & 7) < C) ? cbase + (q & 7) : 0;
        const int rhs = cl / Ls, s = cl - rhs * Ls;
        const int i0 = 16 * m + 4 * kg;
        const bool minus = (i0 >= H);
        const bool from_up = DAG ? !minus : minus;
        int so;
        float f = 1.f;
        if (from_up) { so = s + 1; if (so == Ls) { so = 0; f = mwrap; } }
        else         { so = s - 1; if (so < 0) { so = Ls - 1; f = mwrap; } }
        // stage the five neighbour vectors of columns cbase..cbase+TW-1, entries
        // e = (d * TW + c8) * N + k.  The loads do not depend on the column flags
        // (columns past the end read column 0), so all of them are in flight
        // together; dead columns are zeroed afterwards.
        cpx<TI> v[PER];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = min(tid_in_site + p * MT * 64, SLAB - 1);   // (past the end: a repeat, not stored)
            const int k = e % N;
            const int c8 = (e / N) % TW, d = (e / N) / TW;
            const int c = (cbase + c8 < C) ? cbase + c8 : 0;
            v[p] = in[((uint32_t)c * nsites + nb[d]) * N + k];
        }
        // the site-local terms (a site past the end reads site 0): with one tile last
        // in this group, since the compiler converts them as soon as they arrive and
        // waiting for them then finds every other load issued; with several tiles in
        // the epilogue, by the writing lanes only (measured faster there)
        float cr[4], ci[4], hr[4], hi[4];
        // (only lanes of an existing column slot load: with tiles of 2 or 4 columns
        // the others would repeat column 0, and every lane address costs the address
        // unit a cycle share; the rest take zeros)
        auto load_local = [&]() {
#pragma unroll
            for (int e = 0; e < 4; ++e) { cr[e] = ci[e] = hr[e] = hi[e] = 0.f; }
            if ((q & 7) < TW) {
                load4<TI>(in + ((uint32_t)cl * nsites + nb[0]) * N + i0, cr, ci);
                load4<TI>(in + ((uint32_t)(rhs * Ls + so) * nsites + nb[0]) * N + i0, hr, hi);
            }
        };
        if (TW < 8) {
            load_links();
            load_local();
        }
        // keep the uses below (the ballot first) from being scheduled above the loads
        __builtin_amdgcn_sched_barrier(0);
        const unsigned live = (unsigned)(__ballot(lane_live) & ((1ull << TW) - 1));
        auto col_ok = [&](int c) { return ((live >> (c - cbase)) & 1u) != 0; };
        float vr[PER], vi[PER];
        float mx = 0.f;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = min(tid_in_site + p * MT * 64, SLAB - 1);
            const int k = e % N;
            const int c8 = (e / N) % TW, d = (e / N) / TW;
            const bool bwd = (d == 2 || d == 4);
            // dead columns zeroed and on the bits (exact; selects on loaded values would
            // again become branches) the sign s_k: sigma_3 of the adjoint, and for the
            // backward hops sigma_3 of the sigma_3-adjoint links
            const uint32_t keep = (valid_site && col_ok(cbase + c8)) ? 0xffffffffu : 0u;
            const uint32_t sign = (k >= H && DAG != bwd) ? 0x80000000u : 0u;
            const float re = __uint_as_float((__float_as_uint((float)v[p].re) & keep) ^ (sign & keep));
            const float im = __uint_as_float((__float_as_uint((float)v[p].im) & keep) ^ (sign & keep));
            vr[p] = re;
            vi[p] = im;
            if (F16) mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
        float scale = 1.f, unscale = 1.f;
        if (F16) {
            for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
            if (lane == 0) smax[sl][m] = mx;
            __syncthreads();
            float smx = 0.f;
#pragma unroll
            for (int w = 0; w < MT; ++w) smx = fmaxf(smx, smax[sl][w]);
            if (smx > 0.f) {
                int ex;
                frexpf(smx, &ex);            // smx in [2^(ex-1), 2^ex)
                scale = ldexpf(1.f, -ex);    // scaled maximum in [1/2, 1)
                unscale = ldexpf(1.f, ex);
            }
        }
        // (straight-line: written for every site and slot, zeros where the site or the
        // column is dead, so that no load is sunk into a branch)
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = tid_in_site + p * MT * 64;   // LDS slot (d * TW + c8) * N + k
            const int d = (min(e, SLAB - 1) / N) / TW;
            // forward hops (links as stored): [re, -im] and [im, re]; backward hops
            // (conjugated links): [re, im] and [im, -re]
            const uint32_t x0 = (d == 2 || d == 4) ? 0u : 0x8000u, x1 = x0 ^ 0x8000u;
            const float re = vr[p] * scale, im = vi[p] * scale;
            const uint32_t hre = HF::bits(re), him = HF::bits(im);
            const uint32_t lre = HF::bits(re - HF::value(hre)), lim = HF::bits(im - HF::value(him));
            sB[sl][0][0][e] = hre | ((him ^ x0) << 16);
            sB[sl][0][1][e] = him | ((hre ^ x1) << 16);
            sB[sl][1][0][e] = lre | ((lim ^ x0) << 16);
            sB[sl][1][1][e] = lim | ((lre ^ x1) << 16);
        }
        if (TW < 8) put_bwd();
        __syncthreads();
        if (TW < 8) get_bwd();
        // (with TW < 8 the B columns TW..7 repeat staged columns and feed only unused outputs)
        // forward hops and site term in acc, backward hops in acb (their row sign s_i
        // is applied below)
        // With one tile the site-local terms start the accumulator: this lane's part
        // (real for q < 8, imaginary for q >= 8, picked on the bits) of
        // cdiag psi_s + f psi_so, scaled by 1 / unscale and the adjoint's row sign
        // (both exact), so that the epilogue needs no load of its own.
        const float osg = (DAG && minus) ? -1.f : 1.f;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f}, acb = {0.f, 0.f, 0.f, 0.f};
        if (TW < 8) {
            const uint32_t mre = imag_col ? 0u : 0xffffffffu;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float lr = cdiag * cr[e] + f * hr[e], li = cdiag * ci[e] + f * hi[e];
                const float l = __uint_as_float((__float_as_uint(lr) & mre) | (__float_as_uint(li) & ~mre));
                acc[e] = l * scale * osg;
            }
        }
        {   // (unconditional, so that no load feeding it is sunk into a branch; a dead
            // site multiplies zeros and stores nothing)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int d = (ks * 16) / N;
                const int kd = (ks * 16) % N + 4 * kg;
                const int off = (d * TW + (q & 7) % TW) * N + kd;
                const u32x4 uh = *reinterpret_cast<const u32x4*>(&sB[sl][0][form][off]);
                const u32x4 ul = *reinterpret_cast<const u32x4*>(&sB[sl][1][form][off]);
                if (d == 2 || d == 4) {
                    acb = HF::mma(a[ks], uh, acb);
                    acb = HF::mma(a[ks], ul, acb);
                } else {
                    acc = HF::mma(a[ks], uh, acc);
                    acc = HF::mma(a[ks], ul, acc);
                }
            }
        }
        {
            const float si = minus ? -1.f : 1.f;   // rows i0..i0+3 share the chirality
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] += si * acb[e];
        }
        // lanes q and q^8 hold the real and imaginary parts of the same outputs
        f32x4 p;
#pragma unroll
        for (int e = 0; e < 4; ++e) p[e] = __shfl_xor(acc[e], 8, 64);
        const bool wr = valid_site && !imag_col && col_ok(cbase + (q & 7));
        if (wr) {
            cpx<TO>* dst = out + ((uint32_t)cl * nsites + site) * N + i0;
            const float u = unscale * osg;
            if (TW == 8) {   // several tiles: the site-local terms are loaded here, by the writing lanes
                load_local();
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    dst[e] = {(TO)(acc[e] * u + cdiag * cr[e] + f * hr[e]), (TO)(p[e] * u + cdiag * ci[e] + f * hi[e])};
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) dst[e] = {(TO)(acc[e] * u), (TO)(p[e] * u)};
            }
        }
        __syncthreads();   // sB and smax are rewritten for the next column tile
    }
}

namespace {

template <bool F16, typename TI, typename TO, int N>
hipError_t launch_n(const void* links, const cpx<TI>* in, cpx<TO>* out, const CoarseGeom& g, int ncol, double m,
                    double M5, bool dagger, const int* skip, int sks, int tw, int tpb, hipStream_t st) {
    constexpr int MT = N / 16;
    constexpr int SPB = 1;
    const int nsites = g.Lx * g.Ly;
    const int C = g.Ls * ncol;
    if ((tw == 2 && C > 2) || (tw == 4 && C > 4) || (tw != 2 && tw != 4 && tw != 8) || tpb < 1)
        return hipErrorInvalidValue;
    const int ntile = (tw < 8) ? 1 : (C + tw - 1) / tw;
    const int gy = (tw < 8) ? 1 : (ntile + tpb - 1) / tpb;
    dim3 grid((nsites + SPB - 1) / SPB, gy), block(64 * MT * SPB);
    const u32x4* lk = reinterpret_cast<const u32x4*>(links);
    const float cd = (float)(M5 + 1.0), mw = (float)(-m);
    // the kernel indexes the vectors and links with 32-bit offsets
    const double vec_bytes = (double)g.Ls * ncol * nsites * N * std::max(sizeof(cpx<TI>), sizeof(cpx<TO>));
    const double link_bytes = (double)nsites * 3 * N * N * 4;
    if (vec_bytes >= 4294967296.0 || link_bytes >= 4294967296.0) return hipErrorInvalidValue;
#define DWF_COARSE_LAUNCH(TWV)                                                                                        \
    do {                                                                                                              \
        if (dagger) hipLaunchKernelGGL((coarse_mfma_kernel<F16, TI, TO, N, true, TWV>), grid, block, 0, st, lk, in,  \
                                       out, skip, sks, g.Lx, g.Ly, g.Ls, nsites, ncol, cd, mw, tpb);                  \
        else        hipLaunchKernelGGL((coarse_mfma_kernel<F16, TI, TO, N, false, TWV>), grid, block, 0, st, lk, in, \
                                       out, skip, sks, g.Lx, g.Ly, g.Ls, nsites, ncol, cd, mw, tpb);                  \
    } while (0)
    if (tw == 2) DWF_COARSE_LAUNCH(2);        // one tile of 2 columns (one rhs on 2 coarse slices)
    else if (tw == 4) DWF_COARSE_LAUNCH(4);   // one tile of 4 columns
    else DWF_COARSE_LAUNCH(8);                // tiles of 8 columns, tpb of them per workgroup
#undef DWF_COARSE_LAUNCH
    return hipGetLastError();
}

template <bool F16, typename TI, typename TO>
hipError_t launch_p(const void* links, const cpx<TI>* in, cpx<TO>* out, const CoarseGeom& g, int ncol, double m,
                    double M5, bool dagger, const int* skip, int sks, int tw, int tpb, hipStream_t st) {
    switch (g.n) {
        case 16: return launch_n<F16, TI, TO, 16>(links, in, out, g, ncol, m, M5, dagger, skip, sks, tw, tpb, st);
        case 32: return launch_n<F16, TI, TO, 32>(links, in, out, g, ncol, m, M5, dagger, skip, sks, tw, tpb, st);
        case 48: return launch_n<F16, TI, TO, 48>(links, in, out, g, ncol, m, M5, dagger, skip, sks, tw, tpb, st);
        case 64: return launch_n<F16, TI, TO, 64>(links, in, out, g, ncol, m, M5, dagger, skip, sks, tw, tpb, st);
        default: return hipErrorInvalidValue;
    }
}

// Launch configuration (tile width TW, tiles per workgroup) chosen by timing the
// candidates once per coarse shape, column count, precisions and adjoint flag,
// as the fine stencil's is (DWF_AUTOTUNE=0 keeps the heuristic).  The heuristic:
// the narrowest tile that holds every column, all tiles in one workgroup.
// Tile widths 2 and 4 start the accumulator with the site-local terms, width 8 adds
// them after the hops, so the two can differ by FP32 rounding (far below the split
// vector's 2^-16); configurations of one width agree bit for bit.
constexpr int kTpbStride = 1024;
inline int pack_cfg(int tw, int tpb) { return tw * kTpbStride + tpb; }
inline int heuristic_cfg(int C) {
    const int tw = C <= 2 ? 2 : (C <= 4 ? 4 : 8);
    return pack_cfg(tw, tw < 8 ? 1 : (C + 7) / 8);
}

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

std::string tune_key(bool f16, size_t tsz, const CoarseGeom& g, int ncol, bool dagger) {
    char k[128];
    std::snprintf(k, sizeof k, "coarse_mfma/%d/%zu/%d/%d/%d/%d/%d/%d", f16 ? 1 : 0, tsz, g.n, g.Lx, g.Ly, g.Ls, ncol,
                  dagger ? 1 : 0);
    return k;
}

// (key: the vector size, or input size * 100 + output size when the two differ)
template <typename TI, typename TO>
constexpr size_t vec_key() {
    return std::is_same<TI, TO>::value ? sizeof(TI) : sizeof(TI) * 100 + sizeof(TO);
}

template <bool F16, typename TI, typename TO>
int choose_cfg(const void* links, const cpx<TI>* in, cpx<TO>* out, const CoarseGeom& g, int ncol, double m, double M5,
               bool dagger, hipStream_t st) {
    const int C = g.Ls * ncol;
    const int heur = heuristic_cfg(C);
    const char* en = std::getenv("DWF_AUTOTUNE");
    if (en && en[0] == '0') return heur;
    const std::string key = tune_key(F16, vec_key<TI, TO>(), g, ncol, dagger);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        return it != g_tune_cache.end() ? it->second : heur;
    }
    std::lock_guard<std::recursive_mutex> rlk(runtime_mutex());
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) return it->second;
    std::vector<int> cand;
    if (C <= 2) cand.push_back(pack_cfg(2, 1));
    if (C <= 4) cand.push_back(pack_cfg(4, 1));
    const int ntile8 = (C + 7) / 8;
    for (int tpb : {ntile8, (ntile8 + 1) / 2, (ntile8 + 3) / 4, 1}) {
        const int c = pack_cfg(8, tpb);
        if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    }
    int best = heur;
    if (cand.size() > 1) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return heur;
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return heur; }
        float best_t = 1e30f, heur_t = 1e30f;
        for (int c : cand) {
            const int tw = c / kTpbStride, tpb = c % kTpbStride;
            if (launch_p<F16, TI, TO>(links, in, out, g, ncol, m, M5, dagger, nullptr, 1, tw, tpb, st) != hipSuccess)
                continue;
            float tc = 1e30f;
            for (int trial = 0; trial < 3; ++trial) {
                (void)hipEventRecord(e0, st);
                for (int r = 0; r < 10; ++r)
                    (void)launch_p<F16, TI, TO>(links, in, out, g, ncol, m, M5, dagger, nullptr, 1, tw, tpb, st);
                (void)hipEventRecord(e1, st);
                (void)hipEventSynchronize(e1);
                float t = 0.f;
                if (hipEventElapsedTime(&t, e0, e1) == hipSuccess && t < tc) tc = t;
            }
            if (c == heur) heur_t = tc;
            if (tc < best_t) { best_t = tc; best = c; }
        }
        if (heur_t < 1e30f && heur_t <= 1.03f * best_t) best = heur;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    g_tune_cache[key] = best;
    return best;
}

}  // namespace

bool coarse_mfma_supported(int n, int link_prec) {
    return (link_prec == P_BF16 || link_prec == P_F16) && (n % 16) == 0 && n <= 64;
}

template <typename TI, typename TO>
hipError_t coarse_apply_mfma_io(const void* links, int link_prec, const cpx<TI>* in, cpx<TO>* out, const CoarseGeom& g,
                                int ncol, double m, double M5, bool dagger, const int* skip, int sks, hipStream_t st) {
    if (link_prec == P_F16) {
        const int c = choose_cfg<true, TI, TO>(links, in, out, g, ncol, m, M5, dagger, st);
        return launch_p<true, TI, TO>(links, in, out, g, ncol, m, M5, dagger, skip, sks, c / kTpbStride,
                                      c % kTpbStride, st);
    }
    const int c = choose_cfg<false, TI, TO>(links, in, out, g, ncol, m, M5, dagger, st);
    return launch_p<false, TI, TO>(links, in, out, g, ncol, m, M5, dagger, skip, sks, c / kTpbStride, c % kTpbStride,
                                   st);
}

template <typename T>
hipError_t coarse_apply_mfma(const void* links, int link_prec, const cpx<T>* in, cpx<T>* out, const CoarseGeom& g,
                             int ncol, double m, double M5, bool dagger, const int* skip, int sks, hipStream_t st) {
    return coarse_apply_mfma_io<T, T>(links, link_prec, in, out, g, ncol, m, M5, dagger, skip, sks, st);
}

bool coarse_mfma_config(int link_prec, int vec_prec, const CoarseGeom& g, int ncol, bool dagger, int* tw, int* tpb) {
    if (!coarse_mfma_supported(g.n, link_prec)) return false;
    const size_t tsz = (vec_prec == P_F32) ? sizeof(float) : sizeof(double);
    const std::string key = tune_key(link_prec == P_F16, tsz, g, ncol, dagger);
    int c = heuristic_cfg(g.Ls * ncol);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) c = it->second;
    }
    *tw = c / kTpbStride;
    *tpb = c % kTpbStride;
    return true;
}

size_t links_fragment16_entries(int nsites, int n) { return (size_t)nsites * 3 * n * n; }

// FP64 column layout blk[d][k][i] (d: 0 site, 1 +x, 2 -x, 3 +y, 4 -y) -> fragment order
// [site][m][ks][lane][e] of the site term and the forward hops, complex 16-bit pairs
// (round to nearest even); see the layout note at the top of this file
__global__ void k_links_fragment16(const cpx<double>* in, uint32_t* out, int nsites, int n, int f16) {
    const long long total = (long long)nsites * 3 * n * n;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int ks_n = 3 * n / 16;
    const int e = (int)(t & 3);
    const int lane = (int)((t >> 2) & 63);
    const long long frag = t >> 8;                     // (site * (n/16) + m) * ks_n + ks
    const int ks = (int)(frag % ks_n);
    const long long sm = frag / ks_n;
    const int m = (int)(sm % (n / 16));
    const int site = (int)(sm / (n / 16));
    const int i = 16 * m + (lane & 15);
    const int j = 16 * ks + 4 * (lane >> 4) + e;
    const int h = j / n, k = j - h * n;
    const int d = (h == 2) ? 3 : h;                    // stored hops: site, +x, +y
    const cpx<double> v = in[(((size_t)site * 5 + d) * n + k) * n + i];
    uint32_t re, im;
    if (f16) {
        re = (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)v.re);
        im = (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)v.im);
    } else {
        re = f32_to_bf16_bits((float)v.re);
        im = f32_to_bf16_bits((float)v.im);
    }
    out[t] = re | (im << 16);
}

hipError_t convert_links_fragment16(const cpx<double>* in, void* out, int link_prec, int nsites, int n, hipStream_t st) {
    if (n % 16) return hipErrorInvalidValue;
    const long long total = (long long)links_fragment16_entries(nsites, n);
    hipLaunchKernelGGL(k_links_fragment16, dim3(grid_for(total)), dim3(kBlock), 0, st, in, (uint32_t*)out, nsites, n,
                       link_prec == P_F16 ? 1 : 0);
    return hipGetLastError();
}

template hipError_t coarse_apply_mfma<float>(const void*, int, const cpx<float>*, cpx<float>*, const CoarseGeom&, int, double, double, bool, const int*, int, hipStream_t);
template hipError_t coarse_apply_mfma_io<double, float>(const void*, int, const cpx<double>*, cpx<float>*, const CoarseGeom&, int, double, double, bool, const int*, int, hipStream_t);
template hipError_t coarse_apply_mfma_io<float, double>(const void*, int, const cpx<float>*, cpx<double>*, const CoarseGeom&, int, double, double, bool, const int*, int, hipStream_t);
template hipError_t coarse_apply_mfma<double>(const void*, int, const cpx<double>*, cpx<double>*, const CoarseGeom&, int, double, double, bool, const int*, int, hipStream_t);

}  // namespace dwf
