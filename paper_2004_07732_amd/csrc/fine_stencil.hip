// Fine-level operators: 2-d Wilson kernel with U(1) links (Sec. 2), the Shamir
// domain-wall operator D_DW(m) of eq. DWoperator, the Pauli-Villars operator
// D_PV = D_DW(1), and their adjoints.
//
// Layout: fields [ncol][Ls][Ly][Lx] of 2-spinors (one 16-byte load per site in
// FP32, two in FP64); links [2][Ly][Lx].  One thread owns one 2-d site of one
// column and walks a chunk of consecutive slices, keeping psi_{s-1}, psi_s and
// psi_{s+1} in registers: the fifth-dimension hop never re-reads memory and the
// two links of the site are loaded once per chunk.  The four spatial
// neighbours are read through the L1/L2 caches (consecutive threads own
// consecutive x, so a wavefront reads whole rows).
//
// In 2-d every Wilson hop goes through a rank-1 spin projector (1 -+ gamma_mu)/2,
// so a hop is one complex projection, one complex link multiply and a
// reconstruction of the second component (a fixed phase of the first).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace dwf {

template <typename R, bool DAG>
__device__ __forceinline__ void wilson_hops(const spinor<R>& fx, const spinor<R>& bx,
                                            const spinor<R>& fy, const spinor<R>& by,
                                            cpx<R> hu0, cpx<R> hu0m, cpx<R> hu1, cpx<R> hu1m,
                                            cpx<R>& a0, cpx<R>& a1) {
    // hu* hold U/2 (forward) and U/2 of the backward neighbour (conjugated here).
    // Non-adjoint: forward x uses (1 - s1)/2, backward x (1 + s1)/2,
    //              forward y (1 - s2)/2, backward y (1 + s2)/2.  The adjoint swaps.
    cpx<R> h;
    if (!DAG) {
        h = cmul(hu0, fx.c0 - fx.c1);            a0 = a0 + h; a1 = a1 - h;
        h = cjmul(hu0m, bx.c0 + bx.c1);          a0 = a0 + h; a1 = a1 + h;
        h = cmul(hu1, fy.c0 + mul_i(fy.c1));     a0 = a0 + h; a1 = a1 - mul_i(h);
        h = cjmul(hu1m, by.c0 - mul_i(by.c1));   a0 = a0 + h; a1 = a1 + mul_i(h);
    } else {
        h = cmul(hu0, fx.c0 + fx.c1);            a0 = a0 + h; a1 = a1 + h;
        h = cjmul(hu0m, bx.c0 - bx.c1);          a0 = a0 + h; a1 = a1 - h;
        h = cmul(hu1, fy.c0 - mul_i(fy.c1));     a0 = a0 + h; a1 = a1 + mul_i(h);
        h = cjmul(hu1m, by.c0 + mul_i(by.c1));   a0 = a0 + h; a1 = a1 - mul_i(h);
    }
}

// out = D psi  (RESID: out = b - D psi).  DW selects the domain-wall operator
// (diagonal D_W(M5)+1 plus the fifth-dimension hop); otherwise a stack of
// independent 2-d Wilson fields D_W(M).  `diag` = d + M5 + 1 or d + M,
// `mwrap` = -m (the corner blocks of eq. DWoperator).
template <typename R, bool DAG, bool DW, bool RESID>
__global__ void __launch_bounds__(kBlock)
fine_kernel(const cpx<R>* __restrict__ U, const spinor<R>* __restrict__ in,
            spinor<R>* __restrict__ out, const spinor<R>* __restrict__ b,
            const int* __restrict__ skip, int skip_stride, int Lx, int Ly, int Ls, int nchunk, int cs,
            int nsb, R diag, R mwrap) {
    // logical workgroup -> (column, block of 2-d sites, slice chunk), chunk fastest: the chunks of
    // one block of sites share their boundary slices, and on one XCD (xcd_block) they run side by
    // side, so those slices come from L2 rather than being fetched again
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int chunk = (int)(lb % (unsigned)nchunk);
    const unsigned t = lb / (unsigned)nchunk;
    const int sb = (int)(t % (unsigned)nsb);
    const int col = (int)(t / (unsigned)nsb);
    const int V = Lx * Ly;
    const int site = sb * (int)blockDim.x + (int)threadIdx.x;
    if (site >= V) return;
    if (skip && skip[(size_t)col * skip_stride]) return;
    const int x = site % Lx, y = site / Lx;
    const int xp = (x + 1 == Lx) ? 0 : x + 1, xm = (x == 0) ? Lx - 1 : x - 1;
    const int yp = (y + 1 == Ly) ? 0 : y + 1, ym = (y == 0) ? Ly - 1 : y - 1;
    const int sxp = y * Lx + xp, sxm = y * Lx + xm, syp = yp * Lx + x, sym = ym * Lx + x;
    const R half = R(0.5);
    const cpx<R> hu0 = half * U[site], hu0m = half * U[sxm];
    const cpx<R> hu1 = half * U[V + site], hu1m = half * U[V + sym];

    const size_t colbase = (size_t)col * Ls * V;
    const spinor<R>* src = in + colbase;
    const int s0 = chunk * cs;
    const int s1 = min(s0 + cs, Ls);

    spinor<R> cur, prv, nxt;
    if (DW) {
        cur = src[(size_t)s0 * V + site];
        if (s0 == 0) {
            prv = src[(size_t)(Ls - 1) * V + site];
            prv.c0 = mwrap * prv.c0; prv.c1 = mwrap * prv.c1;
        } else {
            prv = src[(size_t)(s0 - 1) * V + site];
        }
    }
    for (int s = s0; s < s1; ++s) {
        const spinor<R>* sl = src + (size_t)s * V;
        if (DW) {
            if (s + 1 == Ls) {
                nxt = src[site];
                nxt.c0 = mwrap * nxt.c0; nxt.c1 = mwrap * nxt.c1;
            } else {
                nxt = src[(size_t)(s + 1) * V + site];
            }
        } else {
            cur = sl[site];
        }
        const spinor<R> fx = sl[sxp], bx = sl[sxm], fy = sl[syp], by = sl[sym];
        cpx<R> a0 = {R(0), R(0)}, a1 = {R(0), R(0)};
        wilson_hops<R, DAG>(fx, bx, fy, by, hu0, hu0m, hu1, hu1m, a0, a1);
        spinor<R> res;
        res.c0 = diag * cur.c0 - a0;
        res.c1 = diag * cur.c1 - a1;
        if (DW) {
            if (!DAG) {  // P_- psi_{s+1} + P_+ psi_{s-1}
                res.c1 = res.c1 + nxt.c1;
                res.c0 = res.c0 + prv.c0;
            } else {     // P_+ psi_{s+1} + P_- psi_{s-1}
                res.c0 = res.c0 + nxt.c0;
                res.c1 = res.c1 + prv.c1;
            }
        }
        const size_t o = colbase + (size_t)s * V + site;
        if (RESID) {
            const spinor<R> bb = b[o];
            res.c0 = bb.c0 - res.c0;
            res.c1 = bb.c1 - res.c1;
        }
        out[o] = res;
        if (DW) { prv = cur; cur = nxt; }
    }
}

static inline int pick_chunk(int Lx, int Ly, int Ls, int ncol) {
    // enough threads to fill 256 CUs with several waves each, but long enough
    // chunks that the fifth-dimension window amortises its two extra loads
    const long long want = 256LL * 64 * 16;
    long long sites = (long long)Lx * Ly * ncol;
    int cs = Ls;
    while (cs > 2 && sites * ((Ls + cs - 1) / cs) < want) cs = (cs + 1) / 2;
    return cs;
}

template <typename R>
static hipError_t launch_fine(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, const cpx<R>* b, int Lx, int Ly,
                              int Ls, int ncol, double m, double M5, bool dagger, const int* skip, int skip_stride,
                              int cs, hipStream_t st);

// Chunk length (slices per thread) of the fine stencil, chosen by timing the
// candidates once per shape and precision (DWF_AUTOTUNE=0 disables it); the
// choices persist in the file named by DWF_TUNE_CACHE when that is set.
template <typename R>
static int tuned_chunk(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, int Lx, int Ly, int Ls, int ncol,
                       double m, double M5, bool dagger, hipStream_t st) {
    static std::mutex mu;
    static std::map<std::string, int> cache;
    static bool loaded = false;
    const int heuristic = pick_chunk(Lx, Ly, Ls, ncol);
    const char* en = std::getenv("DWF_AUTOTUNE");
    if (en && en[0] == '0') return heuristic;
    char keyb[128];
    std::snprintf(keyb, sizeof keyb, "fine_dw/%zu/%d/%d/%d/%d/%d", sizeof(R), Lx, Ly, Ls, ncol, dagger ? 1 : 0);
    const std::string key(keyb);
    // inside a graph capture: use a choice already made, never time
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        return it != cache.end() ? it->second : heuristic;
    }
    // the timing runs synchronise: keep them apart from captures on other threads
    std::lock_guard<std::recursive_mutex> rlk(runtime_mutex());
    std::lock_guard<std::mutex> lk(mu);
    const char* path = std::getenv("DWF_TUNE_CACHE");
    if (!loaded) {
        loaded = true;
        if (path) {
            std::ifstream f(path);
            std::string k;
            int v;
            while (f >> k >> v) cache[k] = v;
        }
    }
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    std::vector<int> cand;
    for (int c : {Ls, (Ls + 1) / 2, (Ls + 3) / 4, 8, 4, 2})
        if (c >= 1 && c <= Ls && std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return heuristic;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return heuristic; }
    int best = heuristic;
    float best_t = 1e30f;
    for (int c : cand) {
        (void)launch_fine<R>(U, in, out, nullptr, Lx, Ly, Ls, ncol, m, M5, dagger, nullptr, 1, c, st);
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 5; ++r)
            (void)launch_fine<R>(U, in, out, nullptr, Lx, Ly, Ls, ncol, m, M5, dagger, nullptr, 1, c, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float t = 0.f;
        if (hipEventElapsedTime(&t, e0, e1) == hipSuccess && t < best_t) { best_t = t; best = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cache[key] = best;
    if (path) {
        std::ofstream f(path, std::ios::app);
        f << key << " " << best << "\n";
    }
    return best;
}

template <typename R>
hipError_t fine_dw(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, const cpx<R>* b,
                   int Lx, int Ly, int Ls, int ncol, double m, double M5, bool dagger,
                   const int* skip, int skip_stride, hipStream_t st) {
    const int cs = tuned_chunk<R>(U, in, out, Lx, Ly, Ls, ncol, m, M5, dagger, st);
    return launch_fine<R>(U, in, out, b, Lx, Ly, Ls, ncol, m, M5, dagger, skip, skip_stride, cs, st);
}

template <typename R>
static hipError_t launch_fine(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, const cpx<R>* b, int Lx, int Ly,
                              int Ls, int ncol, double m, double M5, bool dagger, const int* skip, int skip_stride,
                              int cs, hipStream_t st) {
    const int nchunk = (Ls + cs - 1) / cs;
    const int nsb = (Lx * Ly + kBlock - 1) / kBlock;
    const long long nblocks = (long long)nsb * nchunk * ncol;
    const R diag = R(2.0 + M5 + 1.0), mwrap = R(-m);
    auto* si = reinterpret_cast<const spinor<R>*>(in);
    auto* so = reinterpret_cast<spinor<R>*>(out);
    auto* sb = reinterpret_cast<const spinor<R>*>(b);
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblocks), block(kBlock);
    if (b) {
        if (dagger) hipLaunchKernelGGL((fine_kernel<R, true, true, true>), grid, block, 0, st, U, si, so, sb, skip, skip_stride, Lx, Ly, Ls, nchunk, cs, nsb, diag, mwrap);
        else        hipLaunchKernelGGL((fine_kernel<R, false, true, true>), grid, block, 0, st, U, si, so, sb, skip, skip_stride, Lx, Ly, Ls, nchunk, cs, nsb, diag, mwrap);
    } else {
        if (dagger) hipLaunchKernelGGL((fine_kernel<R, true, true, false>), grid, block, 0, st, U, si, so, sb, skip, skip_stride, Lx, Ly, Ls, nchunk, cs, nsb, diag, mwrap);
        else        hipLaunchKernelGGL((fine_kernel<R, false, true, false>), grid, block, 0, st, U, si, so, sb, skip, skip_stride, Lx, Ly, Ls, nchunk, cs, nsb, diag, mwrap);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t wilson2d(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, int Lx, int Ly, int ncol,
                    double M, bool dagger, hipStream_t st) {
    // each column is an independent 2-d field: treat columns as slices of one
    // column with no fifth-dimension coupling
    const int Ls = ncol, cs = 1, nchunk = ncol;
    const int nsb = (Lx * Ly + kBlock - 1) / kBlock;
    const long long nblocks = (long long)nsb * nchunk;
    const R diag = R(2.0 + M), mwrap = R(0);
    auto* si = reinterpret_cast<const spinor<R>*>(in);
    auto* so = reinterpret_cast<spinor<R>*>(out);
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblocks), block(kBlock);
    if (dagger) hipLaunchKernelGGL((fine_kernel<R, true, false, false>), grid, block, 0, st, U, si, so, nullptr, nullptr, 1, Lx, Ly, Ls, nchunk, cs, nsb, diag, mwrap);
    else        hipLaunchKernelGGL((fine_kernel<R, false, false, false>), grid, block, 0, st, U, si, so, nullptr, nullptr, 1, Lx, Ly, Ls, nchunk, cs, nsb, diag, mwrap);
    return hipGetLastError();
}

template hipError_t fine_dw<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, const cpx<float>*, int, int, int, int, double, double, bool, const int*, int, hipStream_t);
template hipError_t fine_dw<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, const cpx<double>*, int, int, int, int, double, double, bool, const int*, int, hipStream_t);
template hipError_t wilson2d<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, int, int, int, double, bool, hipStream_t);
template hipError_t wilson2d<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, int, int, int, double, bool, hipStream_t);

}  // namespace dwf
