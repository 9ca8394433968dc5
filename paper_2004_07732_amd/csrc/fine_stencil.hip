// Fine-level operators: 2-d Wilson kernel with U(1) links (Sec. 2), the Shamir
// domain-wall operator D_DW(m) of eq. DWoperator, the Pauli-Villars operator
// D_PV = D_DW(1), and their adjoints.
//
// Layout: fields [ncol][Ls][Ly][Lx] of 2-spinors (one 16-byte load per site in
// FP32, two in FP64); links [2][Ly][Lx].  One thread owns one 2-d site of one
// column and walks a chunk of consecutive slices, keeping psi_{s-1}, psi_s and
// psi_{s+1} in registers: the fifth-dimension hop never re-reads memory and the
// two links of the site are loaded once per chunk.
//
// Two kernels share that walk and differ in how the four spatial neighbours
// arrive.  The tiled kernel (the one used whenever the lattice divides into its
// tiles) gives a workgroup a TX x TY tile of sites: at every slice each thread
// puts its own psi_s, which it already holds, into an LDS tile, the halo ring
// (one row above and below, one column left and right) is loaded one slice
// ahead, and the neighbours are read back from LDS after one barrier; the LDS
// tile is double-buffered so that barrier is the only one per slice.  Global
// traffic is then psi once plus the ring, instead of four neighbour loads per
// site through L1/L2, which measured about 40% slower.  The row kernel (any
// lattice) reads the neighbours through the caches.  Results are written with
// streaming (nontemporal) stores; both kernels evaluate each site with the same
// expression, so they agree bit for bit.
//
// In 2-d every Wilson hop goes through a rank-1 spin projector (1 -+ gamma_mu)/2,
// so a hop is one complex projection, one complex link multiply and a
// reconstruction of the second component (a fixed phase of the first).
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <type_traits>

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

// One site and slice of D_DW (or its adjoint): diagonal D_W(M5)+1 with the four
// hops, plus the fifth-dimension terms through P_-+ (prv and nxt already carry
// the -m of the wrap where it applies).
template <typename R, bool DAG>
__device__ __forceinline__ spinor<R> dw_site(const spinor<R>& fx, const spinor<R>& bx, const spinor<R>& fy,
                                             const spinor<R>& by, const spinor<R>& cur, const spinor<R>& prv,
                                             const spinor<R>& nxt, cpx<R> hu0, cpx<R> hu0m, cpx<R> hu1, cpx<R> hu1m,
                                             R diag) {
    cpx<R> a0 = {R(0), R(0)}, a1 = {R(0), R(0)};
    wilson_hops<R, DAG>(fx, bx, fy, by, hu0, hu0m, hu1, hu1m, a0, a1);
    spinor<R> res;
    res.c0 = diag * cur.c0 - a0;
    res.c1 = diag * cur.c1 - a1;
    if (!DAG) {  // P_- psi_{s+1} + P_+ psi_{s-1}
        res.c1 = res.c1 + nxt.c1;
        res.c0 = res.c0 + prv.c0;
    } else {     // P_+ psi_{s+1} + P_- psi_{s-1}
        res.c0 = res.c0 + nxt.c0;
        res.c1 = res.c1 + prv.c1;
    }
    return res;
}

// the four components of a spinor as one vector value: values that are loaded
// conditionally and carried across loop iterations stay in registers in this
// form (as a 32-byte FP64 struct they were kept in scratch memory)
template <typename R> struct vec4_of;
template <> struct vec4_of<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct vec4_of<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <typename R>
__device__ __forceinline__ typename vec4_of<R>::type load4(const spinor<R>* p) {
    return *reinterpret_cast<const typename vec4_of<R>::type*>(p);
}
template <typename R>
__device__ __forceinline__ spinor<R> unpack4(const typename vec4_of<R>::type& v) {
    spinor<R> r;
    r.c0 = {v[0], v[1]};
    r.c1 = {v[2], v[3]};
    return r;
}

// Output stores.  A large write-once output goes out with nontemporal stores, which
// keep it from displacing the input slices that neighbouring workgroups are still
// reading from L2; an output that fits the Infinity Cache with room to spare (the
// solver's vectors, read again by the next launch) is stored normally so that it
// stays there (kStreamStoreBytes, decided per launch).
constexpr double kStreamStoreBytes = 64.0 * 1024 * 1024;
template <bool NT>
__device__ __forceinline__ void store_out(spinor<float>* p, const spinor<float>& v) {
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    const f32x4 x = {v.c0.re, v.c0.im, v.c1.re, v.c1.im};
    if constexpr (NT) __builtin_nontemporal_store(x, reinterpret_cast<f32x4*>(p));
    else *reinterpret_cast<f32x4*>(p) = x;
}
template <bool NT>
__device__ __forceinline__ void store_out(spinor<double>* p, const spinor<double>& v) {
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    f64x2* q = reinterpret_cast<f64x2*>(p);
    const f64x2 x0 = {v.c0.re, v.c0.im}, x1 = {v.c1.re, v.c1.im};
    if constexpr (NT) {
        __builtin_nontemporal_store(x0, q);
        __builtin_nontemporal_store(x1, q + 1);
    } else {
        q[0] = x0;
        q[1] = x1;
    }
}

// out = D psi  (RESID: out = b - D psi).  DW selects the domain-wall operator
// (diagonal D_W(M5)+1 plus the fifth-dimension hop); otherwise a stack of
// independent 2-d Wilson fields D_W(M).  `diag` = d + M5 + 1 or d + M,
// `mwrap` = -m (the corner blocks of eq. DWoperator).
template <typename R, bool DAG, bool DW, bool RESID, bool NT>
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
        spinor<R> res;
        if (DW) {
            res = dw_site<R, DAG>(fx, bx, fy, by, cur, prv, nxt, hu0, hu0m, hu1, hu1m, diag);
        } else {
            cpx<R> a0 = {R(0), R(0)}, a1 = {R(0), R(0)};
            wilson_hops<R, DAG>(fx, bx, fy, by, hu0, hu0m, hu1, hu1m, a0, a1);
            res.c0 = diag * cur.c0 - a0;
            res.c1 = diag * cur.c1 - a1;
        }
        const size_t o = colbase + (size_t)s * V + site;
        if (RESID) {
            const spinor<R> bb = b[o];
            res.c0 = bb.c0 - res.c0;
            res.c1 = bb.c1 - res.c1;
        }
        store_out<NT>(out + o, res);
        if (DW) { prv = cur; cur = nxt; }
    }
}

// Tiled D_DW: a workgroup owns a TX x TY tile of 2-d sites of one column and one
// chunk of slices (same logical-workgroup order as the row kernel).  LDS holds
// the tile of the current slice with a one-site ring, double-buffered by slice
// parity.  Per slice: write own psi_s and the prefetched ring into the buffer,
// issue the loads for the next slice (ring) and the slice after it (own site),
// barrier, read the four neighbours, evaluate, store.  The buffer written at
// slice s was last read at slice s-2, before the barrier of slice s-1, so one
// barrier per slice suffices.  Requires Lx % TX == 0 and Ly % TY == 0.
template <typename R, bool DAG, bool RESID, int TX, int TY, bool NT>
__global__ void __launch_bounds__(TX * TY)
fine_tile_kernel(const cpx<R>* __restrict__ U, const spinor<R>* __restrict__ in, spinor<R>* __restrict__ out,
                 const spinor<R>* __restrict__ b, const int* __restrict__ skip, int skip_stride, int Lx, int Ly,
                 int Ls, int nchunk, int cs, int ntile, R diag, R mwrap) {
    static_assert(TX >= 2 && TY >= 2, "the ring needs two distinct edges per direction");
    __shared__ spinor<R> tile[2][TY + 2][TX + 2];
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int chunk = (int)(lb % (unsigned)nchunk);
    const unsigned t = lb / (unsigned)nchunk;
    const int tl = (int)(t % (unsigned)ntile);
    const int col = (int)(t / (unsigned)ntile);
    if (skip && skip[(size_t)col * skip_stride]) return;   // the same for the whole workgroup
    const int V = Lx * Ly;
    const int ntx = Lx / TX;
    const int x0 = (tl % ntx) * TX, y0 = (tl / ntx) * TY;
    const int lx = (int)threadIdx.x % TX, ly = (int)threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    const int site = y * Lx + x;
    const int xm = (x == 0) ? Lx - 1 : x - 1, ym = (y == 0) ? Ly - 1 : y - 1;
    const R half = R(0.5);
    const cpx<R> hu0 = half * U[site], hu0m = half * U[y * Lx + xm];
    const cpx<R> hu1 = half * U[V + site], hu1m = half * U[V + ym * Lx + x];
    // the ring (row below, row above, left column, right column; 2 TX + 2 TY
    // sites) is loaded by the first threads of the workgroup, one site each, in
    // whole wavefronts; the spare lanes of the last of those wavefronts repeat
    // its final site
    constexpr int kRing = 2 * TX + 2 * TY;
    constexpr int kRingThreads = (kRing + 63) / 64 * 64;
    static_assert(kRingThreads <= TX * TY, "the ring needs enough threads");
    const int tid = (int)threadIdx.x;
    const bool ring = tid < kRingThreads;
    int hsite = 0, hlds = 0;
    {
        const int r = min(tid, kRing - 1);
        const int ybelow = (y0 == 0) ? Ly - 1 : y0 - 1, yabove = (y0 + TY == Ly) ? 0 : y0 + TY;
        const int xleft = (x0 == 0) ? Lx - 1 : x0 - 1, xright = (x0 + TX == Lx) ? 0 : x0 + TX;
        if (r < TX) { hsite = ybelow * Lx + x0 + r; hlds = r + 1; }
        else if (r < 2 * TX) { hsite = yabove * Lx + x0 + (r - TX); hlds = (TY + 1) * (TX + 2) + (r - TX) + 1; }
        else if (r < 2 * TX + TY) { hsite = (y0 + r - 2 * TX) * Lx + xleft; hlds = (r - 2 * TX + 1) * (TX + 2); }
        else { hsite = (y0 + r - 2 * TX - TY) * Lx + xright; hlds = (r - 2 * TX - TY + 1) * (TX + 2) + TX + 1; }
    }

    const size_t colbase = (size_t)col * Ls * V;
    const spinor<R>* src = in + colbase;
    const int s0 = chunk * cs;
    const int s1 = min(s0 + cs, Ls);
    spinor<R> prv = src[(size_t)((s0 == 0) ? Ls - 1 : s0 - 1) * V + site];
    if (s0 == 0) { prv.c0 = mwrap * prv.c0; prv.c1 = mwrap * prv.c1; }
    spinor<R> cur = src[(size_t)s0 * V + site];
    spinor<R> nxt = src[(size_t)((s0 + 1 == Ls) ? 0 : s0 + 1) * V + site];
    typedef typename vec4_of<R>::type vec4;
    vec4 hv = {};
    if (ring) hv = load4(src + (size_t)s0 * V + hsite);
    for (int s = s0; s < s1; ++s) {
        spinor<R>(*bf)[TX + 2] = tile[s & 1];
        bf[ly + 1][lx + 1] = cur;
        if (ring) *reinterpret_cast<vec4*>(&bf[0][0] + hlds) = hv;
        vec4 nn = {};
        if (s + 1 < s1) {   // the same for the whole workgroup
            const int sn = (s + 1 == Ls) ? 0 : s + 1;
            const int s2 = (s + 2 >= Ls) ? s + 2 - Ls : s + 2;
            nn = load4(src + (size_t)s2 * V + site);
            if (ring) hv = load4(src + (size_t)sn * V + hsite);
        }
        __syncthreads();
        const spinor<R> fx = bf[ly + 1][lx + 2], bx = bf[ly + 1][lx], fy = bf[ly + 2][lx + 1], by = bf[ly][lx + 1];
        spinor<R> nx = nxt;
        if (s + 1 == Ls) { nx.c0 = mwrap * nx.c0; nx.c1 = mwrap * nx.c1; }
        spinor<R> res = dw_site<R, DAG>(fx, bx, fy, by, cur, prv, nx, hu0, hu0m, hu1, hu1m, diag);
        const size_t o = colbase + (size_t)s * V + site;
        if (RESID) {
            const spinor<R> bb = b[o];
            res.c0 = bb.c0 - res.c0;
            res.c1 = bb.c1 - res.c1;
        }
        store_out<NT>(out + o, res);
        prv = cur;
        cur = nxt;
        nxt = unpack4<R>(nn);
    }
}

// A launch configuration of D_DW: kernel shape (0: row kernel, k >= 1: tiled
// kernel with kTiles[k-1]) and slice-chunk length, packed as shape * 4096 + cs.
struct TileShape { int tx, ty; };
static constexpr TileShape kTiles[] = {{64, 8}, {32, 16}, {128, 4}};
static constexpr int kNumTiles = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
static constexpr int kCfgStride = 4096;

static inline bool tile_fits(int shape, int Lx, int Ly) {
    return shape >= 1 && shape <= kNumTiles && Lx % kTiles[shape - 1].tx == 0 && Ly % kTiles[shape - 1].ty == 0;
}

static inline int pick_cfg(int Lx, int Ly, int Ls, int ncol) {
    // the first tile shape that divides the lattice, else the row kernel; chunks of at
    // most 8 slices (measured best at the HBM-bound shapes), shorter while the grid
    // would not give every CU several workgroups
    const long long want = 256LL * 64 * 16;
    const long long sites = (long long)Lx * Ly * ncol;
    int shape = 0;
    for (int k = 1; k <= kNumTiles && !shape; ++k)
        if (tile_fits(k, Lx, Ly)) shape = k;
    int cs = std::min(std::min(Ls, 8), kCfgStride - 1);
    while (cs > 2 && sites * ((Ls + cs - 1) / cs) < want) cs = (cs + 1) / 2;
    return shape * kCfgStride + cs;
}

template <typename R>
static hipError_t launch_fine(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, const cpx<R>* b, int Lx, int Ly,
                              int Ls, int ncol, double m, double M5, bool dagger, const int* skip, int skip_stride,
                              int cfg, hipStream_t st);

// Launch configuration of the fine stencil (kernel shape and chunk length),
// chosen by timing the candidates once per lattice shape, column count,
// precision and adjoint flag (DWF_AUTOTUNE=0 disables it); the choices persist
// in the file named by DWF_TUNE_CACHE when that is set.
template <typename R>
static int tuned_cfg(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, int Lx, int Ly, int Ls, int ncol,
                     double m, double M5, bool dagger, hipStream_t st, bool may_time = true) {
    static std::mutex mu;
    static std::map<std::string, int> cache;
    static bool loaded = false;
    const int heuristic = pick_cfg(Lx, Ly, Ls, ncol);
    const char* en = std::getenv("DWF_AUTOTUNE");
    if (en && en[0] == '0') return heuristic;
    char keyb[128];
    std::snprintf(keyb, sizeof keyb, "fine_dw2/%zu/%d/%d/%d/%d/%d", sizeof(R), Lx, Ly, Ls, ncol, dagger ? 1 : 0);
    const std::string key(keyb);
    // inside a graph capture, or for a caller that must not synchronise: use a
    // choice already made, never time
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (!may_time || hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
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
    std::vector<int> chunks;
    for (int c : {Ls, (Ls + 1) / 2, (Ls + 3) / 4, 8, 4, 2})
        if (c >= 1 && c <= Ls && c < kCfgStride && std::find(chunks.begin(), chunks.end(), c) == chunks.end())
            chunks.push_back(c);
    std::vector<int> cand;
    for (int shape = 0; shape <= kNumTiles; ++shape)
        if (shape == 0 || tile_fits(shape, Lx, Ly))
            for (int c : chunks) cand.push_back(shape * kCfgStride + c);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return heuristic;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return heuristic; }
    // each candidate: the best of three runs of ten launches (launch-rate and cache
    // noise made single short runs pick the slower kernel now and then); the
    // heuristic choice is kept unless another is faster by more than 3%
    int best = heuristic;
    float best_t = 1e30f, heur_t = 1e30f;
    for (int c : cand) {
        if (launch_fine<R>(U, in, out, nullptr, Lx, Ly, Ls, ncol, m, M5, dagger, nullptr, 1, c, st) != hipSuccess)
            continue;
        float tc = 1e30f;
        for (int trial = 0; trial < 3; ++trial) {
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < 10; ++r)
                (void)launch_fine<R>(U, in, out, nullptr, Lx, Ly, Ls, ncol, m, M5, dagger, nullptr, 1, c, st);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float t = 0.f;
            if (hipEventElapsedTime(&t, e0, e1) == hipSuccess && t < tc) tc = t;
        }
        if (c == heuristic) heur_t = tc;
        if (tc < best_t) { best_t = tc; best = c; }
    }
    if (heur_t < 1e30f && heur_t <= 1.03f * best_t) best = heuristic;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cache[key] = best;
    if (path) {
        std::ofstream f(path, std::ios::app);
        f << key << " " << best << "\n";
    }
    return best;
}

// configuration pinned by the caller (packed as above), or -1
static std::atomic<int> g_fine_pin{-1};

bool set_fine_config(int shape, int chunk) {
    if (shape == -1) { g_fine_pin.store(-1); return true; }
    if (shape < 0 || shape > kNumTiles || chunk < 1 || chunk >= kCfgStride) return false;
    g_fine_pin.store(shape * kCfgStride + chunk);
    return true;
}

template <typename R>
static hipError_t fine_dw_impl(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, const cpx<R>* b, int Lx, int Ly,
                               int Ls, int ncol, double m, double M5, bool dagger, const int* skip, int skip_stride,
                               hipStream_t st, bool may_time) {
    const int pin = g_fine_pin.load(std::memory_order_relaxed);
    int cfg;
    if (pin >= 0 && (pin / kCfgStride == 0 || tile_fits(pin / kCfgStride, Lx, Ly)))
        cfg = (pin / kCfgStride) * kCfgStride + std::min(pin % kCfgStride, Ls);
    else
        cfg = tuned_cfg<R>(U, in, out, Lx, Ly, Ls, ncol, m, M5, dagger, st, may_time);
    return launch_fine<R>(U, in, out, b, Lx, Ly, Ls, ncol, m, M5, dagger, skip, skip_stride, cfg, st);
}

template <typename R>
hipError_t fine_dw(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, const cpx<R>* b,
                   int Lx, int Ly, int Ls, int ncol, double m, double M5, bool dagger,
                   const int* skip, int skip_stride, hipStream_t st) {
    return fine_dw_impl<R>(U, in, out, b, Lx, Ly, Ls, ncol, m, M5, dagger, skip, skip_stride, st, true);
}

template <typename R>
hipError_t fine_dw_untimed(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, int Lx, int Ly, int Ls, int ncol,
                           double m, double M5, bool dagger, hipStream_t st) {
    return fine_dw_impl<R>(U, in, out, nullptr, Lx, Ly, Ls, ncol, m, M5, dagger, nullptr, 1, st, false);
}

template <typename R, int TX, int TY>
static hipError_t launch_tile(const cpx<R>* U, const spinor<R>* si, spinor<R>* so, const spinor<R>* sb, int Lx,
                              int Ly, int Ls, int ncol, R diag, R mwrap, bool dagger, const int* skip,
                              int skip_stride, int cs, hipStream_t st) {
    if (Lx % TX || Ly % TY) return hipErrorInvalidValue;
    const int nt = (double)Lx * Ly * Ls * ncol * sizeof(spinor<R>) >= kStreamStoreBytes ? 1 : 0;
    const int nchunk = (Ls + cs - 1) / cs;
    const int ntile = (Lx / TX) * (Ly / TY);
    const long long nblocks = (long long)ntile * nchunk * ncol;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblocks), block(TX * TY);
    auto go = [&](auto dag, auto resid, auto ntc) {
        hipLaunchKernelGGL((fine_tile_kernel<R, decltype(dag)::value, decltype(resid)::value, TX, TY,
                                             decltype(ntc)::value>),
                           grid, block, 0, st, U, si, so, sb, skip, skip_stride, Lx, Ly, Ls, nchunk, cs, ntile, diag,
                           mwrap);
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (sb) {
        if (dagger) { if (nt) go(T_{}, T_{}, T_{}); else go(T_{}, T_{}, F_{}); }
        else        { if (nt) go(F_{}, T_{}, T_{}); else go(F_{}, T_{}, F_{}); }
    } else {
        if (dagger) { if (nt) go(T_{}, F_{}, T_{}); else go(T_{}, F_{}, F_{}); }
        else        { if (nt) go(F_{}, F_{}, T_{}); else go(F_{}, F_{}, F_{}); }
    }
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_fine(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, const cpx<R>* b, int Lx, int Ly,
                              int Ls, int ncol, double m, double M5, bool dagger, const int* skip, int skip_stride,
                              int cfg, hipStream_t st) {
    const int shape = cfg / kCfgStride, cs = cfg % kCfgStride;
    if (cs < 1 || shape < 0 || shape > kNumTiles) return hipErrorInvalidValue;
    const R diag = R(2.0 + M5 + 1.0), mwrap = R(-m);
    auto* si = reinterpret_cast<const spinor<R>*>(in);
    auto* so = reinterpret_cast<spinor<R>*>(out);
    auto* sb = reinterpret_cast<const spinor<R>*>(b);
    static_assert(kNumTiles == 3, "one case per tile shape");
    switch (shape) {
        case 1: return launch_tile<R, kTiles[0].tx, kTiles[0].ty>(U, si, so, sb, Lx, Ly, Ls, ncol, diag, mwrap, dagger, skip, skip_stride, cs, st);
        case 2: return launch_tile<R, kTiles[1].tx, kTiles[1].ty>(U, si, so, sb, Lx, Ly, Ls, ncol, diag, mwrap, dagger, skip, skip_stride, cs, st);
        case 3: return launch_tile<R, kTiles[2].tx, kTiles[2].ty>(U, si, so, sb, Lx, Ly, Ls, ncol, diag, mwrap, dagger, skip, skip_stride, cs, st);
        default: break;
    }
    const int nchunk = (Ls + cs - 1) / cs;
    const int nsb = (Lx * Ly + kBlock - 1) / kBlock;
    const long long nblocks = (long long)nsb * nchunk * ncol;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const int nt = (double)Lx * Ly * Ls * ncol * sizeof(spinor<R>) >= kStreamStoreBytes ? 1 : 0;
    dim3 grid((unsigned)nblocks), block(kBlock);
    auto go = [&](auto dag, auto resid, auto ntc) {
        hipLaunchKernelGGL((fine_kernel<R, decltype(dag)::value, true, decltype(resid)::value, decltype(ntc)::value>),
                           grid, block, 0, st, U, si, so, sb, skip, skip_stride, Lx, Ly, Ls, nchunk, cs, nsb, diag,
                           mwrap);
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (b) {
        if (dagger) { if (nt) go(T_{}, T_{}, T_{}); else go(T_{}, T_{}, F_{}); }
        else        { if (nt) go(F_{}, T_{}, T_{}); else go(F_{}, T_{}, F_{}); }
    } else {
        if (dagger) { if (nt) go(T_{}, F_{}, T_{}); else go(T_{}, F_{}, F_{}); }
        else        { if (nt) go(F_{}, F_{}, T_{}); else go(F_{}, F_{}, F_{}); }
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ fused A = D_PV^dag D_DW(m)
// One launch for both stencils of the fine A (eq. NormalExp): the intermediate
// t = D_DW(m) psi never goes to memory.  A workgroup owns a TX x TY tile of one column
// and a chunk [s0, s1) of output slices and walks k = s0-1 .. s1:
//  - t_k is evaluated on the tile and its one-site ring (each ring site again, from the
//    LDS box of psi_k with a two-site margin and the boxes of psi_{k-1}, psi_{k+1}) into an
//    LDS tile, so that D_PV^dag finds all four neighbours of every tile site;
//  - out_{k-1} = D_PV^dag t follows from the tile of t_{k-1} and, at the thread's own site,
//    t_{k-2} (lower chirality, from below) and t_k (upper chirality, from above);
//  - psi_{k+2}'s box is loaded while t_k is evaluated and written to LDS after it.
// Four psi boxes and two t tiles rotate, so one barrier per slice suffices: the psi box
// written at step k was last read at step k-1, the t tile written at step k was last read
// at step k-1, both before step k-1's barrier.  Every site evaluates the same expressions
// as the two separate stencil kernels (dw_site), in the same order.
// Requires Lx % TX == 0 and Ly % TY == 0.
template <typename R, int TX, int TY, bool NTS>
__global__ void __launch_bounds__(TX * TY)
fine_a_kernel(const cpx<R>* __restrict__ U, const spinor<R>* __restrict__ in, spinor<R>* __restrict__ out,
              const int* __restrict__ skip, int skip_stride, int Lx, int Ly, int Ls, int nchunk, int cs, int ntile,
              R diag, R mdw, R mpv) {
    constexpr int NTH = TX * TY;
    constexpr int BX = TX + 4, BY = TY + 4;                            // psi box: two-site margin
    constexpr int EX = TX + 2, EY = TY + 2;                            // t tile: one-site margin
    constexpr int NBOX = (TX + 2) * (TY + 2) + 2 * TX + 2 * TY;        // psi sites read per slice
    constexpr int NRING = 2 * TX + 2 * TY;                             // ring sites of t
    static_assert(NBOX <= 2 * NTH && NRING <= NTH, "two box sites and one ring site per thread at most");
    __shared__ __attribute__((aligned(16))) spinor<R> pb[4][BY][BX];
    __shared__ __attribute__((aligned(16))) spinor<R> tb[2][EY][EX];
    typedef typename vec4_of<R>::type vec4;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int chunk = (int)(lb % (unsigned)nchunk);
    const unsigned tt = lb / (unsigned)nchunk;
    const int tl = (int)(tt % (unsigned)ntile);
    const int col = (int)(tt / (unsigned)ntile);
    if (skip && skip[(size_t)col * skip_stride]) return;   // the same for the whole workgroup
    const int V = Lx * Ly;
    const int ntx = Lx / TX;
    const int x0 = (tl % ntx) * TX, y0 = (tl / ntx) * TY;
    const int tid = (int)threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    auto wx = [&](int x) { return x < 0 ? x + Lx : (x >= Lx ? x - Lx : x); };   // |offset| <= 2 < Lx
    auto wy = [&](int y) { return y < 0 ? y + Ly : (y >= Ly ? y - Ly : y); };
    const R half = R(0.5);
    // links of a site: U/2 forward, U/2 of the backward neighbour
    auto links = [&](int gx, int gy, cpx<R>& h0, cpx<R>& h0m, cpx<R>& h1, cpx<R>& h1m) {
        const int site = gy * Lx + gx;
        h0 = half * U[site];
        h0m = half * U[gy * Lx + wx(gx - 1)];
        h1 = half * U[V + site];
        h1m = half * U[V + wy(gy - 1) * Lx + gx];
    };
    const int x = x0 + lx, y = y0 + ly;
    const int site = y * Lx + x;
    cpx<R> hu0, hu0m, hu1, hu1m;
    links(x, y, hu0, hu0m, hu1, hu1m);
    // this thread's ring site of t (threads tid < NRING): row below, row above, left
    // column, right column, in tile-local coordinates
    const bool has_ring = tid < NRING;
    int rpx = 0, rpy = 0;
    {
        const int r = has_ring ? tid : 0;
        if (r < TX) { rpx = r; rpy = -1; }
        else if (r < 2 * TX) { rpx = r - TX; rpy = TY; }
        else if (r < 2 * TX + TY) { rpx = -1; rpy = r - 2 * TX; }
        else { rpx = TX; rpy = r - 2 * TX - TY; }
    }
    cpx<R> ru0 = {}, ru0m = {}, ru1 = {}, ru1m = {};
    if (has_ring) links(wx(x0 + rpx), wy(y0 + rpy), ru0, ru0m, ru1, ru1m);
    // this thread's (at most two) psi box sites: the (TX+2) x (TY+2) box, then the four
    // arms of the two-site margin (left, right, below, above)
    int gs[2] = {-1, -1}, ls[2] = {0, 0};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int i = tid + e * NTH;
        if (i < NBOX) {
            int px, py;
            if (i < (TX + 2) * (TY + 2)) { px = i % (TX + 2) - 1; py = i / (TX + 2) - 1; }
            else {
                const int j = i - (TX + 2) * (TY + 2);
                if (j < TY) { px = -2; py = j; }
                else if (j < 2 * TY) { px = TX + 1; py = j - TY; }
                else if (j < 2 * TY + TX) { px = j - 2 * TY; py = -2; }
                else { px = j - 2 * TY - TX; py = TY + 1; }
            }
            gs[e] = wy(y0 + py) * Lx + wx(x0 + px);
            ls[e] = (py + 2) * BX + (px + 2);
        }
    }
    const size_t colbase = (size_t)col * Ls * V;
    const spinor<R>* src = in + colbase;
    const int s0 = chunk * cs;
    const int s1 = min(s0 + cs, Ls);
    auto slice = [&](int k) { k %= Ls; return k < 0 ? k + Ls : k; };   // walk index -> slice
    auto buf = [&](int k) -> spinor<R>(*)[BX] { return pb[(k + 8) & 3]; };   // k >= -2
    auto load_box = [&](int k, vec4 (&a)[2]) {
        const spinor<R>* sl = src + (size_t)slice(k) * V;
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (gs[e] >= 0) a[e] = load4(sl + gs[e]);
    };
    auto put_box = [&](int k, const vec4 (&a)[2]) {
        spinor<R>* b = &buf(k)[0][0];
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (gs[e] >= 0) *reinterpret_cast<vec4*>(b + ls[e]) = a[e];
    };
    // t_k at tile-local (px, py): D_DW(m) from the psi boxes (corner blocks -m at the wrap)
    auto t_at = [&](int k, int px, int py, cpx<R> h0, cpx<R> h0m, cpx<R> h1, cpx<R> h1m) {
        const spinor<R>(*c)[BX] = buf(k);
        const spinor<R>(*pv)[BX] = buf(k - 1);
        const spinor<R>(*nx)[BX] = buf(k + 1);
        const int bx = px + 2, by = py + 2;
        spinor<R> prv = pv[by][bx], nxt = nx[by][bx];
        const int sk = slice(k);
        if (sk == 0) { prv.c0 = mdw * prv.c0; prv.c1 = mdw * prv.c1; }
        if (sk == Ls - 1) { nxt.c0 = mdw * nxt.c0; nxt.c1 = mdw * nxt.c1; }
        return dw_site<R, false>(c[by][bx + 1], c[by][bx - 1], c[by + 1][bx], c[by - 1][bx], c[by][bx], prv, nxt,
                                 h0, h0m, h1, h1m, diag);
    };
    {   // the boxes of psi_{s0-2}, psi_{s0-1}, psi_{s0}
        vec4 a[3][2] = {};
        load_box(s0 - 2, a[0]);
        load_box(s0 - 1, a[1]);
        load_box(s0, a[2]);
        put_box(s0 - 2, a[0]);
        put_box(s0 - 1, a[1]);
        put_box(s0, a[2]);
    }
    __syncthreads();
    spinor<R> tp = {}, tc = {}, tn = {};   // t at the own site, walk k-2, k-1, k
    for (int k = s0 - 1; k <= s1; ++k) {   // (the same bounds for the whole workgroup)
        vec4 a[2] = {};
        const bool pre = k + 2 <= s1 + 1;
        if (pre) load_box(k + 2, a);
        tn = t_at(k, lx, ly, hu0, hu0m, hu1, hu1m);
        spinor<R>(*tw)[EX] = tb[k & 1];
        tw[ly + 1][lx + 1] = tn;
        if (has_ring && k >= s0 && k < s1) tw[rpy + 1][rpx + 1] = t_at(k, rpx, rpy, ru0, ru0m, ru1, ru1m);
        if (k - 1 >= s0) {   // out_{k-1} = D_PV^dag t (corner blocks -1 at the wrap)
            const int so = k - 1;
            const spinor<R>(*q)[EX] = tb[so & 1];
            spinor<R> prv = tp, nxt = tn;
            if (so == 0) { prv.c0 = mpv * prv.c0; prv.c1 = mpv * prv.c1; }
            if (so == Ls - 1) { nxt.c0 = mpv * nxt.c0; nxt.c1 = mpv * nxt.c1; }
            const spinor<R> res = dw_site<R, true>(q[ly + 1][lx + 2], q[ly + 1][lx], q[ly + 2][lx + 1], q[ly][lx + 1],
                                                   tc, prv, nxt, hu0, hu0m, hu1, hu1m, diag);
            store_out<NTS>(out + colbase + (size_t)so * V + site, res);
        }
        if (pre) put_box(k + 2, a);
        tp = tc;
        tc = tn;
        __syncthreads();
    }
}

// Launch configuration of the fine A: 0 = the two stencil launches (each with its own
// configuration), else fused tile shape * kCfgStride + slice chunk
struct ATileShape { int tx, ty; };
static constexpr ATileShape kATiles[] = {{16, 16}, {32, 8}, {16, 8}};
static constexpr int kNumATiles = (int)(sizeof(kATiles) / sizeof(kATiles[0]));

// the fused kernel's LDS (four psi boxes, two t tiles) must fit one workgroup's 64 KB
template <typename R>
static constexpr bool a_tile_lds_ok(int tx, int ty) {
    return (4 * (tx + 4) * (ty + 4) + 2 * (tx + 2) * (ty + 2)) * (int)sizeof(spinor<R>) <= 64 * 1024;
}
template <typename R>
static bool a_tile_fits(int shape, int Lx, int Ly) {
    if (shape < 1 || shape > kNumATiles) return false;
    const ATileShape t = kATiles[shape - 1];
    return Lx % t.tx == 0 && Ly % t.ty == 0 && a_tile_lds_ok<R>(t.tx, t.ty);
}

template <typename R, int TX, int TY>
static hipError_t launch_a_tile(const cpx<R>* U, const spinor<R>* si, spinor<R>* so, int Lx, int Ly, int Ls,
                                int ncol, R diag, R mdw, R mpv, const int* skip, int skip_stride, int cs,
                                hipStream_t st) {
    if constexpr (!a_tile_lds_ok<R>(TX, TY)) {
        return hipErrorInvalidValue;
    } else {
        if (Lx % TX || Ly % TY || Ls < 2) return hipErrorInvalidValue;
        const int nt = (double)Lx * Ly * Ls * ncol * sizeof(spinor<R>) >= kStreamStoreBytes ? 1 : 0;
        const int nchunk = (Ls + cs - 1) / cs;
        const int ntile = (Lx / TX) * (Ly / TY);
        const long long nblocks = (long long)ntile * nchunk * ncol;
        if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
        dim3 grid((unsigned)nblocks), block(TX * TY);
        if (nt)
            hipLaunchKernelGGL((fine_a_kernel<R, TX, TY, true>), grid, block, 0, st, U, si, so, skip, skip_stride,
                               Lx, Ly, Ls, nchunk, cs, ntile, diag, mdw, mpv);
        else
            hipLaunchKernelGGL((fine_a_kernel<R, TX, TY, false>), grid, block, 0, st, U, si, so, skip, skip_stride,
                               Lx, Ly, Ls, nchunk, cs, ntile, diag, mdw, mpv);
        return hipGetLastError();
    }
}

template <typename R>
static hipError_t launch_a(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, cpx<R>* tmp, int Lx, int Ly, int Ls,
                           int ncol, double m, double M5, const int* skip, int skip_stride, int cfg, hipStream_t st,
                           bool may_time) {
    const int shape = cfg / kCfgStride, cs = cfg % kCfgStride;
    if (shape == 0) {
        hipError_t e = fine_dw_impl<R>(U, in, tmp, nullptr, Lx, Ly, Ls, ncol, m, M5, false, skip, skip_stride, st,
                                       may_time);
        if (e != hipSuccess) return e;
        return fine_dw_impl<R>(U, tmp, out, nullptr, Lx, Ly, Ls, ncol, 1.0, M5, true, skip, skip_stride, st,
                               may_time);
    }
    if (cs < 1 || !a_tile_fits<R>(shape, Lx, Ly)) return hipErrorInvalidValue;
    const R diag = R(2.0 + M5 + 1.0), mdw = R(-m), mpv = R(-1.0);
    auto* si = reinterpret_cast<const spinor<R>*>(in);
    auto* so = reinterpret_cast<spinor<R>*>(out);
    static_assert(kNumATiles == 3, "one case per fused tile shape");
    switch (shape) {
        case 1: return launch_a_tile<R, kATiles[0].tx, kATiles[0].ty>(U, si, so, Lx, Ly, Ls, ncol, diag, mdw, mpv, skip, skip_stride, cs, st);
        case 2: return launch_a_tile<R, kATiles[1].tx, kATiles[1].ty>(U, si, so, Lx, Ly, Ls, ncol, diag, mdw, mpv, skip, skip_stride, cs, st);
        case 3: return launch_a_tile<R, kATiles[2].tx, kATiles[2].ty>(U, si, so, Lx, Ly, Ls, ncol, diag, mdw, mpv, skip, skip_stride, cs, st);
        default: return hipErrorInvalidValue;
    }
}

// pinned configuration of the fine A (shape * kCfgStride + chunk), or -1 (timed choice)
static std::atomic<int> g_a_pin{-1};

bool set_fine_a_config(int shape, int chunk) {
    if (shape == -1) { g_a_pin.store(-1); return true; }
    if (shape < 0 || shape > kNumATiles || (shape > 0 && (chunk < 1 || chunk >= kCfgStride))) return false;
    g_a_pin.store(shape * kCfgStride + (shape > 0 ? chunk : 0));
    return true;
}

// the fine A's configuration, timed once per lattice shape, column count and precision
// (two launches or one fused launch per tile shape and chunk); the two launches stay
// unless a fused configuration is faster by more than 3%
static std::mutex g_a_mu;
static std::map<std::string, int> g_a_cache;

template <typename R>
static int tuned_a_cfg(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, cpx<R>* tmp, int Lx, int Ly, int Ls,
                       int ncol, double m, double M5, hipStream_t st, bool may_time) {
    std::mutex& mu = g_a_mu;
    std::map<std::string, int>& cache = g_a_cache;
    const int heuristic = 0;
    const char* en = std::getenv("DWF_AUTOTUNE");
    if (en && en[0] == '0') return heuristic;
    char keyb[128];
    std::snprintf(keyb, sizeof keyb, "fine_a/%zu/%d/%d/%d/%d", sizeof(R), Lx, Ly, Ls, ncol);
    const std::string key(keyb);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (!may_time || hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        return it != cache.end() ? it->second : heuristic;
    }
    std::lock_guard<std::recursive_mutex> rlk(runtime_mutex());
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    std::vector<int> cand = {0};
    for (int shape = 1; shape <= kNumATiles; ++shape) {
        if (!a_tile_fits<R>(shape, Lx, Ly) || Ls < 2) continue;
        std::vector<int> chunks;
        for (int c : {Ls, (Ls + 1) / 2, (Ls + 3) / 4, 4, 2})
            if (c >= 1 && c <= Ls && std::find(chunks.begin(), chunks.end(), c) == chunks.end()) chunks.push_back(c);
        for (int c : chunks) cand.push_back(shape * kCfgStride + c);
    }
    int best = heuristic;
    if (cand.size() > 1) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return heuristic;
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return heuristic; }
        float best_t = 1e30f, heur_t = 1e30f;
        for (int c : cand) {
            if (launch_a<R>(U, in, out, tmp, Lx, Ly, Ls, ncol, m, M5, nullptr, 1, c, st, true) != hipSuccess) continue;
            float tc = 1e30f;
            for (int trial = 0; trial < 3; ++trial) {
                (void)hipEventRecord(e0, st);
                for (int r = 0; r < 10; ++r)
                    (void)launch_a<R>(U, in, out, tmp, Lx, Ly, Ls, ncol, m, M5, nullptr, 1, c, st, true);
                (void)hipEventRecord(e1, st);
                (void)hipEventSynchronize(e1);
                float t = 0.f;
                if (hipEventElapsedTime(&t, e0, e1) == hipSuccess && t < tc) tc = t;
            }
            if (c == heuristic) heur_t = tc;
            if (tc < best_t) { best_t = tc; best = c; }
        }
        if (heur_t < 1e30f && heur_t <= 1.03f * best_t) best = heuristic;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    cache[key] = best;
    return best;
}

template <typename R>
hipError_t fine_a(const cpx<R>* U, const cpx<R>* in, cpx<R>* out, cpx<R>* tmp, int Lx, int Ly, int Ls, int ncol,
                  double m, double M5, const int* skip, int skip_stride, hipStream_t st) {
    const int pin = g_a_pin.load(std::memory_order_relaxed);
    int cfg;
    if (pin >= 0 && (pin / kCfgStride == 0 || (a_tile_fits<R>(pin / kCfgStride, Lx, Ly) && Ls >= 2)))
        cfg = pin / kCfgStride == 0 ? 0 : (pin / kCfgStride) * kCfgStride + std::min(pin % kCfgStride, Ls);
    else
        cfg = tuned_a_cfg<R>(U, in, out, tmp, Lx, Ly, Ls, ncol, m, M5, st, true);
    return launch_a<R>(U, in, out, tmp, Lx, Ly, Ls, ncol, m, M5, skip, skip_stride, cfg, st, true);
}

bool fine_a_chosen(int prec_bytes, int Lx, int Ly, int Ls, int ncol, int* shape, int* chunk) {
    char keyb[128];
    std::snprintf(keyb, sizeof keyb, "fine_a/%d/%d/%d/%d/%d", prec_bytes, Lx, Ly, Ls, ncol);
    std::lock_guard<std::mutex> lk(g_a_mu);
    auto it = g_a_cache.find(keyb);
    if (it == g_a_cache.end()) return false;
    *shape = it->second / kCfgStride;
    *chunk = it->second % kCfgStride;
    return true;
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
    const int nt = (double)Lx * Ly * ncol * sizeof(spinor<R>) >= kStreamStoreBytes ? 1 : 0;
    dim3 grid((unsigned)nblocks), block(kBlock);
    auto go = [&](auto dag, auto ntc) {
        hipLaunchKernelGGL((fine_kernel<R, decltype(dag)::value, false, false, decltype(ntc)::value>), grid, block, 0,
                           st, U, si, so, nullptr, nullptr, 1, Lx, Ly, Ls, nchunk, cs, nsb, diag, mwrap);
    };
    if (dagger) { if (nt) go(std::true_type{}, std::true_type{}); else go(std::true_type{}, std::false_type{}); }
    else        { if (nt) go(std::false_type{}, std::true_type{}); else go(std::false_type{}, std::false_type{}); }
    return hipGetLastError();
}

template hipError_t fine_dw<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, const cpx<float>*, int, int, int, int, double, double, bool, const int*, int, hipStream_t);
template hipError_t fine_dw<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, const cpx<double>*, int, int, int, int, double, double, bool, const int*, int, hipStream_t);
template hipError_t fine_dw_untimed<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, int, int, int, int, double, double, bool, hipStream_t);
template hipError_t fine_dw_untimed<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, int, int, int, int, double, double, bool, hipStream_t);
template hipError_t fine_a<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, cpx<float>*, int, int, int, int, double, double, const int*, int, hipStream_t);
template hipError_t fine_a<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, cpx<double>*, int, int, int, int, double, double, const int*, int, hipStream_t);
template hipError_t wilson2d<float>(const cpx<float>*, const cpx<float>*, cpx<float>*, int, int, int, double, bool, hipStream_t);
template hipError_t wilson2d<double>(const cpx<double>*, const cpx<double>*, cpx<double>*, int, int, int, double, bool, hipStream_t);

}  // namespace dwf
