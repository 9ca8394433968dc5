// Shared device-side types and helpers of the dwfmg HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace dwf {

// ---------------------------------------------------------------- complex
template <typename R>
struct __align__(2 * sizeof(R)) cpx {
    R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cpx<R> mkc(R a, R b) { return cpx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cpx<R> cjmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> conj(cpx<R> a) { return {a.re, -a.im}; }
// i * a
template <typename R>
__host__ __device__ __forceinline__ cpx<R> mul_i(cpx<R> a) { return {-a.im, a.re}; }
template <typename R>
__host__ __device__ __forceinline__ void cfma(cpx<R>& acc, cpx<R> a, cpx<R> b) {
    acc.re += a.re * b.re - a.im * b.im;
    acc.im += a.re * b.im + a.im * b.re;
}

// two-component spinor of one 2-d site and slice: one 16-byte (float) or two
// 16-byte (double) vector loads
template <typename R>
struct __align__(4 * sizeof(R)) spinor {
    cpx<R> c0, c1;
};

// ---------------------------------------------------------------- precision codes
enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_F16 = 3 };

inline size_t cplx_bytes(int prec) {
    switch (prec) {
        case P_F64: return 16;
        case P_F32: return 8;
        default: return 4;
    }
}

// bfloat16 complex packed in 32 bits: low half = re, high half = im
struct cbf16 { uint32_t v; };
// binary16 complex
struct cf16 { _Float16 re, im; };

__device__ __forceinline__ cpx<float> load_link(const cbf16* p, size_t i) {
    uint32_t u = p[i].v;
    return {__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u)};
}
__device__ __forceinline__ cpx<float> load_link(const cf16* p, size_t i) {
    cf16 h = p[i];
    return {(float)h.re, (float)h.im};
}
__device__ __forceinline__ cpx<float> load_link(const cpx<float>* p, size_t i) { return p[i]; }
__device__ __forceinline__ cpx<double> load_link(const cpx<double>* p, size_t i) { return p[i]; }

// round-to-nearest-even float -> bfloat16 bits
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// arithmetic type used with a given link storage type
template <typename L> struct acc_of { using type = float; };
template <> struct acc_of<cpx<double>> { using type = double; };

// ---------------------------------------------------------------- launch helpers
constexpr int kBlock = 256;

// Workgroups are dealt round-robin to the 8 XCDs (workgroup b runs on XCD
// b % 8), each with its own L2.  Stencil kernels renumber their workgroups so
// that every XCD owns one contiguous range of logical workgroups: lattice
// neighbours (the next row, the next site) are then fetched into the same L2
// instead of into three different ones.  Bijective for any grid size.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    const unsigned x = b % kXcds, k = b / kXcds, q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + k;
}

inline unsigned grid_for(long long n, int block = kBlock) {
    long long g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace dwf
