// Counter-based random numbers for the MLMC sampler (device side).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): a 128-bit counter is mixed by ten rounds of two 32x32
// -> 64-bit products and xors with a 64-bit key that is bumped by the Weyl
// constants between rounds.  Keyed by the user seed, so every random number
// of an estimate is a pure function of (seed, stream, realisation, position):
// realisations can be produced in any order, by any work item, and extended
// later (the target-RMSE mode reuses its pilot realisations).
//
// Stream layout (word 3 of the counter): tag << 28 | level << 20 | problem.
//   tag 1, index stream:  counter (t / 2, k, 0, .) -> draws t, t+1 of realisation k
//   tag 2, value stream:  counter (e / 4, k, j, .) -> elements e..e+3 of column j
//   tag 3, experiment stream: counter (e, k, j, .) -> element e of column j
//          (the laws of the experiments of Sec. 4, one call per element)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlmc {

constexpr uint32_t kTagIndex = 1u;
constexpr uint32_t kTagValue = 2u;
constexpr uint32_t kTagExperiment = 3u;

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__host__ __device__ inline uint32_t stream_id(uint32_t tag, uint32_t level_field, uint32_t problem)
{
    return (tag << 28) | ((level_field & 0xFFu) << 20) | (problem & 0xFFFFFu);
}

// a ^ b ^ k in one VALU instruction: gfx950's three-input bit operation
// (v_bitop3_b32) with the XOR truth table 0x96.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k)
{
    return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// One Philox4x32-10 evaluation.  The key schedule depends only on the seed,
// which is uniform across a launch, so it stays in scalar registers; each
// round costs two 32x32->64-bit multiply-adds and two three-input xors.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t prod_a = (uint64_t)0xD2511F53u * c0;
        const uint64_t prod_b = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_key((uint32_t)(prod_b >> 32), c1, k0);
        const uint32_t n2 = xor3_key((uint32_t)(prod_a >> 32), c3, k1);
        c1 = (uint32_t)prod_b;
        c3 = (uint32_t)prod_a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{c0, c1, c2, c3};
}

// Uniform index in [0, n) from a 64-bit word x = hi:lo, r = floor(x n / 2^64),
// evaluated exactly in 64-bit arithmetic for n < 2^32.
__device__ __forceinline__ uint32_t index_from_words(uint32_t lo, uint32_t hi, uint32_t n)
{
    const uint64_t low_part = ((uint64_t)lo * n) >> 32;
    return (uint32_t)(((uint64_t)hi * n + low_part) >> 32);
}

// Both draws 2q and 2q+1 of realisation k.
__device__ __forceinline__ void draw_index_pair(uint32_t q, uint32_t k, uint32_t sid_index,
                                                uint32_t key0, uint32_t key1, uint32_t n,
                                                uint32_t& r_even, uint32_t& r_odd)
{
    const Words4 w = philox4x32_10(q, k, 0u, sid_index, key0, key1);
    r_even = index_from_words(w.w0, w.w1, n);
    r_odd = index_from_words(w.w2, w.w3, n);
}

__device__ __forceinline__ uint32_t draw_index(uint32_t t, uint32_t k, uint32_t sid_index,
                                               uint32_t key0, uint32_t key1, uint32_t n)
{
    const Words4 w = philox4x32_10(t >> 1, k, 0u, sid_index, key0, key1);
    return (t & 1u) ? index_from_words(w.w2, w.w3, n) : index_from_words(w.w0, w.w1, n);
}

// Non-uniform index probabilities xi_j = w_j / W (eq. (18) with a general
// xi): cum[j] = w_0 + ... + w_j (exact integers), W = cum[n-1].  The same
// 64-bit word x = hi:lo as the uniform draw gives T = floor(x W / 2^64), and
// the index is the smallest j with cum[j] > T.  With every w_j = 1 this is
// floor(x n / 2^64): the uniform draw.
__device__ __forceinline__ uint32_t index_from_cumulative(uint32_t lo, uint32_t hi, const uint64_t* cum,
                                                          uint32_t n, uint64_t total)
{
    const uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    const uint64_t T = __umul64hi(x, total);
    uint32_t a = 0, b = n - 1u;
    while (a < b) {
        const uint32_t mid = a + (b - a) / 2u;
        if (cum[mid] > T) b = mid;
        else a = mid + 1u;
    }
    return a;
}

__device__ __forceinline__ uint32_t draw_index_weighted(uint32_t t, uint32_t k, uint32_t sid_index, uint32_t key0,
                                                        uint32_t key1, const uint64_t* cum, uint32_t n,
                                                        uint64_t total)
{
    const Words4 w = philox4x32_10(t >> 1, k, 0u, sid_index, key0, key1);
    return (t & 1u) ? index_from_cumulative(w.w2, w.w3, cum, n, total)
                    : index_from_cumulative(w.w0, w.w1, cum, n, total);
}

// u = ((w >> 9) + 1/2) 2^-23: 2^23 equally spaced points in (0, 1), exactly
// representable in FP32 and FP64, never 0 or 1.  (w >> 9) 2^-23 + 2^-24 is
// exact in FP32, so the single fma gives the same value.
__device__ __forceinline__ float unit_f32(uint32_t w)
{
    return __builtin_fmaf((float)(w >> 9), 0x1p-23f, 0x1p-24f);
}

__device__ __forceinline__ double unit_f64(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

// Box-Muller pair from two uniforms: (rho cos 2 pi v, rho sin 2 pi v),
// rho = sqrt(-2 ln u).  FP32 uses the hardware transcendental units:
// v_log_f32 gives log2, v_sqrt_f32 (1 ulp, no IEEE fix-up sequence: its
// argument is at least 2^-23 ln 2 > 0), v_sin/v_cos take their argument in
// revolutions.
__device__ __forceinline__ void box_muller(float u, float v, float& z0, float& z1)
{
    const float rho = __builtin_amdgcn_sqrtf(-2.0f * 0.69314718055994530942f * __builtin_amdgcn_logf(u));
    z0 = rho * __builtin_amdgcn_cosf(v);
    z1 = rho * __builtin_amdgcn_sinf(v);
}

// FP64 pair for the uniforms of this library only (u, v on the grids
// (h + 1/2) 2^-23 or 2^-16: in (0, 1), at most 24 significant bits), from
// series with their range reductions done exactly:
//   ln u: u = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
//     s = (m - 1) / (m + 1), |s| <= 0.1716, summed as
//     2 s (1 + s^2/3 + s^4/5 + ... + s^20/21) (the next term is below 1e-18
//     relative);
//   cos 2 pi v, sin 2 pi v: v = k/4 + r with k = rint(4 v) and |r| <= 1/8
//     (both exact), the Taylor series of cos and sin at x = 2 pi r
//     (|x| <= pi/4; terms to x^18 and x^17, the rest below 1e-19), then k
//     quarter turns.
// About two units in the last place; no argument reduction for large
// arguments, no special cases.
__device__ __forceinline__ double ln_unit(double u)
{
    int e;
    double m = frexp(u, &e);                       // u = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    p = fma(p, s2, 1.0);
    return fma((double)e, 0.69314718055994530942, 2.0 * s * p);
}

__device__ __forceinline__ void sincos_turns(double v, double& sn, double& cs)
{
    const double k = rint(4.0 * v);
    const double r = fma(k, -0.25, v);
    const double x = r * 6.283185307179586476925286766559;
    const double x2 = x * x;
    // sin x = x (1 - x^2/3! + x^4/5! - ... - x^16/17!)
    double ps = -1.0 / 355687428096000.0;
    ps = fma(ps, x2, 1.0 / 1307674368000.0);
    ps = fma(ps, x2, -1.0 / 6227020800.0);
    ps = fma(ps, x2, 1.0 / 39916800.0);
    ps = fma(ps, x2, -1.0 / 362880.0);
    ps = fma(ps, x2, 1.0 / 5040.0);
    ps = fma(ps, x2, -1.0 / 120.0);
    ps = fma(ps, x2, 1.0 / 6.0);
    const double sx = fma(-x * x2, ps, x);
    // cos x = 1 - x^2/2! + x^4/4! - ... - x^18/18!
    double pc = -1.0 / 6402373705728000.0;
    pc = fma(pc, x2, 1.0 / 20922789888000.0);
    pc = fma(pc, x2, -1.0 / 87178291200.0);
    pc = fma(pc, x2, 1.0 / 479001600.0);
    pc = fma(pc, x2, -1.0 / 3628800.0);
    pc = fma(pc, x2, 1.0 / 40320.0);
    pc = fma(pc, x2, -1.0 / 720.0);
    pc = fma(pc, x2, 1.0 / 24.0);
    pc = fma(pc, x2, -0.5);
    const double cx = fma(x2, pc, 1.0);
    const int q = (int)k & 3;
    sn = q == 0 ? sx : (q == 1 ? cx : (q == 2 ? -sx : -cx));
    cs = q == 0 ? cx : (q == 1 ? -sx : (q == 2 ? -cx : sx));
}

__device__ __forceinline__ void box_muller(double u, double v, double& z0, double& z1)
{
    const double rho = sqrt(-2.0 * ln_unit(u));
    double s, c;
    sincos_turns(v, s, c);
    z0 = rho * c;
    z1 = rho * s;
}

// 16-bit uniforms (the optional cheaper value generation): u = (h + 1/2)
// 2^-16 for a 16-bit h, exact in FP32 and FP64, never 0 or 1.
template <typename T>
__device__ __forceinline__ T unit16(uint32_t h);
template <>
__device__ __forceinline__ float unit16<float>(uint32_t h) { return __builtin_fmaf((float)h, 0x1p-16f, 0x1p-17f); }
template <>
__device__ __forceinline__ double unit16<double>(uint32_t h) { return ((double)h + 0.5) * 0x1p-16; }

template <typename T>
__device__ __forceinline__ T unit(uint32_t w);
template <>
__device__ __forceinline__ float unit<float>(uint32_t w) { return unit_f32(w); }
template <>
__device__ __forceinline__ double unit<double>(uint32_t w) { return unit_f64(w); }

}  // namespace mlmc
