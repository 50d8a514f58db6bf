// Shared definitions of the MLMC library (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.hpp"

namespace mlmc {

constexpr int kWave = 64;

// Entry law as the kernels see it (mirrors mlmc_dist of the C ABI).
struct Law {
    int32_t kind;      // 0 normal, 1 uniform, 2 reparam, 3 .. 6 the laws of Sec. 4
    double loc;
    double scale;
    const float* mean;
    const float* stdev;
    int64_t ld;
    double aux;        // exp(-loc) for the Poisson laws (4, 6), computed on the host
};

// Laws of the experiments of Sec. 4 (kinds 3 .. 6).  Column j is counted
// from 1 as in the paper; K ~ Poisson(loc), E ~ Exp(1), z, z' ~ N(0, 1),
// u ~ U(0, 1):
//   3  (j scale)(loc - z)                       Sec. 4.1, x_j
//   4  cos(K + 2E) [u < scale]                  Sec. 4.1, y_j
//   5  sin(x) + z' x,  x = (j scale)(loc - z)   Sec. 4.2, A_ij
//   6  cos(K) H(5 - K) [u < scale]              Sec. 4.2, B_jk
// Element e of the column vector v_j = [A[:, j]; B[j, :]] of realisation k
// takes a Philox call of its own, counter (e, k, j, experiment stream), and
// its uniforms u0, u1, u2: Box-Muller on (u0, u1) gives z (cosine half) and
// z' (sine half); K is the smallest integer with F(K) >= u0, the Poisson CDF
// accumulated term by term from exp(-loc); E = -ln u1; the Bernoulli factor
// is u2 < scale (kind 4) or u1 < scale (kind 6).  Evaluated in FP64 in every
// precision, so the integer decisions (K, the mask) never depend on it.
constexpr int kLawExperimentFirst = 3;

__device__ inline double experiment_value(int kind, double loc, double scale, double exp_neg_loc, uint32_t e,
                                          uint32_t k, uint32_t j, uint32_t sid_experiment, uint32_t key0,
                                          uint32_t key1)
{
    const Words4 w = philox4x32_10(e, k, j, sid_experiment, key0, key1);
    const double u0 = unit_f64(w.w0), u1 = unit_f64(w.w1);
    if (kind == 3 || kind == 5) {
        const double rho = sqrt(-2.0 * log(u0));
        double s, c;
        sincos(6.283185307179586476925286766559 * u1, &s, &c);
        const double x = (((double)j + 1.0) * scale) * (loc - rho * c);
        return kind == 3 ? x : sin(x) + (rho * s) * x;
    }
    int K = 0;
    double pk = exp_neg_loc, F = pk;
    while (u0 > F && K < 1000) {
        K += 1;
        pk = (pk * loc) / (double)K;
        F = F + pk;
    }
    if (kind == 4) return unit_f64(w.w2) < scale ? cos((double)K - 2.0 * log(u1)) : 0.0;
    // the stepped law takes cos(K) for K = 0 .. 5 only: a table of the
    // correctly rounded values instead of an FP64 cosine per element
    if (!(u1 < scale && K <= 5)) return 0.0;
    switch (K) {
    case 0: return 1.0;
    case 1: return 0x1.14a280fb5068cp-1;
    case 2: return -0x1.aa22657537205p-2;
    case 3: return -0x1.fae04be85e5d2p-1;
    case 4: return -0x1.4eaa606db24c1p-1;
    default: return 0x1.22785706b4ad9p-2;
    }
}

// Welford / Chan statistics of a set of scalars: count, mean, sum of squared
// deviations.  Merging two sets is exact in exact arithmetic (Chan, Golub,
// LeVeque 1979) and is evaluated in a fixed order everywhere, so results are
// bitwise reproducible.
// Remark 3.6, eq. (28): N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_j sqrt(V_j C_j))
// with C_l = c_l, over levels 0 .. nlev - 1, each at least `pilot`.  One
// definition for the host and the device (the same operations in the same
// order, no contraction), so both schedule the same N_l.  Returns 0, 1 when
// some N_l reaches 2^32 (bad_level: which), or 2 when the draws
// sum_l N_l c_l exceed max_total_draws (> 0).
__host__ __device__ inline int schedule_counts(double eps, const int64_t* c, const double* var, int nlev,
                                               int64_t pilot, int64_t max_total_draws, int64_t* n_out,
                                               int* bad_level, double* bad_value)
{
#pragma clang fp contract(off)
    double total = 0.0;
    for (int l = 0; l < nlev; ++l) total += sqrt(var[l] * (double)c[l]);
    for (int l = 0; l < nlev; ++l) {
        const double nl = ceil(2.0 / (eps * eps) * sqrt(var[l] / (double)c[l]) * total);
        if (!(nl < 4294967296.0)) {
            *bad_level = l;
            *bad_value = nl;
            return 1;
        }
        int64_t v = (int64_t)nl;
        if (v < pilot) v = pilot;
        n_out[l] = v;
    }
    if (max_total_draws > 0) {
        double draws = 0.0;
        for (int l = 0; l < nlev; ++l) draws += (double)n_out[l] * (double)c[l];
        if (draws > (double)max_total_draws) {
            *bad_value = draws;
            return 2;
        }
    }
    return 0;
}

struct Moments {
    double n;
    double mean;
    double m2;
};

__host__ __device__ inline Moments chan_merge(Moments a, Moments b)
{
    if (b.n == 0.0) return a;
    if (a.n == 0.0) return b;
    const double n = a.n + b.n;
    const double delta = b.mean - a.mean;
    Moments r;
    r.n = n;
    r.mean = a.mean + delta * (b.n / n);
    r.m2 = a.m2 + b.m2 + delta * delta * (a.n * b.n / n);
    return r;
}

// Element e (0-based) of the column vector v_j = [A[:, j]; B[j, :]] from the
// Philox words of its quad.  Normal elements use the Box-Muller pair
// (e & ~1, e | 1) of the same quad.
// Uniform entries are loc + scale (2u - 1), evaluated as one fused
// multiply-add u (2 scale) + (loc - scale) whose constants are launch-uniform.
template <typename T>
__device__ __forceinline__ T law_value(const Law& law, T z_normal, T u_uniform, int64_t mat_index)
{
    if (law.kind == 1) return fma(u_uniform, (T)(2.0 * law.scale), (T)(law.loc - law.scale));
    if (law.kind == 2) return fma((T)law.stdev[mat_index], z_normal, (T)law.mean[mat_index]);
    return fma(z_normal, (T)law.scale, (T)law.loc);
}

// Target function f of Sec. 3, applied entrywise to every sketch (kinds as
// mlmc_func): 0 f(x) = x; 1 f(x) = |x| H(theta0 - x); 2 f(x) =
// 1 / (|x| H(x + theta0) + theta1); H(0) = 1.  x <= theta0 and x >= -theta0
// are the exact floating-point forms of the two step conditions.
struct TargetFunc {
    int32_t kind;
    double theta0, theta1;
};

template <typename T>
__device__ __forceinline__ T target_value(int kind, T x, T theta0, T theta1)
{
    if (kind == 1) return x <= theta0 ? fabs(x) : (T)0;
    if (kind == 2) return (T)1 / ((x >= -theta0 ? fabs(x) : (T)0) + theta1);
    return x;
}

// Law pairs with a specialised kernel instantiation (no per-value law branches
// in hot loops); every other combination takes the general path.
// kLawsExperiment: both laws are laws of Sec. 4 (they pair only with each
// other; the entry points reject a mixed pair).
enum { kLawsAny = 0, kLawsUniform = 1, kLawsNormal = 2, kLawsExperiment = 3 };

__host__ __device__ inline int law_pair_kind(int a, int b)
{
    if (a >= kLawExperimentFirst && b >= kLawExperimentFirst) return kLawsExperiment;
    return (a == 1 && b == 1) ? kLawsUniform : (a == 0 && b == 0) ? kLawsNormal : kLawsAny;
}

// A law with its affine constants precomputed in the arithmetic type T, held
// in registers: value = fma(u, mul, add) (uniform), fma(z, mul, add) (normal),
// fma(stdev[i], z, mean[i]) (reparameterised).
template <typename T>
struct LawEval {
    int kind;
    T mul, add;
    const float* mean;
    const float* stdev;
    int64_t ld;

    __device__ __forceinline__ static LawEval make(const Law& law)
    {
        LawEval e;
        e.kind = law.kind;
        e.mul = (T)(law.kind == 1 ? 2.0 * law.scale : law.scale);
        e.add = (T)(law.kind == 1 ? law.loc - law.scale : law.loc);
        e.mean = law.mean;
        e.stdev = law.stdev;
        e.ld = law.ld;
        return e;
    }
    __device__ __forceinline__ T operator()(T z, T u, int64_t idx) const
    {
        if (kind == 1) return fma(u, mul, add);
        if (kind == 2) return fma((T)stdev[idx], z, (T)mean[idx]);
        return fma(z, mul, add);
    }
    // the same with the kind fixed at compile time by the law pair
    template <int LAWS>
    __device__ __forceinline__ T eval(T z, T u, int64_t idx) const
    {
        if (LAWS == kLawsUniform) return fma(u, mul, add);
        if (LAWS == kLawsNormal) return fma(z, mul, add);
        return (*this)(z, u, idx);
    }
};

template <typename T>
__device__ __forceinline__ void quad_values(const Words4& w, bool need_normal, T& u0, T& u1,
                                            T& u2, T& u3, T& z0, T& z1, T& z2, T& z3)
{
    u0 = unit<T>(w.w0);
    u1 = unit<T>(w.w1);
    u2 = unit<T>(w.w2);
    u3 = unit<T>(w.w3);
    if (need_normal) {
        box_muller(u0, u1, z0, z1);
        box_muller(u2, u3, z2, z3);
    } else {
        z0 = z1 = z2 = z3 = (T)0;
    }
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace mlmc
