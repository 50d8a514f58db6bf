/*
 * Reference oracle for the multilevel Monte Carlo (MLMC) estimator of E[AB]
 * of Wu & Polydorides, "A Multilevel Monte Carlo Estimator for Matrix
 * Multiplication" (arXiv:1904.00429).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, sequential FP64
 * implementation used to check the GPU library.  It shares no code with the
 * HIP path and the product never links it: only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.
 *
 * What it computes, step by step (uniform probabilities; f = identity unless
 * a target function is given):
 *   - Sec. 2, eq. (4): index probabilities xi_j = 1/n, draws with replacement.
 *   - Sec. 3, eq. (18): the sketch Z = (n/c) sum_t A[:, r_t] B[r_t, :].
 *   - Sec. 3.1, Alg. 1 (level_estimation): for every realisation k a pair
 *     A^(k), B^(k) and c_l indices; the fine sketch uses all c_l indices, the
 *     coarse sketch uses c_{l-1} of the same indices, and the level sample is
 *     their difference (at level 0 the fine sketch alone).
 *   - Sec. 3 and Alg. 1 with a target function f: both sketches are mapped
 *     entrywise by f before the difference, D = f(Zf) - f(Zc) (f(Zf) at
 *     level 0).  The functions are those of the experiments of Sec. 4 (see
 *     orc_func below).
 *   - Sec. 2, eq. (9): the level estimator is the mean of the level samples;
 *     the per-level variance V_l (Remark 3.6) is the vectorised variance of a
 *     single level sample, i.e. the sum over entries of the entry variances.
 *
 * Readings where the paper is silent (random number generation):
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 *     easy as 1, 2, 3", SC'11) keyed by the 64-bit seed.
 *   - Index draw t of sample k: counter (t/2, k, 0, 1<<28 | level<<20 | problem);
 *     the two words 2(t%2), 2(t%2)+1 form x = hi<<32 | lo and
 *     r_t = floor(x * n / 2^64).
 *   - Values of column j of sample k: v = [A^(k)[:, j]; B^(k)[j, :]] of length
 *     m+p; element e uses word e%4 of Philox(e/4, k, j, 2<<28 | level<<20 | problem).
 *     The uniform is u = ((w >> 9) + 1/2) 2^-23 (exact in FP32 and FP64);
 *     pairs (e, e+1), e even, give Box-Muller normals
 *     z_e = sqrt(-2 ln u_e) cos(2 pi u_{e+1}), z_{e+1} = ... sin(...).
 *     Values are keyed by the column, so a repeated index reuses the same
 *     column of the same realisation A^(k), B^(k) (Alg. 1 draws the pair first).
 *   - Optional 16-bit uniforms for the laws normal, uniform and reparam
 *     (orc_law.value16): element e uses half (e & 1) of word (e/2) % 4 of the
 *     call (e/8, k, j, 2<<28 | level<<20 | problem), eight per call.
 *   - Optional non-uniform probabilities xi_j = w_j / W from integer weights
 *     (eq. (18) with a general xi; Theorem 3.1's xi** quantised, see
 *     orc_optimal_weights): the same 64-bit word x gives T = floor(x W / 2^64)
 *     and r is the column whose cumulative-weight interval holds T.
 *   - The laws of the experiments of Sec. 4 (orc_law below): element e of
 *     column j draws its own Philox call, counter (e, k, j, 3<<28 | level<<20
 *     | problem), and uses its four uniforms for the normal (Box-Muller from
 *     u0, u1, both of its normals where the law needs two), the Poisson
 *     variable (inverse CDF from u0), the exponential (-ln u1) and the
 *     Bernoulli decision (u < scale, u2 or u1).
 *   - The coarse sketch uses the first c_{l-1} of the c_l fine indices.
 *     Draws are i.i.d., so any fixed subset of c_{l-1} indices has the law the
 *     paper requires; the prefix nests the levels exactly.  The stride
 *     coupling of Sec. 3.1 (every M-th fine index, r_{jM}, j = 1 .. c_{l-1},
 *     M = c_l / c_{l-1}) is the other subset offered: `stride` = M, or 0 for
 *     the prefix.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

#define ORC_TAG_INDEX 1u
#define ORC_TAG_VALUE 2u
#define ORC_TAG_EXPERIMENT 3u

enum { ORC_LAW_NORMAL = 0, ORC_LAW_UNIFORM = 1, ORC_LAW_REPARAM = 2, ORC_LAW_RAMP_NORMAL = 3,
       ORC_LAW_COS_POISSON_EXP = 4, ORC_LAW_SIN_RAMP = 5, ORC_LAW_COS_POISSON_STEP = 6 };

/* Distribution of the entries of A (m x n) or B (n x p).
 *   NORMAL:  loc + scale * z, z ~ N(0, 1)
 *   UNIFORM: loc + scale * (2u - 1), u ~ U(0, 1)
 *   REPARAM: mean[.] + stdev[.] * z; A is column-major (element (i, j) at
 *            j*ld + i), B is row-major (element (j, q) at j*ld + q).
 * The laws of the experiments of Sec. 4 (column j counted from 1 as in the
 * paper, K ~ Poisson(loc), E ~ Exp(1), z, z' ~ N(0, 1), u ~ U(0, 1)):
 *   RAMP_NORMAL:       (j scale) (loc - z)                    (Sec. 4.1, a_j: scale 1/50, loc 0.4)
 *   COS_POISSON_EXP:   cos(K + 2 E) [u < scale]               (Sec. 4.1, b_j: loc 10, scale 0.05)
 *   SIN_RAMP:          sin(x) + z' x, x = (j scale)(loc - z)  (Sec. 4.2, A_ij: scale 1e-4, loc 0.5)
 *   COS_POISSON_STEP:  cos(K) H(5 - K) [u < scale]            (Sec. 4.2, B_jk: loc 2, scale 0.2)
 * exp_neg_loc = exp(-loc) for the Poisson laws (the first term of the
 * inverse-CDF walk). */
typedef struct {
    int32_t law;
    double loc;
    double scale;
    const double* mean;
    const double* stdev;
    int64_t ld;
    double exp_neg_loc;
    int32_t value16;   /* laws 0-2: 16-bit uniforms, two per 32-bit word (see value_uniform16) */
    int32_t operand;   /* ORC_OPERAND_*: the format the contraction reads the value in (see operand_value) */
    const int32_t* scale_exp;  /* FP8: exponent s of the power-of-two scale 2^s of each row of A (length m)
                                  or column of B (length p); NULL: s = 0 */
} orc_law;

/* Operand formats of the precision form (Sec. 3's sketch with its gathered
 * operands held in a narrower format; the contraction itself stays exact
 * here, in FP64). */
enum { ORC_OPERAND_EXACT = 0, ORC_OPERAND_BF16 = 1, ORC_OPERAND_FP8_E4M3 = 2 };

/* Target function f of Sec. 3, applied entrywise to a sketch.
 *   ORC_F_IDENTITY:     f(x) = x
 *   ORC_F_ABS_STEP:     f(x) = |x| H(theta0 - x)              (Sec. 4.2: theta0 = 2)
 *   ORC_F_INV_ABS_STEP: f(x) = 1 / (|x| H(x + theta0) + theta1)  (Sec. 4.1: 0.4, 0.01)
 * H is the Heaviside step; the paper does not fix H(0), read here as H(0) = 1. */
enum { ORC_F_IDENTITY = 0, ORC_F_ABS_STEP = 1, ORC_F_INV_ABS_STEP = 2 };

typedef struct {
    int32_t kind;
    double theta0;
    double theta1;
} orc_func;

static double heaviside(double x)
{
    return x >= 0.0 ? 1.0 : 0.0;
}

/* f(x); a NULL f is the identity. */
double orc_apply_func(const orc_func* f, double x)
{
    if (!f || f->kind == ORC_F_IDENTITY)
        return x;
    if (f->kind == ORC_F_ABS_STEP)
        return fabs(x) * heaviside(f->theta0 - x);
    return 1.0 / (fabs(x) * heaviside(x + f->theta0) + f->theta1);
}

/* Philox4x32-10: ten rounds of the Philox S-box, the key bumped by the
 * Weyl constants between rounds (SC'11, Sec. 5). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += ORC_PHILOX_W0;
        k1 += ORC_PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox_batch(int64_t count, const uint32_t* ctr, uint64_t seed, uint32_t* out)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int64_t i = 0; i < count; ++i)
        orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

static uint32_t stream_word(uint32_t tag, uint32_t level_field, uint32_t problem)
{
    return (tag << 28) | ((level_field & 0xFFu) << 20) | (problem & 0xFFFFFu);
}

/* Index draw t of realisation k: uniform on {0, ..., n-1}, with replacement
 * (Sec. 2, eq. (4)).  r = floor(x n / 2^64) from a 64-bit word x. */
int64_t orc_draw_index(uint64_t seed, uint32_t problem, uint32_t level_field,
                       uint32_t k, int64_t t, int64_t n)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)(t >> 1), k, 0u,
                        stream_word(ORC_TAG_INDEX, level_field, problem) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    int h = (int)(t & 1);
    uint64_t x = ((uint64_t)w[2 * h + 1] << 32) | (uint64_t)w[2 * h];
    unsigned __int128 prod = (unsigned __int128)x * (unsigned __int128)(uint64_t)n;
    return (int64_t)(uint64_t)(prod >> 64);
}

/* The same draw from a 32-bit word: draw t uses word t % 4 of the call
 * (t / 4, k, 0, index stream) and r = floor(w n / 2^32), four draws per
 * Philox call.  Exactly uniform when n is a power of two (r is then the top
 * log2 n bits of w); the library offers it for such n only. */
int64_t orc_draw_index32(uint64_t seed, uint32_t problem, uint32_t level_field,
                         uint32_t k, int64_t t, int64_t n)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)(t >> 2), k, 0u,
                        stream_word(ORC_TAG_INDEX, level_field, problem) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    uint64_t prod = (uint64_t)w[t & 3] * (uint64_t)n;
    return (int64_t)(prod >> 32);
}

/* Draws 0 .. c-1 of realisation k (word32: the 32-bit draw). */
void orc_draw_indices_mode(uint64_t seed, uint32_t problem, uint32_t level_field,
                           uint32_t k, int64_t c, int64_t n, int32_t word32, int64_t* r)
{
    for (int64_t t = 0; t < c; ++t)
        r[t] = word32 ? orc_draw_index32(seed, problem, level_field, k, t, n)
                      : orc_draw_index(seed, problem, level_field, k, t, n);
}

void orc_draw_indices(uint64_t seed, uint32_t problem, uint32_t level_field,
                      uint32_t k, int64_t c, int64_t n, int64_t* r)
{
    orc_draw_indices_mode(seed, problem, level_field, k, c, n, 0, r);
}

/* Non-uniform index probabilities (eq. (18) with a general xi): xi_j = w_j / W
 * for integer weights w_j >= 1, W = sum_j w_j, cum[j] = w_0 + ... + w_j.
 * Draw t uses the same 64-bit word x as the uniform draw:
 * T = floor(x W / 2^64) is uniform on {0, ..., W-1} (to within 2^-64 per
 * value) and r is the column whose interval [cum[r] - w_r, cum[r]) holds T.
 * With every w_j = 1, W = n and r = T: exactly the uniform draw. */
typedef struct {
    const uint32_t* w;
    const uint64_t* cum;
    uint64_t total;
} orc_weights;

void orc_weights_cumulative(const uint32_t* w, int64_t n, uint64_t* cum)
{
    uint64_t s = 0;
    for (int64_t j = 0; j < n; ++j) {
        s += w[j];
        cum[j] = s;
    }
}

int64_t orc_draw_index_weighted(uint64_t seed, uint32_t problem, uint32_t level_field,
                                uint32_t k, int64_t t, int64_t n, const orc_weights* iw)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)(t >> 1), k, 0u,
                        stream_word(ORC_TAG_INDEX, level_field, problem) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    int h = (int)(t & 1);
    uint64_t x = ((uint64_t)w[2 * h + 1] << 32) | (uint64_t)w[2 * h];
    uint64_t T = (uint64_t)(((unsigned __int128)x * (unsigned __int128)iw->total) >> 64);
    /* smallest j with cum[j] > T */
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (iw->cum[mid] > T) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

/* Theorem 3.1's xi**_j, proportional to sqrt(E||A_{:,j}||^2 E||B_{j,:}||^2),
 * quantised to integer weights: s_j = sqrt(EA_j) sqrt(EB_j) with
 * EA_j = sum_i (mean_ij^2 + stdev_ij^2) accumulated in FP64 for i = 0, 1, ...
 * (the mean's square first), likewise EB_j over the row of B;
 * w_j = max(1, floor(2^24 s_j / max_i s_i)).  For i.i.d. laws every column
 * has the same moments: w_j = 2^24 (xi** is uniform). */
void orc_optimal_weights(int64_t m, int64_t n, int64_t p, const orc_law* A, const orc_law* B, uint32_t* w)
{
    if (A->law != ORC_LAW_REPARAM || B->law != ORC_LAW_REPARAM) {
        for (int64_t j = 0; j < n; ++j)
            w[j] = 1u << 24;
        return;
    }
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    double smax = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double ea = 0.0, eb = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            double mu = A->mean[j * A->ld + i], sd = A->stdev[j * A->ld + i];
            ea = ea + mu * mu;
            ea = ea + sd * sd;
        }
        for (int64_t q = 0; q < p; ++q) {
            double mu = B->mean[j * B->ld + q], sd = B->stdev[j * B->ld + q];
            eb = eb + mu * mu;
            eb = eb + sd * sd;
        }
        s[j] = sqrt(ea) * sqrt(eb);
        if (s[j] > smax)
            smax = s[j];
    }
    for (int64_t j = 0; j < n; ++j) {
        double v = smax > 0.0 ? floor(s[j] / smax * 16777216.0) : 1.0;
        w[j] = v < 1.0 ? 1u : (uint32_t)v;
    }
    free(s);
}

double orc_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

static uint32_t value_word(uint64_t seed, uint32_t problem, uint32_t level_field,
                           uint32_t k, int64_t j, int64_t e)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)(e >> 2), k, (uint32_t)j,
                        stream_word(ORC_TAG_VALUE, level_field, problem) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    return w[e & 3];
}

/* 16-bit uniforms: element e of column j uses the call (e/8, k, j, value
 * stream) and, of its word (e/2) % 4, the low half for even e and the high
 * half for odd e: u = (h + 1/2) 2^-16, eight uniforms per call. */
static double value_uniform16(uint64_t seed, uint32_t problem, uint32_t level_field,
                              uint32_t k, int64_t j, int64_t e)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)(e >> 3), k, (uint32_t)j,
                        stream_word(ORC_TAG_VALUE, level_field, problem) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    uint32_t word = w[(e >> 1) & 3];
    uint32_t h = (e & 1) ? (word >> 16) : (word & 0xFFFFu);
    return ((double)h + 0.5) * 0x1p-16;
}

/* Standard normal number e of the vector of column j (Box-Muller on the
 * uniforms of elements e & ~1 and e | 1). */
static double std_normal_mode(uint64_t seed, uint32_t problem, uint32_t level_field,
                              uint32_t k, int64_t j, int64_t e, int32_t value16)
{
    const double two_pi = 6.283185307179586476925286766559;
    int64_t e0 = e & ~(int64_t)1;
    double u1, u2;
    if (value16) {
        u1 = value_uniform16(seed, problem, level_field, k, j, e0);
        u2 = value_uniform16(seed, problem, level_field, k, j, e0 + 1);
    } else {
        u1 = orc_uniform(value_word(seed, problem, level_field, k, j, e0));
        u2 = orc_uniform(value_word(seed, problem, level_field, k, j, e0 + 1));
    }
    double radius = sqrt(-2.0 * log(u1));
    double angle = two_pi * u2;
    return (e & 1) ? radius * sin(angle) : radius * cos(angle);
}

/* Poisson(lambda) by walking the CDF from 0: the smallest K with
 * F(K) >= u, F accumulated term by term (p_K = p_{K-1} lambda / K). */
static int64_t poisson_inverse(double u, double lambda, double exp_neg_lambda)
{
    int64_t K = 0;
    double p = exp_neg_lambda, F = p;
    while (u > F && K < 1000) {
        K += 1;
        p = (p * lambda) / (double)K;
        F = F + p;
    }
    return K;
}

/* The experiment laws: element e of column j of realisation k draws its own
 * Philox call (counter (e, k, j, 3<<28 | level<<20 | problem)), four uniforms
 * u0..u3; normals by Box-Muller from (u0, u1). */
static double experiment_value(const orc_law* law, uint64_t seed, uint32_t problem, uint32_t level_field,
                               uint32_t k, int64_t j, int64_t e)
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)e, k, (uint32_t)j, stream_word(ORC_TAG_EXPERIMENT, level_field, problem) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u[4];
    for (int i = 0; i < 4; ++i)
        u[i] = orc_uniform(w[i]);
    double col = (double)(j + 1);
    if (law->law == ORC_LAW_RAMP_NORMAL || law->law == ORC_LAW_SIN_RAMP) {
        double radius = sqrt(-2.0 * log(u[0]));
        double z = radius * cos(two_pi * u[1]);
        double x = (col * law->scale) * (law->loc - z);
        if (law->law == ORC_LAW_RAMP_NORMAL)
            return x;
        double z2 = radius * sin(two_pi * u[1]);
        return sin(x) + z2 * x;
    }
    int64_t K = poisson_inverse(u[0], law->loc, law->exp_neg_loc);
    if (law->law == ORC_LAW_COS_POISSON_EXP) {
        double E = -log(u[1]);
        return u[2] < law->scale ? cos((double)K + 2.0 * E) : 0.0;
    }
    return (u[1] < law->scale && K <= 5) ? cos((double)K) : 0.0;
}

/* x rounded to `bits` significant bits, ties to even (rint in the default
 * rounding mode), with the spacing of the binade 2^min_exp kept below it
 * (gradual underflow). */
static double round_significand(double x, int bits, int min_exp)
{
    if (x == 0.0)
        return x;
    int E;
    frexp(x, &E);                 /* |x| in [2^(E-1), 2^E) */
    int e = E - 1;
    if (e < min_exp)
        e = min_exp;
    double quantum = ldexp(1.0, e - (bits - 1));
    return rint(x / quantum) * quantum;
}

/* The value v of a row of A or column of B (index idx) as the contraction
 * reads it.  Values are generated in FP32 by the precision form, so v is
 * first rounded to FP32; then
 *   BF16: 8 significant bits (FP32's exponent range);
 *   FP8 e4m3 (OCP: 4 exponent bits with bias 7, 3 mantissa bits, no
 *   infinities, largest finite value 448, spacing 2^-9 below 2^-6): v is
 *   multiplied by the power of two 2^s of its row or column, clamped to
 *   [-448, 448], rounded to 4 significant bits, and divided by 2^s again
 *   (the contraction undoes the scales exactly). */
double orc_operand_value(const orc_law* law, int64_t idx, double v)
{
    if (law->operand == ORC_OPERAND_BF16)
        return round_significand((double)(float)v, 8, -126);
    if (law->operand == ORC_OPERAND_FP8_E4M3) {
        int s = law->scale_exp ? law->scale_exp[idx] : 0;
        double x = (double)(float)ldexp(v, s);
        if (x > 448.0)
            x = 448.0;
        if (x < -448.0)
            x = -448.0;
        return ldexp(round_significand(x, 4, -6), -s);
    }
    return v;
}

/* Bound of the reparameterised entries of each row i < count of A
 * (element (i, j) at j*ld + i) or column of B (element (j, q) at j*ld + q):
 * out[i] = max over the n columns (rows) j of fma(6, |stdev|, |mean|), the
 * input of the FP8 scale rule. */
void orc_reparam_bounds(const double* mean, const double* stdev, int64_t n, int64_t ld, int64_t count,
                        double* out)
{
    for (int64_t i = 0; i < count; ++i) {
        double b = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double v = fma(6.0, fabs(stdev[j * ld + i]), fabs(mean[j * ld + i]));
            if (v > b)
                b = v;
        }
        out[i] = b;
    }
}

/* Entry (row, col) of one realisation, produced from the element number e of
 * the column vector v_j. */
static double law_value(const orc_law* law, uint64_t seed, uint32_t problem,
                        uint32_t level_field, uint32_t k, int64_t j, int64_t e,
                        int64_t mat_index)
{
    if (law->law >= ORC_LAW_RAMP_NORMAL)
        return experiment_value(law, seed, problem, level_field, k, j, e);
    if (law->law == ORC_LAW_UNIFORM) {
        double u = law->value16 ? value_uniform16(seed, problem, level_field, k, j, e)
                                : orc_uniform(value_word(seed, problem, level_field, k, j, e));
        return law->loc + law->scale * (2.0 * u - 1.0);
    }
    double z = std_normal_mode(seed, problem, level_field, k, j, e, law->value16);
    if (law->law == ORC_LAW_REPARAM)
        return law->mean[mat_index] + law->stdev[mat_index] * z;
    return law->loc + law->scale * z;
}

/* Column j of A^(k) (length m) and row j of B^(k) (length p). */
void orc_column(uint64_t seed, uint32_t problem, uint32_t level_field, uint32_t k,
                int64_t j, int64_t m, int64_t p, const orc_law* A, const orc_law* B,
                double* a, double* b)
{
    for (int64_t i = 0; i < m; ++i)
        a[i] = orc_operand_value(A, i, law_value(A, seed, problem, level_field, k, j, i, j * A->ld + i));
    for (int64_t q = 0; q < p; ++q)
        b[q] = orc_operand_value(B, q, law_value(B, seed, problem, level_field, k, j, m + q, j * B->ld + q));
}

/* Draw number of the j-th coarse draw (0-based j): j (prefix), or
 * stride (j + 1) - 1, the 0-based position of r_{(j+1) M} (stride coupling). */
static int64_t coarse_draw(int64_t j, int64_t stride)
{
    return stride > 0 ? stride * (j + 1) - 1 : j;
}

/* Sketches of eq. (18) with general probabilities: Zf = (1/c_f) sum_{t < c_f}
 * a_t b_t^T / xi_t (xi_t = w_{r_t} / W: factor[t] = W / w_{r_t}), likewise
 * Zc over the c_c coarse draws (coarse_draw). */
void orc_sketch_pair_weighted(int64_t m, int64_t p, int64_t c_f, int64_t c_c, int64_t stride,
                              const double* factor, const double* AS, const double* BS, double* Zf,
                              double* Zc)
{
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t q = 0; q < p; ++q) {
            double sf = 0.0;
            for (int64_t t = 0; t < c_f; ++t)
                sf += factor[t] * (AS[t * m + i] * BS[t * p + q]);
            Zf[i * p + q] = sf / (double)c_f;
            if (c_c > 0) {
                double sc = 0.0;
                for (int64_t j = 0; j < c_c; ++j) {
                    int64_t t = coarse_draw(j, stride);
                    sc += factor[t] * (AS[t * m + i] * BS[t * p + q]);
                }
                Zc[i * p + q] = sc / (double)c_c;
            }
        }
    }
}

/* Sketches of Sec. 3, eq. (18) with xi_j = 1/n from gathered columns:
 *   Zf = (n / c_f) sum_{t < c_f} a_t b_t^T,  Zc = (n / c_c) sum over the c_c
 * coarse draws t = coarse_draw(j, stride) of a_t b_t^T.
 * AS holds a_t at AS + t*m, BS holds b_t at BS + t*p.  Z is m x p row-major.
 * c_c == 0 leaves Zc untouched. */
void orc_sketch_pair(int64_t m, int64_t p, int64_t n, int64_t c_f, int64_t c_c, int64_t stride,
                     const double* AS, const double* BS, double* Zf, double* Zc)
{
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t q = 0; q < p; ++q) {
            double sf = 0.0;
            for (int64_t t = 0; t < c_f; ++t)
                sf += AS[t * m + i] * BS[t * p + q];
            Zf[i * p + q] = ((double)n / (double)c_f) * sf;
            if (c_c > 0) {
                double sc = 0.0;
                for (int64_t j = 0; j < c_c; ++j) {
                    int64_t t = coarse_draw(j, stride);
                    sc += AS[t * m + i] * BS[t * p + q];
                }
                Zc[i * p + q] = ((double)n / (double)c_c) * sc;
            }
        }
    }
}

static int cmp_int64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* The tuple (r_0, ..., r_{c_f - 1}) of one realisation as a set with
 * multiplicities (the simplification noted after Alg. 1 in Sec. 3.1): its
 * distinct values in increasing order into j_out, and for each the number of
 * all draws (mu_f) and of the c_c coarse draws (coarse_draw(i, stride),
 * i < c_c: mu_c) that took it.  Returns the number of distinct values, or -1
 * on bad arguments / allocation failure.  The outputs hold c_f entries. */
int64_t orc_multiset(int64_t c_f, const int64_t* r, int64_t c_c, int64_t stride, int64_t* j_out,
                     int64_t* mu_f, int64_t* mu_c)
{
    if (c_f < 1 || c_c < 0 || c_c > c_f || stride < 0 || (stride > 0 && stride * c_c > c_f)) return -1;
    int64_t* sorted = (int64_t*)malloc(sizeof(int64_t) * (size_t)c_f);
    if (!sorted) return -1;
    memcpy(sorted, r, sizeof(int64_t) * (size_t)c_f);
    qsort(sorted, (size_t)c_f, sizeof(int64_t), cmp_int64);
    int64_t u = 0;
    for (int64_t t = 0; t < c_f; ++t) {
        if (u == 0 || sorted[t] != j_out[u - 1]) {
            j_out[u] = sorted[t];
            mu_f[u] = 0;
            mu_c[u] = 0;
            ++u;
        }
        mu_f[u - 1] += 1;
    }
    for (int64_t i = 0; i < c_c; ++i) {
        const int64_t j = r[coarse_draw(i, stride)];
        int64_t lo = 0, hi = u - 1;          /* binary search: j is in j_out */
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (j_out[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        mu_c[lo] += 1;
    }
    free(sorted);
    return u;
}

/* The sketches of eq. (18) from the set form: with the u distinct columns
 * a_j (AS + i*m) and rows b_j (BS + i*p) read once each,
 *   Zf = (1 / c_f) sum_i mu_f(i) g_i a_i b_i^T,   Zc = (1 / c_c) sum_i mu_c(i) g_i a_i b_i^T,
 * g_i = n (uniform draws) or factor[i] = W / w_j (weighted draws).  Equal to
 * orc_sketch_pair / orc_sketch_pair_weighted up to the order of the sums.
 * c_c == 0 leaves Zc untouched. */
void orc_sketch_pair_set(int64_t m, int64_t p, int64_t n, int64_t c_f, int64_t c_c, int64_t u,
                         const int64_t* mu_f, const int64_t* mu_c, const double* factor, const double* AS,
                         const double* BS, double* Zf, double* Zc)
{
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t q = 0; q < p; ++q) {
            double sf = 0.0, sc = 0.0;
            for (int64_t v = 0; v < u; ++v) {
                const double g = factor ? factor[v] : (double)n;
                const double ab = g * (AS[v * m + i] * BS[v * p + q]);
                sf += (double)mu_f[v] * ab;
                if (c_c > 0) sc += (double)mu_c[v] * ab;
            }
            Zf[i * p + q] = sf / (double)c_f;
            if (c_c > 0) Zc[i * p + q] = sc / (double)c_c;
        }
    }
}

/* Alg. 1 (level_estimation) for realisations k_begin <= k < k_end of one
 * level.  Level sample D = f(Zf) - f(Zc) (l > 0) or f(Zf) (l = 0,
 * c_prev == 0), f entrywise (NULL: identity).  Per entry, Welford's running
 * mean/M2 are updated in place, so
 * a call can continue the samples of an earlier call (Alg. 2 reuses earlier
 * evaluations).  samples_out (nullable) receives every D, row-major.
 * as_set: each realisation's index tuple is taken as a set with
 * multiplicities (orc_multiset), its distinct columns read once
 * (orc_sketch_pair_set).  Returns 0, or -1 on bad arguments / allocation
 * failure. */
int orc_level_estimation(int64_t m, int64_t n, int64_t p, const orc_law* A, const orc_law* B,
                         int64_t c_l, int64_t c_prev, int64_t stride, int32_t word32, uint64_t seed,
                         uint32_t problem,
                         uint32_t level_field, int64_t k_begin, int64_t k_end, const orc_func* f,
                         const orc_weights* iw, int32_t as_set, int64_t* count, double* mean, double* m2,
                         double* samples_out)
{
    if (m < 1 || p < 1 || n < 1 || c_l < 1 || c_prev < 0 || c_prev > c_l || k_end < k_begin)
        return -1;
    if (stride < 0 || (stride > 0 && stride * c_prev > c_l))
        return -1;
    int64_t mp = m * p;
    int64_t* r = (int64_t*)malloc(sizeof(int64_t) * (size_t)c_l);
    double* AS = (double*)malloc(sizeof(double) * (size_t)(c_l * m));
    double* BS = (double*)malloc(sizeof(double) * (size_t)(c_l * p));
    double* Zf = (double*)malloc(sizeof(double) * (size_t)mp);
    double* Zc = (double*)malloc(sizeof(double) * (size_t)mp);
    double* factor = (double*)malloc(sizeof(double) * (size_t)c_l);
    int64_t* js = (int64_t*)malloc(sizeof(int64_t) * (size_t)c_l * 3);
    if (!r || !AS || !BS || !Zf || !Zc || !factor || !js) {
        free(r); free(AS); free(BS); free(Zf); free(Zc); free(factor); free(js);
        return -1;
    }
    int64_t* mu_f = js + c_l;
    int64_t* mu_c = js + 2 * c_l;
    for (int64_t k = k_begin; k < k_end; ++k) {
        /* Sample c_l indices (uniformly, or with probabilities w_j / W), then
         * read the sampled columns of the realisation A^(k), B^(k). */
        if (iw) {
            for (int64_t t = 0; t < c_l; ++t) {
                r[t] = orc_draw_index_weighted(seed, problem, level_field, (uint32_t)k, t, n, iw);
                factor[t] = (double)iw->total / (double)iw->w[r[t]];
            }
        } else {
            orc_draw_indices_mode(seed, problem, level_field, (uint32_t)k, c_l, n, word32, r);
        }
        if (as_set) {
            const int64_t u = orc_multiset(c_l, r, c_prev, stride, js, mu_f, mu_c);
            if (u < 0) {
                free(r); free(AS); free(BS); free(Zf); free(Zc); free(factor); free(js);
                return -1;
            }
            for (int64_t v = 0; v < u; ++v) {
                orc_column(seed, problem, level_field, (uint32_t)k, js[v], m, p, A, B, AS + v * m, BS + v * p);
                if (iw) factor[v] = (double)iw->total / (double)iw->w[js[v]];
            }
            orc_sketch_pair_set(m, p, n, c_l, c_prev, u, mu_f, mu_c, iw ? factor : NULL, AS, BS, Zf, Zc);
        } else {
            for (int64_t t = 0; t < c_l; ++t)
                orc_column(seed, problem, level_field, (uint32_t)k, r[t], m, p, A, B,
                           AS + t * m, BS + t * p);
            if (iw)
                orc_sketch_pair_weighted(m, p, c_l, c_prev, stride, factor, AS, BS, Zf, Zc);
            else
                orc_sketch_pair(m, p, n, c_l, c_prev, stride, AS, BS, Zf, Zc);
        }
        *count += 1;
        double cnt = (double)(*count);
        for (int64_t e = 0; e < mp; ++e) {
            double d = (c_prev > 0) ? orc_apply_func(f, Zf[e]) - orc_apply_func(f, Zc[e])
                                    : orc_apply_func(f, Zf[e]);
            if (samples_out)
                samples_out[(k - k_begin) * mp + e] = d;
            double delta = d - mean[e];
            mean[e] += delta / cnt;
            m2[e] += delta * (d - mean[e]);
        }
    }
    free(r); free(AS); free(BS); free(Zf); free(Zc); free(factor); free(js);
    return 0;
}

/* Alg. 1 restricted to the entries (rows[a], cols[b]), 0 <= a < nr,
 * 0 <= b < nc, of the level sample: the same definition as
 * orc_level_estimation (eq. (18) per entry, the same realisations, index
 * draws and values, the same summation order), evaluated only where it is
 * asked for, so that products far too large for the whole sketch can be
 * checked entry by entry.  mean and m2 are nr x nc, row-major. */
int orc_level_entries(int64_t m, int64_t n, int64_t p, const orc_law* A, const orc_law* B,
                      int64_t c_l, int64_t c_prev, int64_t stride, uint64_t seed, uint32_t problem,
                      uint32_t level_field, int64_t k_begin, int64_t k_end,
                      int64_t nr, const int64_t* rows, int64_t nc, const int64_t* cols,
                      int64_t* count, double* mean, double* m2)
{
    if (m < 1 || p < 1 || n < 1 || c_l < 1 || c_prev < 0 || c_prev > c_l || k_end < k_begin ||
        nr < 1 || nc < 1 || stride < 0 || (stride > 0 && stride * c_prev > c_l))
        return -1;
    for (int64_t a = 0; a < nr; ++a)
        if (rows[a] < 0 || rows[a] >= m) return -1;
    for (int64_t b = 0; b < nc; ++b)
        if (cols[b] < 0 || cols[b] >= p) return -1;
    int64_t* r = (int64_t*)malloc(sizeof(int64_t) * (size_t)c_l);
    double* AS = (double*)malloc(sizeof(double) * (size_t)(c_l * nr));
    double* BS = (double*)malloc(sizeof(double) * (size_t)(c_l * nc));
    if (!r || !AS || !BS) {
        free(r); free(AS); free(BS);
        return -1;
    }
    for (int64_t k = k_begin; k < k_end; ++k) {
        orc_draw_indices(seed, problem, level_field, (uint32_t)k, c_l, n, r);
        for (int64_t t = 0; t < c_l; ++t) {
            int64_t j = r[t];
            for (int64_t a = 0; a < nr; ++a)
                AS[t * nr + a] = orc_operand_value(A, rows[a], law_value(A, seed, problem, level_field, (uint32_t)k, j,
                                                                         rows[a], j * A->ld + rows[a]));
            for (int64_t b = 0; b < nc; ++b)
                BS[t * nc + b] = orc_operand_value(B, cols[b], law_value(B, seed, problem, level_field, (uint32_t)k, j,
                                                                         m + cols[b], j * B->ld + cols[b]));
        }
        *count += 1;
        double cnt = (double)(*count);
        for (int64_t a = 0; a < nr; ++a) {
            for (int64_t b = 0; b < nc; ++b) {
                double sf = 0.0;
                for (int64_t t = 0; t < c_l; ++t)
                    sf += AS[t * nr + a] * BS[t * nc + b];
                double d = ((double)n / (double)c_l) * sf;
                if (c_prev > 0) {
                    double sc = 0.0;
                    for (int64_t j = 0; j < c_prev; ++j) {
                        int64_t t = coarse_draw(j, stride);
                        sc += AS[t * nr + a] * BS[t * nc + b];
                    }
                    d = d - ((double)n / (double)c_prev) * sc;
                }
                int64_t e = a * nc + b;
                double delta = d - mean[e];
                mean[e] += delta / cnt;
                m2[e] += delta * (d - mean[e]);
            }
        }
    }
    free(r); free(AS); free(BS);
    return 0;
}
