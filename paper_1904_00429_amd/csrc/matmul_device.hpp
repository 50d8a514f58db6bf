// Device code of the matrix-product pipeline shared by its launchers: the
// contraction policies, the gather of sampled columns and the sketch with its
// per-entry statistics, as device functions over one work item each, and the
// kernels that walk a grid of them.
#pragma once

#include <hip/hip_bf16.h>
#include <math.h>
#include <stdlib.h>

#include <type_traits>

#include "internal.hpp"

namespace mlmc {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(1))) void* GlobalPtr;   // the operands of global_load_lds
typedef __attribute__((address_space(3))) void* LdsPtr;

constexpr int kMergeThreads = 256;
constexpr int kGatherThreads = 64;
constexpr int kGatherPositions = 8;           // positions of one packed group (KPACK = 8)
constexpr int kGatherMaxOctets = 8;           // position groups per gather block, at most
constexpr int64_t kGatherBudgetBytes = 768ll << 20;
constexpr int64_t kSketchMaxBlocks = 8192;
constexpr int kXcds = 8;                     // accelerator complex dies of an MI355X
constexpr int64_t kDualMaxDraws = 32;        // realisations this short use the two-accumulator statistics
static_assert(kGatherThreads == kWave, "a gather unit is one wave");
// single-launch form: per step one claim counter per XCD queue of the
// sketch, one per XCD queue of the gather and one arrival counter, each on a
// 64-byte line of its own
constexpr int64_t kPersistentMaxPasses = 1 << 16;
constexpr int kSyncStride = 16;                    // uint32 words between counters
constexpr int kPhaseWords = (2 * kXcds + 1) * kSyncStride;

// ---------------------------------------------------------------------------
// Contraction policies: operand type, MFMA shape, fragment layout.  A
// workgroup is 2 x 2 waves; a wave computes NB x NB MFMA blocks of BLK x BLK.
// ---------------------------------------------------------------------------
struct PolicyF64 {  // v_mfma_f64_16x16x4_f64
    using In = double;
    using Acc = double;
    using AccVec = f64x4;
    using FragT = double;
    static constexpr int KSTEP = 4, KPACK = 1, BLK = 16, REGS = 4;
    static constexpr bool SCALED = false;
    // f64 results: lane l, register r holds row l / 16 + 4 r, column l % 16
    static __device__ __forceinline__ int row_of(int lane, int r) { return lane / 16 + 4 * r; }
    static __device__ __forceinline__ int col_of(int lane) { return lane % 16; }
    static __device__ __forceinline__ f64x4 mma(double a, double b, f64x4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// 32 x 32 output blocks: lane l, register r holds row 8 (r/4) + 4 (l/32) + r%4, column l % 32
struct Block32 {
    static __device__ __forceinline__ int row_of(int lane, int r) { return 8 * (r / 4) + 4 * (lane / 32) + (r % 4); }
    static __device__ __forceinline__ int col_of(int lane) { return lane % 32; }
};

struct PolicyF32 : Block32 {  // v_mfma_f32_32x32x2_f32
    using In = float;
    using Acc = float;
    using AccVec = f32x16;
    using FragT = float;
    static constexpr int KSTEP = 2, KPACK = 1, BLK = 32, REGS = 16;
    static constexpr bool SCALED = false;
    static __device__ __forceinline__ f32x16 mma(float a, float b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
};

struct PolicyBF16 : Block32 {  // v_mfma_f32_32x32x16_bf16: a lane holds 8 consecutive draws of one row
    using In = __bf16;
    using Acc = float;
    using AccVec = f32x16;
    using FragT = bf16x8;
    static constexpr int KSTEP = 16, KPACK = 8, BLK = 32, REGS = 16;
    static constexpr bool SCALED = false;
    static __device__ __forceinline__ f32x16 mma(bf16x8 a, bf16x8 b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// v_mfma_scale_f32_32x32x64_f8f6f4 with both operands OCP e4m3 (format code
// 0): lane l holds 32 consecutive draws of row (A) or column (B) l % 32, the
// draws 32 (l / 32) .. 32 (l / 32) + 31 of the step, and an E8M0 scale (a
// biased exponent, 2^(e - 127)) for them in byte 0 of its scale operand.
// The scales are the inverses of the power-of-two factors the gather
// multiplied each row of A and column of B by, so the FP32 accumulator holds
// the unscaled sum.
struct PolicyFP8 : Block32 {
    using In = uint8_t;
    using Acc = float;
    using AccVec = f32x16;
    using FragT = i32x8;
    static constexpr int KSTEP = 64, KPACK = 8, BLK = 32, REGS = 16;
    static constexpr bool SCALED = true;
    static __device__ __forceinline__ f32x16 mma(const i32x8& a, const i32x8& b, f32x16 c, int sa, int sb)
    {
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
    }
};

// ---------------------------------------------------------------------------
// Gather: only the sampled columns of each realisation are generated.
// ---------------------------------------------------------------------------
struct GatherParams {
    const ProblemDesc* descs;
    uint32_t c, c_prev, level_field;
    int64_t kc, kpad;        // padded coarse length, padded total length
    int64_t batch;           // realisations in this pass
    int octets;              // groups of 8 positions per block (1 .. kGatherMaxOctets)
    double omega;            // 1 - c_l / c_{l-1}: weight of the coarse draws, folded into a_t
    const uint32_t* iw;      // index weights (NULL: uniform draws)
    const uint64_t* cum;     // their cumulative sums
    uint32_t stride;         // stride coupling M (0: prefix)
    uint32_t key0, key1;
    uint32_t k_first;        // realisation of batch slot 0
    int elem;
    char* gbuf;              // per product: batch x [kpad/KPACK][m][KPACK], then batch x [..][p][..]
    const double* setw;      // set form: weight of every position, [product][slot][kpad] (0: not generated); else NULL
};

// Draw number t of padded position `pos`, or -1 for padding.  Positions
// [0, kc) hold the c_prev coarse draws, positions [kc, kpad) the others, in
// increasing t: with the prefix coupling draws 0 .. c_prev - 1, then the
// rest; with the stride coupling (M = stride) draws M - 1, 2M - 1, ..., then
// the q-th draw outside that set, t = q + floor(q / (M - 1)).  Within a
// level the sum over positions is a sum over all c draws either way.
__device__ __forceinline__ int64_t draw_of_position(int64_t pos, int64_t kc, uint32_t c, uint32_t c_prev,
                                                   uint32_t stride)
{
    if (pos < kc) {
        if (pos >= (int64_t)c_prev) return -1;
        return stride ? (int64_t)stride * (pos + 1) - 1 : pos;
    }
    const int64_t q = pos - kc;
    if (q >= (int64_t)c - (int64_t)c_prev) return -1;
    return stride ? q + q / ((int64_t)stride - 1) : (int64_t)c_prev + q;
}

template <typename Store> struct StoreOf;
template <> struct StoreOf<double> {
    static __device__ __forceinline__ double from(double v, float) { return v; }
};
template <> struct StoreOf<float> {
    static __device__ __forceinline__ float from(float v, float) { return v; }
};
template <> struct StoreOf<__bf16> {
    static __device__ __forceinline__ __bf16 from(float v, float) { return (__bf16)v; }
};
template <> struct StoreOf<uint8_t> {
    // OCP e4m3 with round-to-nearest-even after the operand pre-scale,
    // saturated to +-448
    static __device__ __forceinline__ uint8_t from(float v, float pre)
    {
        const float s = __builtin_amdgcn_fmed3f(v * pre, 448.0f, -448.0f);
        return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(s, s, 0, false) & 0xFF);
    }
};

// Column of each of the block's positions (kNoDrawColumn for padding) and
// its per-draw factor 1 / (n xi_j) (eq. (18) with a general xi; 1 for
// uniform draws), into LDS.  A gather unit is one wave (nthreads = kWave,
// tid its lane): it ends with the wave's LDS writes complete before any of its
// lanes reads them, with no workgroup barrier, so several waves of a
// workgroup can each run units of their own.
constexpr uint32_t kNoDrawColumn = 0xFFFFFFFFu;

template <typename Compute>
__device__ __forceinline__ void draw_block_columns(const GatherParams& prm, int64_t pos_base, int npos_block,
                                                   uint32_t k, uint32_t n, uint32_t sid_index, uint32_t* cols,
                                                   Compute* colf, int tid, int nthreads, const double* setw)
{
    for (int i = tid; i < npos_block; i += nthreads) {
        const int64_t t = draw_of_position(pos_base + i, prm.kc, prm.c, prm.c_prev, prm.stride);
        uint32_t j = kNoDrawColumn;
        Compute f = (Compute)1;
        if (setw) {
            // set form: the position's weight, or 0 for a repeat of an
            // earlier position's column (left zero, not generated)
            const double v = setw[pos_base + i];
            if (t >= 0 && v != 0.0) {
                j = draw_index((uint32_t)t, k, sid_index, prm.key0, prm.key1, n);
                f = (Compute)v;
            }
        } else if (t >= 0) {
            if (prm.cum) {
                const uint64_t total = prm.cum[n - 1];
                j = draw_index_weighted((uint32_t)t, k, sid_index, prm.key0, prm.key1, prm.cum, n, total);
                f = (Compute)((double)total / ((double)n * (double)prm.iw[j]));
            } else {
                j = draw_index((uint32_t)t, k, sid_index, prm.key0, prm.key1, n);
            }
        }
        cols[i] = j;
        colf[i] = f;
    }
    // (LDS operations of one wave complete in issue order: the fences and the
    // wave barrier only keep the compiler from moving the reads above the
    // writes; a workgroup-scope fence would also wait for the wave's global
    // stores of the previous unit)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Rows m .. m_pad - 1 of A's block and p .. p_pad - 1 of B's block are zero,
// so the sketch's entries outside the product see D = 0.
template <typename Compute, typename Store, int KPACK>
__device__ __forceinline__ void zero_padding_rows(const GatherParams& prm, int64_t pos_base, int octets, int64_t m,
                                                  int64_t p, int64_t m_pad, int64_t p_pad, Store* GA, Store* GB,
                                                  int tid, int nthreads)
{
    const uint32_t pad_a = (uint32_t)(m_pad - m), pad_rows = (uint32_t)(m_pad - m + p_pad - p);
    const Store zero = StoreOf<Store>::from((Compute)0, 1.0f);
    for (uint32_t it = (uint32_t)tid; it < pad_rows * (uint32_t)octets; it += (uint32_t)nthreads) {
        const uint32_t oc = it / pad_rows;
        const uint32_t qr = it - oc * pad_rows;
        const int64_t pos0 = pos_base + (int64_t)oc * kGatherPositions;
        const int npos = (int)((prm.kpad - pos0) < kGatherPositions ? (prm.kpad - pos0) : kGatherPositions);
        Store* G = qr < pad_a ? GA : GB;
        const int64_t R = qr < pad_a ? m_pad : p_pad;
        const int64_t row = qr < pad_a ? m + qr : p + (qr - pad_a);
        if constexpr (KPACK == 1) {
            for (int ip = 0; ip < npos; ++ip) G[(pos0 + ip) * R + row] = zero;
        } else {
            typedef Store vec_t __attribute__((ext_vector_type(KPACK)));
            vec_t vv;
#pragma unroll
            for (int ip = 0; ip < KPACK; ++ip) vv[ip] = zero;
            *reinterpret_cast<vec_t*>(G + ((pos0 / KPACK) * R + row) * KPACK) = vv;
        }
    }
}

// A block covers prm.octets groups of 8 consecutive padded positions of one
// realisation of one product; its lanes walk the (octet, quad of 4 rows)
// items, so a product with few rows still keeps every lane busy.
// V16: values from 16-bit uniforms, eight per Philox call (rows 8h .. 8h+7 per
// lane item instead of 4q .. 4q+3).
constexpr int kGatherMaxPos = kGatherPositions * kGatherMaxOctets;

// One gather block (bx: group of octets of positions, by: realisation slot,
// bz: product), by `nthreads` threads (tid the thread's index), with the
// LDS arrays cols and colf of kGatherMaxPos entries.
template <typename Compute, typename Store, int KPACK, int LAWS, bool V16>
__device__ __forceinline__ void gather_unit(const GatherParams& prm, uint32_t bx, uint32_t by, uint32_t bz, int tid,
                                            int nthreads, uint32_t* cols, Compute* colf)
{
    // the product's description is copied to registers once: the stores into
    // the gathered buffer below could otherwise alias it and force reloads
    const ProblemDesc* Pp = prm.descs + bz;
    const int64_t m = Pp->m, p = Pp->p;
    const int64_t m_pad = Pp->m_pad, p_pad = Pp->p_pad;
    const uint32_t n = (uint32_t)Pp->n;
    const uint32_t sid_problem = Pp->sid_problem;
    const int64_t rows_prefix = Pp->rows_prefix;
    constexpr bool kFp8 = sizeof(Store) == 1;
    LawEval<Compute> LA = LawEval<Compute>::make(Pp->A);
    LawEval<Compute> LB = LawEval<Compute>::make(Pp->B);
    float pre_a = Pp->pre_a, pre_b = Pp->pre_b;
    // FP8: each row of A (column of B) is multiplied by its factor 2^s before
    // the rounding to e4m3 (the sketch's MFMA scales undo it).  Two i.i.d.
    // laws have one factor each, folded exactly into their constants; other
    // law pairs (reparameterised operands) read the factor of every row from
    // the product's exponent tables.
    constexpr bool kRowScaled = kFp8 && LAWS == kLawsAny;
    const int8_t* exp_a = Pp->exp_a;
    const int8_t* exp_b = Pp->exp_b;
    if constexpr (kFp8 && !kRowScaled) {
        LA.mul *= pre_a; LA.add *= pre_a;
        LB.mul *= pre_b; LB.add *= pre_b;
    }
    if constexpr (kFp8) pre_a = pre_b = 1.0f;
    auto pa = [&](int64_t row) -> float {
        if constexpr (kRowScaled) return ldexpf(1.0f, (int)exp_a[row]);
        else return pre_a;
    };
    auto pb = [&](int64_t col) -> float {
        if constexpr (kRowScaled) return ldexpf(1.0f, (int)exp_b[col]);
        else return pre_b;
    };
    // FP8 values stay FP32 (saturated to +-448) until they are packed in pairs
    using Val = typename std::conditional<kFp8, float, Store>::type;
    auto to_val = [](Compute v, float pre) -> Val {
        if constexpr (kFp8) return __builtin_amdgcn_fmed3f((float)v * pre, 448.0f, -448.0f);
        else return StoreOf<Store>::from(v, pre);
    };
    const int64_t pos_base = (int64_t)bx * kGatherPositions * prm.octets;
    const int64_t slot = by;
    const uint32_t k = prm.k_first + (uint32_t)slot;
    const uint32_t sid_index = stream_id(kTagIndex, prm.level_field, sid_problem);
    const uint32_t sid_value = stream_id(kTagValue, prm.level_field, sid_problem);
    const int npos_block = (int)((prm.kpad - pos_base) < kGatherPositions * prm.octets ? (prm.kpad - pos_base)
                                                                                     : kGatherPositions * prm.octets);
    const int octets = (npos_block + kGatherPositions - 1) / kGatherPositions;
    const double* setw = prm.setw ? prm.setw + ((int64_t)bz * prm.batch + by) * prm.kpad : nullptr;
    draw_block_columns<Compute>(prm, pos_base, npos_block, k, n, sid_index, cols, colf, tid, nthreads, setw);
    const int64_t rows = m + p;
    const uint32_t quads = (uint32_t)ceil_div(rows, 4);
    const bool normal = LAWS == kLawsNormal || (LAWS == kLawsAny && (LA.kind != 1 || LB.kind != 1));
    const int64_t pass_rows = prm.batch * prm.kpad * (int64_t)prm.elem;
    Store* __restrict__ GA = reinterpret_cast<Store*>(prm.gbuf + pass_rows * rows_prefix) + slot * prm.kpad * m_pad;
    Store* __restrict__ GB = reinterpret_cast<Store*>(prm.gbuf + pass_rows * (rows_prefix + m_pad)) + slot * prm.kpad * p_pad;
    // The coarse sketch's weight enters through the operand: a_t of a coarse
    // draw (position < kc) is stored as omega a_t, so the sketch's K loop sums
    // w_t a_t b_t^T directly (D = (n / c_l) sum_t w_t a_t b_t^T, w_t = omega
    // for t < c_{l-1}, 1 otherwise).
    const Compute omega = (Compute)prm.omega;
    // values of rows 4q .. 4q+3 at the 8 positions of group oc
    // V16 helpers (the default path below keeps its own fused form, whose
    // code the compiler schedules better): values of rows 4q .. 4q+3 of one
    // position (column j, a_t weight wa) from their uniforms u and normals z,
    auto values4 = [&](int64_t q, uint32_t j, Compute wa, const Compute* u, const Compute* z, Val* out) {
        const int64_t e0 = 4 * q;
        if (e0 + 3 < m) {            // the whole quad is in A's column
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[r] = to_val(wa * LA.template eval<LAWS>(z[r], u[r], (int64_t)j * LA.ld + e0 + r), pa(e0 + r));
        } else if (e0 >= m) {        // the whole quad is in B's row
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[r] = to_val(LB.template eval<LAWS>(z[r], u[r], (int64_t)j * LB.ld + (e0 + r - m)), pb(e0 + r - m));
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t e = e0 + r;
                Compute v = (Compute)0;
                float pre = 1.0f;
                if (e < m) {
                    v = wa * LA.template eval<LAWS>(z[r], u[r], (int64_t)j * LA.ld + e);
                    pre = pa(e);
                } else if (e < rows) {
                    v = LB.template eval<LAWS>(z[r], u[r], (int64_t)j * LB.ld + (e - m));
                    pre = pb(e - m);
                }
                out[r] = to_val(v, pre);
            }
        }
    };
    // and their stores at the 8 positions of group oc.
    auto store4 = [&](uint32_t oc, int64_t q, Val (&vals)[kGatherPositions][4]) {
        const int64_t pos0 = pos_base + (int64_t)oc * kGatherPositions;
        const int npos = (int)((prm.kpad - pos0) < kGatherPositions ? (prm.kpad - pos0) : kGatherPositions);
        const int64_t e0 = 4 * q;
        if constexpr (KPACK == 1) {
            // rows 4q .. 4q+3 of one position are adjacent: one vector store
            // per position when the quad lies in A, or in B at an aligned row
            const bool in_a = e0 + 3 < m;
            const bool in_b = e0 >= m && e0 + 3 < rows && ((e0 - m) & 3) == 0;
            if (in_a || in_b) {
                typedef Store vec4_t __attribute__((ext_vector_type(4)));
                Store* G = in_a ? GA : GB;
                const int64_t R = in_a ? m_pad : p_pad;
                const int64_t row = in_a ? e0 : e0 - m;
#pragma unroll
                for (int ip = 0; ip < kGatherPositions; ++ip) {
                    if (ip < npos) {
                        vec4_t vv;
#pragma unroll
                        for (int r = 0; r < 4; ++r) vv[r] = vals[ip][r];
                        *reinterpret_cast<vec4_t*>(G + (pos0 + ip) * R + row) = vv;
                    }
                }
                return;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t e = e0 + r;
            if (e >= rows) break;
            Store* G = e < m ? GA : GB;
            const int64_t R = e < m ? m_pad : p_pad;
            const int64_t row = e < m ? e : e - m;
            if constexpr (KPACK == 1) {
#pragma unroll
                for (int ip = 0; ip < kGatherPositions; ++ip)
                    if (ip < npos) G[(pos0 + ip) * R + row] = vals[ip][r];
            } else if constexpr (kFp8) {
                // positions pos0 .. pos0+7 are one packed group of 8 draws:
                // OCP e4m3, round to nearest even, two values per conversion
                uint2 vv;
                int w = __builtin_amdgcn_cvt_pk_fp8_f32(vals[0][r], vals[1][r], 0, false);
                vv.x = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(vals[2][r], vals[3][r], w, true);
                w = __builtin_amdgcn_cvt_pk_fp8_f32(vals[4][r], vals[5][r], 0, false);
                vv.y = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(vals[6][r], vals[7][r], w, true);
                *reinterpret_cast<uint2*>(G + ((pos0 / KPACK) * R + row) * KPACK) = vv;
            } else {
                // positions pos0 .. pos0+7 are one packed group of 8 draws
                typedef Store vec_t __attribute__((ext_vector_type(KPACK)));
                vec_t vv;
#pragma unroll
                for (int ip = 0; ip < KPACK; ++ip) vv[ip] = vals[ip][r];
                *reinterpret_cast<vec_t*>(G + ((pos0 / KPACK) * R + row) * KPACK) = vv;
            }
        }
    };
    // values of rows 4q .. 4q+3 at the 8 positions of group oc: one
    // value-stream call per position (23-bit uniforms, four per call)
    auto generate = [&](uint32_t oc, int64_t q, const uint32_t* jv, const bool* ok) {
        const Compute* fv = colf + oc * kGatherPositions;
        const int64_t pos0 = pos_base + (int64_t)oc * kGatherPositions;
        const int npos = (int)((prm.kpad - pos0) < kGatherPositions ? (prm.kpad - pos0) : kGatherPositions);
        Val vals[kGatherPositions][4];
        const int64_t e0 = 4 * q;
#pragma unroll
        for (int ip = 0; ip < kGatherPositions; ++ip) {
            if (!ok[ip]) {
#pragma unroll
                for (int r = 0; r < 4; ++r) vals[ip][r] = to_val((Compute)0, 1.0f);
                continue;
            }
            const uint32_t j = jv[ip];
            const Compute wa = (pos0 + ip < prm.kc ? omega : (Compute)1) * fv[ip];
            const Words4 w = philox4x32_10((uint32_t)q, k, j, sid_value, prm.key0, prm.key1);
            Compute u[4], z[4];
            quad_values<Compute>(w, normal, u[0], u[1], u[2], u[3], z[0], z[1], z[2], z[3]);
            if (e0 + 3 < m) {            // the whole quad is in A's column
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    vals[ip][r] = to_val(wa * LA.template eval<LAWS>(z[r], u[r], (int64_t)j * LA.ld + e0 + r), pa(e0 + r));
            } else if (e0 >= m) {        // the whole quad is in B's row
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    vals[ip][r] = to_val(LB.template eval<LAWS>(z[r], u[r], (int64_t)j * LB.ld + (e0 + r - m)), pb(e0 + r - m));
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t e = e0 + r;
                    Compute v = (Compute)0;
                    float pre = 1.0f;
                    if (e < m) {
                        v = wa * LA.template eval<LAWS>(z[r], u[r], (int64_t)j * LA.ld + e);
                        pre = pa(e);
                    } else if (e < rows) {
                        v = LB.template eval<LAWS>(z[r], u[r], (int64_t)j * LB.ld + (e - m));
                        pre = pb(e - m);
                    }
                    vals[ip][r] = to_val(v, pre);
                }
            }
        }
        if constexpr (KPACK == 1) {
            // rows 4q .. 4q+3 of one position are adjacent: one vector store
            // per position when the quad lies in A, or in B at an aligned row
            const bool in_a = e0 + 3 < m;
            const bool in_b = e0 >= m && e0 + 3 < rows && ((e0 - m) & 3) == 0;
            if (in_a || in_b) {
                typedef Store vec4_t __attribute__((ext_vector_type(4)));
                Store* G = in_a ? GA : GB;
                const int64_t R = in_a ? m_pad : p_pad;
                const int64_t row = in_a ? e0 : e0 - m;
#pragma unroll
                for (int ip = 0; ip < kGatherPositions; ++ip) {
                    if (ip < npos) {
                        vec4_t vv;
#pragma unroll
                        for (int r = 0; r < 4; ++r) vv[r] = vals[ip][r];
                        *reinterpret_cast<vec4_t*>(G + (pos0 + ip) * R + row) = vv;
                    }
                }
                return;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t e = e0 + r;
            if (e >= rows) break;
            Store* G = e < m ? GA : GB;
            const int64_t R = e < m ? m_pad : p_pad;
            const int64_t row = e < m ? e : e - m;
            if constexpr (KPACK == 1) {
#pragma unroll
                for (int ip = 0; ip < kGatherPositions; ++ip)
                    if (ip < npos) G[(pos0 + ip) * R + row] = vals[ip][r];
            } else if constexpr (kFp8) {
                // positions pos0 .. pos0+7 are one packed group of 8 draws:
                // OCP e4m3, round to nearest even, two values per conversion
                uint2 vv;
                int w = __builtin_amdgcn_cvt_pk_fp8_f32(vals[0][r], vals[1][r], 0, false);
                vv.x = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(vals[2][r], vals[3][r], w, true);
                w = __builtin_amdgcn_cvt_pk_fp8_f32(vals[4][r], vals[5][r], 0, false);
                vv.y = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(vals[6][r], vals[7][r], w, true);
                *reinterpret_cast<uint2*>(G + ((pos0 / KPACK) * R + row) * KPACK) = vv;
            } else {
                // positions pos0 .. pos0+7 are one packed group of 8 draws
                typedef Store vec_t __attribute__((ext_vector_type(KPACK)));
                vec_t vv;
#pragma unroll
                for (int ip = 0; ip < KPACK; ++ip) vv[ip] = vals[ip][r];
                *reinterpret_cast<vec_t*>(G + ((pos0 / KPACK) * R + row) * KPACK) = vv;
            }
        }
    };
    // V16: rows 8h .. 8h+7 (quads 2h and 2h+1) from one call per position,
    // whose four words give eight 16-bit uniforms (element 8h + 2i + b takes
    // half b of word i); normals by Box-Muller on the two halves of a word
    auto generate16 = [&](uint32_t oc, int64_t h, const uint32_t* jv, const bool* ok) {
        const Compute* fv = colf + oc * kGatherPositions;
        const int64_t pos0 = pos_base + (int64_t)oc * kGatherPositions;
        const bool second = 2 * h + 1 < (int64_t)quads;
        Val lo[kGatherPositions][4], hi[kGatherPositions][4];
#pragma unroll
        for (int ip = 0; ip < kGatherPositions; ++ip) {
            if (!ok[ip]) {
#pragma unroll
                for (int r = 0; r < 4; ++r) lo[ip][r] = hi[ip][r] = to_val((Compute)0, 1.0f);
                continue;
            }
            const uint32_t j = jv[ip];
            const Compute wa = (pos0 + ip < prm.kc ? omega : (Compute)1) * fv[ip];
            const Words4 w = philox4x32_10((uint32_t)h, k, j, sid_value, prm.key0, prm.key1);
            const uint32_t wd[4] = {w.w0, w.w1, w.w2, w.w3};
            Compute u[8], z[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                u[2 * i] = unit16<Compute>(wd[i] & 0xFFFFu);
                u[2 * i + 1] = unit16<Compute>(wd[i] >> 16);
                if (normal) box_muller(u[2 * i], u[2 * i + 1], z[2 * i], z[2 * i + 1]);
                else z[2 * i] = z[2 * i + 1] = (Compute)0;
            }
            values4(2 * h, j, wa, u, z, lo[ip]);
            if (second) values4(2 * h + 1, j, wa, u + 4, z + 4, hi[ip]);
        }
        store4(oc, 2 * h, lo);
        if (second) store4(oc, 2 * h + 1, hi);
    };
    uint32_t jv[kGatherPositions];
    bool ok[kGatherPositions];
    if (octets == 1) {
        // one group: its columns are uniform over the block
#pragma unroll
        for (int ip = 0; ip < kGatherPositions; ++ip) {
            jv[ip] = cols[ip];
            ok[ip] = ip < npos_block && jv[ip] != kNoDrawColumn;
        }
        if constexpr (V16) {
            for (int64_t h = tid; h < (int64_t)((quads + 1) / 2); h += nthreads) generate16(0u, h, jv, ok);
        } else {
            for (int64_t q = tid; q < (int64_t)quads; q += nthreads) generate(0u, q, jv, ok);
        }
    } else {
        const uint32_t units = V16 ? (quads + 1) / 2 : quads;   // lane items per position group
        const uint32_t items = units * (uint32_t)octets;
        for (uint32_t it = (uint32_t)tid; it < items; it += (uint32_t)nthreads) {
            const uint32_t oc = it / units;
            const int npos = npos_block - (int)oc * kGatherPositions;
#pragma unroll
            for (int ip = 0; ip < kGatherPositions; ++ip) {
                jv[ip] = cols[oc * kGatherPositions + ip];
                ok[ip] = ip < npos && jv[ip] != kNoDrawColumn;
            }
            if constexpr (V16) generate16(oc, (int64_t)(it - oc * units), jv, ok);
            else generate(oc, (int64_t)(it - oc * units), jv, ok);
        }
    }
    zero_padding_rows<Compute, Store, KPACK>(prm, pos_base, octets, m, p, m_pad, p_pad, GA, GB, tid, nthreads);
}

template <typename Compute, typename Store, int KPACK, int LAWS, bool V16>
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(GatherParams prm)
{
    __shared__ uint32_t cols[kGatherMaxPos];
    // per-draw factor 1 / (n xi_j) of eq. (18) with weighted draws (1 uniform)
    __shared__ Compute colf[kGatherMaxPos];
    gather_unit<Compute, Store, KPACK, LAWS, V16>(prm, blockIdx.x, blockIdx.y, blockIdx.z, threadIdx.x, kGatherThreads,
                                                 cols, colf);
}

// The laws of the experiments of Sec. 4: every element is a Philox call and
// an FP64 evaluation of its own (experiment_value), so the block's lanes walk
// its (position, row) items row-fastest, one element each (a wave then shares
// one position: all of its lanes generate values, or all store padding), and
// store them into the same layouts as gather_kernel.  Not offered with FP8.
template <typename Compute, typename Store, int KPACK>
__global__ __launch_bounds__(kGatherThreads) void gather_experiment_kernel(GatherParams prm)
{
    __shared__ uint32_t cols[kGatherMaxPos];
    __shared__ Compute colf[kGatherMaxPos];
    const ProblemDesc* Pp = prm.descs + blockIdx.z;
    const int64_t m = Pp->m, p = Pp->p;
    const int64_t m_pad = Pp->m_pad, p_pad = Pp->p_pad;
    const uint32_t n = (uint32_t)Pp->n;
    const uint32_t sid_problem = Pp->sid_problem;
    const int64_t rows_prefix = Pp->rows_prefix;
    const Law LA = Pp->A, LB = Pp->B;
    const int64_t pos_base = (int64_t)blockIdx.x * kGatherPositions * prm.octets;
    const int64_t slot = blockIdx.y;
    const uint32_t k = prm.k_first + (uint32_t)slot;
    const uint32_t sid_index = stream_id(kTagIndex, prm.level_field, sid_problem);
    const uint32_t sid_exp = stream_id(kTagExperiment, prm.level_field, sid_problem);
    const int npos_block = (int)((prm.kpad - pos_base) < kGatherPositions * prm.octets ? (prm.kpad - pos_base)
                                                                                     : kGatherPositions * prm.octets);
    const int octets = (npos_block + kGatherPositions - 1) / kGatherPositions;
    const double* setw = prm.setw ? prm.setw + ((int64_t)blockIdx.z * prm.batch + slot) * prm.kpad : nullptr;
    draw_block_columns<Compute>(prm, pos_base, npos_block, k, n, sid_index, cols, colf, threadIdx.x, kGatherThreads,
                                setw);
    const int64_t rows = m + p;
    const int64_t pass_rows = prm.batch * prm.kpad * (int64_t)prm.elem;
    Store* __restrict__ GA = reinterpret_cast<Store*>(prm.gbuf + pass_rows * rows_prefix) + slot * prm.kpad * m_pad;
    Store* __restrict__ GB = reinterpret_cast<Store*>(prm.gbuf + pass_rows * (rows_prefix + m_pad)) + slot * prm.kpad * p_pad;
    const Compute omega = (Compute)prm.omega;
    const int64_t items = (int64_t)npos_block * rows;
    for (int64_t it = threadIdx.x; it < items; it += kGatherThreads) {
        const int ip = (int)(it / rows);
        const int64_t e = it - (int64_t)ip * rows;
        const int64_t pos = pos_base + ip;
        const uint32_t j = cols[ip];
        const bool in_a = e < m;
        Compute v = (Compute)0;
        if (j != kNoDrawColumn) {
            const Law& L = in_a ? LA : LB;
            v = (Compute)experiment_value(L.kind, L.loc, L.scale, L.aux, (uint32_t)e, k, j, sid_exp, prm.key0,
                                          prm.key1);
            // the coarse weight and the per-draw factor enter through a_t, as in gather_kernel
            if (in_a) v = ((pos < prm.kc ? omega : (Compute)1) * colf[ip]) * v;
        }
        Store* G = in_a ? GA : GB;
        const int64_t R = in_a ? m_pad : p_pad;
        const int64_t row = in_a ? e : e - m;
        G[((pos / KPACK) * R + row) * KPACK + (pos % KPACK)] = StoreOf<Store>::from(v, 1.0f);
    }
    zero_padding_rows<Compute, Store, KPACK>(prm, pos_base, octets, m, p, m_pad, p_pad, GA, GB, threadIdx.x,
                                             kGatherThreads);
}

// ---------------------------------------------------------------------------
// Sketch + coupling + per-entry Welford over a group of realisations.
// ---------------------------------------------------------------------------
struct SketchParams {
    const ProblemDesc* descs;
    const int32_t* tile_owner;   // global tile -> product
    int64_t total_tiles, groups;
    int64_t kc, kpad;
    int64_t batch;               // realisations in this pass
    int elem;
    uint32_t c;                  // c_l
    uint32_t c_prev;             // c_{l-1}, 0 at level 0
    TargetFunc func;             // STATS 4: f applied to both sketches
    const char* gbuf;
    void* part_mean;             // groups x sum_mp, in the accumulation type
    double* part_m2;             // groups x total_tiles
    int64_t sum_mp;
    // one group per pass: the epilogue merges straight into the level state
    int fuse;
    double done_before;          // realisations already in the level state
    double* level_mean;          // sum_mp, this level's running means
    double* tile_acc;            // total_tiles, this level's summed squared deviations per tile
};

// LDS fragment reads: the staged chunk keeps the global slab layout
// [position / KPACK][tile rows][KPACK] of the gathered buffer.
template <typename P> struct LdsFrag;
template <> struct LdsFrag<PolicyF64> {
    static __device__ __forceinline__ double load(const double* L, int BM, int kk, int row, int lane)
    {
        return L[(kk + lane / 16) * BM + row + lane % 16];
    }
};
template <> struct LdsFrag<PolicyF32> {
    static __device__ __forceinline__ float load(const float* L, int BM, int kk, int row, int lane)
    {
        return L[(kk + lane / 32) * BM + row + lane % 32];
    }
};
template <> struct LdsFrag<PolicyBF16> {
    static __device__ __forceinline__ bf16x8 load(const __bf16* L, int BM, int kk, int row, int lane)
    {
        return *reinterpret_cast<const bf16x8*>(L + ((kk / 8 + lane / 32) * BM + row + lane % 32) * 8);
    }
};
template <> struct LdsFrag<PolicyFP8> {
    // the lane's 32 draws are four packed groups of 8 of its row; groups
    // 4 (lane / 32) + q at or past valid8 (a step longer than its
    // realisation) are zero and not read
    static __device__ __forceinline__ i32x8 load(const uint8_t* L, int BM, int kk, int row, int lane, int valid8)
    {
        const int g0 = 4 * (lane / 32);
        const uint8_t* base = L + ((kk / 8 + g0) * BM + row + lane % 32) * 8;
        i32x8 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int2 w = make_int2(0, 0);
            if (g0 + q < valid8) w = *reinterpret_cast<const int2*>(base + q * BM * 8);
            v[2 * q] = w.x;
            v[2 * q + 1] = w.y;
        }
        return v;
    }
};

// draws staged per chunk: several MFMA steps per synchronisation
template <typename P> struct ChunkOf { static constexpr int KC = 64; };
template <> struct ChunkOf<PolicyF64> { static constexpr int KC = 16; };
template <> struct ChunkOf<PolicyF32> { static constexpr int KC = 32; };

// Workgroup = WR x WC waves; a wave computes NBR x NBC MFMA blocks of
// BLK x BLK; the workgroup tile is square (rows = columns = tile).
template <typename P, int WR, int WC, int NBR, int NBC>
struct SketchShape {
    static constexpr int THREADS = kWave * WR * WC;
    static constexpr int WTR = NBR * P::BLK, WTC = NBC * P::BLK;  // wave tile
    static constexpr int BM = WR * WTR;
    static_assert(BM == WC * WTC, "square workgroup tile");
};

// Shapes of the sketch's LDS staging: two buffers of [A, B][KC positions x
// BM rows], separate arrays so that the compiler sees the loads into one and
// the fragment reads from the other as disjoint (no wait on the loads in
// flight before each read).
template <typename P, int WR, int WC, int NBR, int NBC>
struct SketchStage {
    static constexpr int BM = SketchShape<P, WR, WC, NBR, NBC>::BM;
    static constexpr int KC = ChunkOf<P>::KC;
    using Buf = typename P::In[2][KC * BM];
};

// One sketch work item: output tile `item % total_tiles` over the
// realisations of group `item / total_tiles` of the pass, by the whole
// workgroup (every thread calls it; it synchronises the workgroup).
// STATS: 0 Welford; 1 sums shifted by E[D] (i.i.d. laws); 2 the same for
// products that fill whole tiles (no masking code); 3 (whole tiles, short
// realisations) a second accumulator collects every realisation's sum
// through the same MFMAs, so a realisation costs one fma per entry; 4 and 5
// a target function f of kind 1 and 2 (fixed at compile time, so only its
// own arithmetic is emitted per entry); 6 and 7 the same at level 0, which
// has no coarse sketch (no copied accumulators, fewer registers).
template <typename P, int WR, int WC, int NBR, int NBC, int STATS>
__device__ __forceinline__ void sketch_item(const SketchParams& prm, int64_t item,
                                            typename SketchStage<P, WR, WC, NBR, NBC>::Buf& lds0,
                                            typename SketchStage<P, WR, WC, NBR, NBC>::Buf& lds1, double* red)
{
    using In = typename P::In;
    using Acc = typename P::Acc;
    using FragT = typename P::FragT;
    using S = SketchShape<P, WR, WC, NBR, NBC>;
    constexpr int THREADS = S::THREADS;
    constexpr int NE = NBR * NBC * P::REGS;          // entries per lane
    constexpr int BM = S::BM;                        // workgroup tile edge
    constexpr int KC = ChunkOf<P>::KC;               // positions per staged chunk
    constexpr int SLABS = KC / P::KPACK;
    constexpr int VEC = 16 / (int)sizeof(In);        // elements per 16-byte vector
    constexpr int V_SLAB = BM * P::KPACK / VEC;      // vectors per slab of one operand
    constexpr int VPT = SLABS * V_SLAB / THREADS;    // vectors per thread per operand
    static_assert(SLABS * V_SLAB % THREADS == 0, "chunk must split evenly over the workgroup");

    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int wrow = (wave / WC) * S::WTR, wcol = (wave % WC) * S::WTC;  // wave tile inside the workgroup tile
    {
        const int64_t group = item / prm.total_tiles;
        const int64_t tt = item % prm.total_tiles;
        const ProblemDesc& Pd = prm.descs[prm.tile_owner[tt]];
        const int tile = (int)(tt - Pd.tile_first);
        const int m = (int)Pd.m, p = (int)Pd.p, m_pad = (int)Pd.m_pad, p_pad = (int)Pd.p_pad;
        const int trow = (tile / (int)Pd.tiles_n) * BM, tcol = (tile % (int)Pd.tiles_n) * BM;
        const int64_t s_begin = group * prm.batch / prm.groups;
        const int64_t s_end = (group + 1) * prm.batch / prm.groups;
        const int64_t pass_rows = prm.batch * prm.kpad * (int64_t)prm.elem;
        // the group's realisations are consecutive blocks [kpad / KPACK][rows][KPACK]:
        // position P of the group's stream (P = s kpad + k) sits at element P * rows
        const In* GA0 = reinterpret_cast<const In*>(prm.gbuf + pass_rows * Pd.rows_prefix) + s_begin * prm.kpad * m_pad;
        const In* GB0 = reinterpret_cast<const In*>(prm.gbuf + pass_rows * (Pd.rows_prefix + m_pad)) +
                        s_begin * prm.kpad * p_pad;
        const double scale64 = (double)Pd.n / (double)prm.c;
        const Acc scale = (Acc)scale64;
        const int kc = (int)prm.kc;
        const int kpad = (int)prm.kpad;
        const int npos = (int)(s_end - s_begin) * kpad;     // positions of the group's stream
        const int total = (npos + KC - 1) / KC;             // chunks; a chunk may span realisations

        // Chunk c holds stream positions [c KC, c KC + KC).  Its loads go
        // straight from global memory into LDS buffer c & 1
        // (global_load_lds_dwordx4: the 16 bytes of lane i land at the wave's
        // base plus 16 i, which is the staging layout), so no registers hold
        // them; chunk c + 1 is in flight while the MFMAs run on chunk c.
        // Vectors past the group's positions are not loaded (their LDS slots
        // are never read).
        auto fetch = [&](auto which, int c) {
            In (&dst)[2][KC * BM] = decltype(which)::value ? lds1 : lds0;
            const int k0 = c * KC;
            const In* ga = GA0 + (int64_t)k0 * m_pad;
            const In* gb = GB0 + (int64_t)k0 * p_pad;
#pragma unroll
            for (int v = 0; v < VPT; ++v) {
                const int vid = threadIdx.x + v * THREADS;
                const int slab = vid / V_SLAB, iv = vid % V_SLAB;
                const int wbase = (wave * kWave + v * THREADS) * VEC;   // the wave's first vector
                if (k0 + slab * P::KPACK < npos) {
                    __builtin_amdgcn_global_load_lds(
                        (GlobalPtr)(ga + (slab * m_pad + trow) * P::KPACK + iv * VEC), (LdsPtr)&dst[0][wbase], 16,
                        0, 0);
                    __builtin_amdgcn_global_load_lds(
                        (GlobalPtr)(gb + (slab * p_pad + tcol) * P::KPACK + iv * VEC), (LdsPtr)&dst[1][wbase], 16,
                        0, 0);
                }
            }
        };

        // Per entry one running value: the Welford mean, or (SHIFTED) the sum
        // of acc - shift, where shift = E[D] / scale in accumulator units
        // (n E[a] E[b] at level 0, 0 above it: E[D_l] = 0).  The squared
        // deviations of a realisation are summed over the lane's entries into
        // one FP64 sum (only the sum over entries enters V_l).  Entries
        // outside the product see zero-padded operand rows: D = 0 there, and
        // the shift is not applied to them.
        constexpr bool DUAL = STATS == 3;
        // STATS 4, 5: a target function f.  The accumulator is copied when the
        // coarse draws are done (the gathered a_t are unweighted), and the
        // level sample of every entry is f(n / c_l acc) - f(n / c_{l-1} snap),
        // or f(n / c_0 acc) at level 0, into Welford's mean and M2.
        constexpr bool FUNC = STATS >= 4;
        constexpr int fkind = FUNC ? (STATS - 4) % 2 + 1 : 0;
        constexpr bool FUNC_COARSE = STATS == 4 || STATS == 5;   // levels above 0
        Acc run[DUAL ? 1 : NE];
#pragma unroll
        for (int e = 0; e < (DUAL ? 1 : NE); ++e) run[e] = (Acc)0;
        typename P::AccVec tot[DUAL ? NBR : 1][DUAL ? NBC : 1];
        if constexpr (DUAL) {
#pragma unroll
            for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                    for (int r = 0; r < P::REGS; ++r) tot[bi][bj][r] = (Acc)0;
        }
        typename P::AccVec snap[FUNC_COARSE ? NBR : 1][FUNC_COARSE ? NBC : 1];
        const bool has_coarse = FUNC_COARSE && prm.c_prev > 0u;
        const Acc scale_c = (Acc)(has_coarse ? (double)Pd.n / (double)prm.c_prev : 0.0);
        const Acc th0 = (Acc)prm.func.theta0, th1 = (Acc)prm.func.theta1;
        double m2_sum = 0.0;
        Acc count = (Acc)0;
        constexpr bool SHIFTED = STATS >= 1 && STATS <= 3;
        const Acc shift = SHIFTED && kc == 0 ? (Acc)(Pd.mean0 / scale64) : (Acc)0;
        // with a non-zero shift, entries outside the product (ragged tiles only)
        // are masked: bit e of `inside` is set for an entry inside the product
        static_assert(NE <= 64, "one mask bit per entry");
        const bool ragged = STATS == 1 && shift != (Acc)0 && (trow + BM > m || tcol + BM > p);
        uint64_t inside = ~0ull;
        if (ragged) {
            inside = 0ull;
            int e = 0;
#pragma unroll
            for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                    for (int r = 0; r < P::REGS; ++r, ++e) {
                        const int i = trow + wrow + bi * P::BLK + P::row_of(lane, r);
                        const int j = tcol + wcol + bj * P::BLK + P::col_of(lane);
                        if (i < m && j < p) inside |= 1ull << e;
                    }
        }
        typename P::AccVec acc[NBR][NBC];
#pragma unroll
        for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
            for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                for (int r = 0; r < P::REGS; ++r) acc[bi][bj][r] = (Acc)0;

        // FP8: the E8M0 scales of the lane's rows of A and columns of B
        // (127 - s for the factor 2^s the gather applied), fixed for the tile
        int sa[P::SCALED ? NBR : 1], sb[P::SCALED ? NBC : 1];
        if constexpr (P::SCALED) {
#pragma unroll
            for (int bi = 0; bi < NBR; ++bi) sa[bi] = 127 - (int)Pd.exp_a[trow + wrow + bi * P::BLK + lane % 32];
#pragma unroll
            for (int bj = 0; bj < NBC; ++bj) sb[bj] = 127 - (int)Pd.exp_b[tcol + wcol + bj * P::BLK + lane % 32];
        }
        // FP8: a realisation shorter than the MFMA's 64 draws (kpad 16 or 32,
        // a divisor of 64, so it never crosses a chunk) is one step whose
        // fragments are zero past its draws; otherwise steps are whole
        int SL = P::KSTEP;
        if constexpr (P::SCALED) SL = kpad < P::KSTEP ? kpad : P::KSTEP;
        // one MFMA step at position offset kk of the staged chunk.  FP32 and
        // narrower: the first step of a realisation starts its accumulator
        // from zero (the MFMA's accumulator input is the constant 0, no
        // clearing after the previous realisation); FP64 clears the
        // accumulator after each realisation (a second copy of the step would
        // not fit its registers)
        constexpr bool kZeroStart = sizeof(In) <= 4;
        auto step = [&](const In* LA, const In* LB, int kk, auto first) {
            constexpr bool FIRST = decltype(first)::value;
            const typename P::AccVec zero = {};
            FragT a[NBR], b[NBC];
            if constexpr (P::SCALED) {
#pragma unroll
                for (int bi = 0; bi < NBR; ++bi) a[bi] = LdsFrag<P>::load(LA, BM, kk, wrow + bi * P::BLK, lane, SL / 8);
#pragma unroll
                for (int bj = 0; bj < NBC; ++bj) b[bj] = LdsFrag<P>::load(LB, BM, kk, wcol + bj * P::BLK, lane, SL / 8);
            } else {
#pragma unroll
                for (int bi = 0; bi < NBR; ++bi) a[bi] = LdsFrag<P>::load(LA, BM, kk, wrow + bi * P::BLK, lane);
#pragma unroll
                for (int bj = 0; bj < NBC; ++bj) b[bj] = LdsFrag<P>::load(LB, BM, kk, wcol + bj * P::BLK, lane);
            }
#pragma unroll
            for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                for (int bj = 0; bj < NBC; ++bj) {
                    if constexpr (P::SCALED) {
                        acc[bi][bj] = P::mma(a[bi], b[bj], FIRST ? zero : acc[bi][bj], sa[bi], sb[bj]);
                        if constexpr (DUAL) tot[bi][bj] = P::mma(a[bi], b[bj], tot[bi][bj], sa[bi], sb[bj]);
                    } else {
                        acc[bi][bj] = P::mma(a[bi], b[bj], FIRST ? zero : acc[bi][bj]);
                        if constexpr (DUAL) tot[bi][bj] = P::mma(a[bi], b[bj], tot[bi][bj]);
                    }
                }
        };
        // the realisation is complete: D = scale * acc enters the statistics
        // The squared deviations go into kParts independent partial sums
        // (entry e into part e % kParts): one running sum would chain every
        // entry's fma on the previous one.
        constexpr int kParts = 4;
        static_assert(kParts == 4, "the partial sums are added pairwise below");
        auto realisation_done = [&]() {
            count += (Acc)1;
            Acc part[kParts];
#pragma unroll
            for (int q = 0; q < kParts; ++q) part[q] = (Acc)0;
            int e = 0;
            if constexpr (DUAL) {
#pragma unroll
                for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                    for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                        for (int r = 0; r < P::REGS; ++r, ++e) {
                            const Acc d = acc[bi][bj][r] - shift;
                            part[e % kParts] = fma(d, d, part[e % kParts]);
                        }
            } else if constexpr (SHIFTED) {
                if (!ragged) {
#pragma unroll
                    for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                        for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                            for (int r = 0; r < P::REGS; ++r, ++e) {
                                const Acc d = acc[bi][bj][r] - shift;
                                run[e] += d;
                                part[e % kParts] = fma(d, d, part[e % kParts]);
                            }
                } else {
#pragma unroll
                    for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                        for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                            for (int r = 0; r < P::REGS; ++r, ++e) {
                                const Acc d = ((inside >> e) & 1ull) ? acc[bi][bj][r] - shift : (Acc)0;
                                run[e] += d;
                                part[e % kParts] = fma(d, d, part[e % kParts]);
                            }
                }
            } else {
                const Acc inv = (Acc)1 / count;
#pragma unroll
                for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                    for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                        for (int r = 0; r < P::REGS; ++r, ++e) {
                            Acc d;
                            if constexpr (FUNC) {
                                d = target_value(fkind, scale * acc[bi][bj][r], th0, th1);
                                if constexpr (FUNC_COARSE)
                                    if (has_coarse) d -= target_value(fkind, scale_c * snap[bi][bj][r], th0, th1);
                            } else {
                                d = scale * acc[bi][bj][r];
                            }
                            const Acc delta = d - run[e];
                            run[e] += delta * inv;
                            part[e % kParts] += delta * (d - run[e]);
                        }
            }
            if constexpr (!kZeroStart) {
#pragma unroll
                for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                    for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                        for (int r = 0; r < P::REGS; ++r) acc[bi][bj][r] = (Acc)0;
            }
            m2_sum += (double)((part[0] + part[1]) + (part[2] + part[3]));
        };

        if (total > 0) fetch(std::integral_constant<int, 0>(), 0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        int o = 0;                               // position within the current realisation
        // chunk c from buffer c & 1 (a compile-time choice), chunk c + 1 into
        // the other buffer, which every wave finished reading before the
        // previous barrier
        auto chunk = [&](auto which, int c) {
            constexpr int W = decltype(which)::value;
            if (c + 1 < total) fetch(std::integral_constant<int, 1 - W>(), c + 1);
            const In* LA = W ? lds1[0] : lds0[0];
            const In* LB = W ? lds1[1] : lds0[1];
            const int left = npos - c * KC;
            const int steps = (left < KC ? left : KC) / SL;
            // runs of steps that end at the chunk's end or the end of a realisation
            for (int st = 0; st < steps;) {
                // FUNC: a run also ends where the coarse draws end (o = kc)
                const int stop = FUNC && o < kc ? kc : kpad;
                int run_steps = (stop - o) / SL;
                if (run_steps > steps - st) run_steps = steps - st;
                int i = 0;
                if constexpr (kZeroStart) {
                    if (o == 0 && run_steps > 0) {
                        step(LA, LB, st * SL, std::true_type());
                        i = 1;
                    }
                }
                for (; i < run_steps; ++i) step(LA, LB, (st + i) * SL, std::false_type());
                st += run_steps;
                o += run_steps * SL;
                if constexpr (FUNC_COARSE) {
                    if (kc > 0 && o == kc) {
#pragma unroll
                        for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
                            for (int bj = 0; bj < NBC; ++bj) snap[bi][bj] = acc[bi][bj];
                    }
                }
                if (o == kpad) {
                    realisation_done();
                    o = 0;
                }
            }
            __builtin_amdgcn_s_waitcnt(0);      // this wave's loads of chunk c + 1
            __syncthreads();
        };
        for (int c = 0; c < total; c += 2) {
            chunk(std::integral_constant<int, 0>(), c);
            if (c + 1 < total) chunk(std::integral_constant<int, 1>(), c + 1);
        }

        // group mean of every in-range entry, and the group's within sum of
        // squares.  With one group per pass (fuse) the group is merged here
        // into the level's running mean (Chan, FP64: the merge kernel's
        // arithmetic), its between-part added to the tile's slot.
        Acc* pm = static_cast<Acc*>(prm.part_mean) + group * prm.sum_mp + Pd.mp_prefix;
        double* mu_row = prm.level_mean + Pd.mp_prefix;
        const double na = prm.done_before, nb = (double)count, nn = na + nb;
        double sq_mean = 0.0, between = 0.0;
        int e = 0;
#pragma unroll
        for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
            for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
                for (int r = 0; r < P::REGS; ++r, ++e) {
                    const int i = trow + wrow + bi * P::BLK + P::row_of(lane, r);
                    const int j = tcol + wcol + bj * P::BLK + P::col_of(lane);
                    if (i < m && j < p) {
                        Acc gm;
                        if constexpr (SHIFTED) {
                            // DUAL: the running total minus count shifts
                            double s1;
                            if constexpr (DUAL) s1 = (double)tot[bi][bj][r] - (double)count * (double)shift;
                            else s1 = (double)run[e];
                            sq_mean += s1 * s1;
                            gm = (Acc)(scale64 * ((double)shift + s1 / (double)count));
                        } else {
                            gm = run[e];
                        }
                        const int64_t idx = (int64_t)i * p + j;
                        if (prm.fuse) {
                            const double mu = mu_row[idx];
                            const double delta = (double)gm - mu;
                            mu_row[idx] = mu + delta * (nb / nn);
                            between += delta * delta * (na * nb / nn);
                        } else {
                            pm[idx] = gm;
                        }
                    }
                }
        // SHIFTED: sum (d - dbar)^2 = sum d^2 - sum_e s1_e^2 / count, in scale^2 units
        double m2_group = m2_sum;
        if constexpr (SHIFTED) m2_group = count > (Acc)0 ? scale64 * scale64 * (m2_sum - sq_mean / (double)count) : 0.0;
        double tile_sum = m2_group + between;
        for (int off = kWave / 2; off > 0; off >>= 1) tile_sum += __shfl_xor(tile_sum, off, kWave);
        if (lane == 0) red[wave] = tile_sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int w = 0; w < THREADS / kWave; ++w) tot += red[w];
            if (prm.fuse) prm.tile_acc[tt] += tot;
            else prm.part_m2[group * prm.total_tiles + tt] = tot;
        }
        __syncthreads();
    }
}

// A grid of workgroups walking the pass's items; WPE: waves per SIMD the
// register allocation must leave room for.
template <typename P, int WR, int WC, int NBR, int NBC, int WPE, int STATS>
__global__ __launch_bounds__(kWave * WR * WC, WPE) void sketch_kernel(SketchParams prm)
{
    using St = SketchStage<P, WR, WC, NBR, NBC>;
    __shared__ __align__(16) typename St::Buf lds0;
    __shared__ __align__(16) typename St::Buf lds1;
    __shared__ double red[SketchShape<P, WR, WC, NBR, NBC>::THREADS / kWave];
    const int64_t items = prm.total_tiles * prm.groups;
    // Workgroups are dealt to the 8 XCDs round-robin by id; renumber them so
    // that each XCD walks a contiguous run of items (one group's consecutive
    // tiles), whose workgroups then share operand rows through that XCD's L2.
    // The grid is a multiple of kXcds.
    const int64_t first = (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
    for (int64_t item = first; item < items; item += gridDim.x)
        sketch_item<P, WR, WC, NBR, NBC, STATS>(prm, item, lds0, lds1, red);
}

}  // namespace mlmc
