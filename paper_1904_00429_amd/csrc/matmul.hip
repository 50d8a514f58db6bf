// Matrix-product MLMC pipeline (Sec. 3; Alg. 1 per level) over a table of
// independent products (one product is the one-entry table).  Described for
// f = identity and the prefix coupling; a target function f keeps the coarse
// sum apart (the accumulator is copied where the coarse draws end), weighted
// draws scale a_t by 1 / (n xi_j), the stride coupling places the draws
// M - 1, 2M - 1, ... in the coarse segment, and the laws of Sec. 4 have a
// gather of their own.
//
// Per pass over a batch of S realisations of one level l (every product of
// the table shares the ladder and N_l; each has its own shape, law and
// Philox stream id):
//   1. gather:  draw the c_l indices of every realisation (index stream) and
//      generate only the sampled columns a_t = A^(k)[:, r_t] and rows
//      b_t = B^(k)[r_t, :] (value stream, keyed by the column j = r_t), in the
//      operand precision, into a gathered buffer laid out for the MFMA
//      fragments.  Draws t < c_{l-1} (the coarse segment) and the remaining
//      draws (the fine segment) are each zero-padded to the contraction step;
//      the coarse draws' a_t are stored multiplied by 1 - c_l / c_{l-1}.
//   2. sketch:  a persistent grid walks the (product, output tile, group of
//      realisations) work items.  Per realisation the K loop sums
//      w_t a_t b_t^T over all c_l draws (w_t = 1 - c_l / c_{l-1} for the
//      coarse draws, 1 for the rest): the result times n / c_l is
//      D_k = Z_l^(k) - Z_{l-1}^(k) (the coupled fine-minus-coarse sample of
//      Alg. 1) without ever forming either sketch.  Each entry's running
//      statistic over the group's realisations is kept in registers.
//   3. merge:   per entry, a fixed-order Chan merge of the group means into
//      the level's running mean (FP64); the between-group part of the sum of
//      squared deviations is reduced per block, the within-group parts are
//      summed by one thread.  V_l = (within + between) / (N_l - 1).  With one
//      group per tile the sketch's epilogue does this merge itself.
// After the last level, `finalize` forms V_l and the telescoping sum
// Y = sum_l Ybar_l (eq. (10)) of every product.
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
// uniform draws), into LDS; ends with a barrier.
constexpr uint32_t kNoDrawColumn = 0xFFFFFFFFu;

template <typename Compute>
__device__ __forceinline__ void draw_block_columns(const GatherParams& prm, int64_t pos_base, int npos_block,
                                                   uint32_t k, uint32_t n, uint32_t sid_index, uint32_t* cols,
                                                   Compute* colf, int tid, int nthreads)
{
    for (int i = tid; i < npos_block; i += nthreads) {
        const int64_t t = draw_of_position(pos_base + i, prm.kc, prm.c, prm.c_prev, prm.stride);
        uint32_t j = kNoDrawColumn;
        Compute f = (Compute)1;
        if (t >= 0) {
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
    __syncthreads();
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
    draw_block_columns<Compute>(prm, pos_base, npos_block, k, n, sid_index, cols, colf, tid, nthreads);
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
    draw_block_columns<Compute>(prm, pos_base, npos_block, k, n, sid_index, cols, colf, threadIdx.x, kGatherThreads);
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

// WPE: waves per SIMD the register allocation must leave room for.
// STATS: 0 Welford; 1 sums shifted by E[D] (i.i.d. laws); 2 the same for
// products that fill whole tiles (no masking code); 3 (whole tiles, short
// realisations) a second accumulator collects every realisation's sum
// through the same MFMAs, so a realisation costs one fma per entry; 4 and 5
// a target function f of kind 1 and 2 (fixed at compile time, so only its
// own arithmetic is emitted per entry); 6 and 7 the same at level 0, which
// has no coarse sketch (no copied accumulators, fewer registers).
template <typename P, int WR, int WC, int NBR, int NBC, int WPE, int STATS>
__global__ __launch_bounds__(kWave * WR * WC, WPE) void sketch_kernel(SketchParams prm)
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
    // two staging buffers, separate arrays so that the compiler sees the
    // loads into one and the fragment reads from the other as disjoint (no
    // wait on the loads in flight before each read)
    __shared__ __align__(16) In lds0[2][KC * BM];     // [A, B][chunk]
    __shared__ __align__(16) In lds1[2][KC * BM];
    __shared__ double red[THREADS / kWave];

    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int wrow = (wave / WC) * S::WTR, wcol = (wave % WC) * S::WTC;  // wave tile inside the workgroup tile
    const int64_t items = prm.total_tiles * prm.groups;
    // Workgroups are dealt to the 8 XCDs round-robin by id; renumber them so
    // that each XCD walks a contiguous run of items (one group's consecutive
    // tiles), whose workgroups then share operand rows through that XCD's L2.
    // The grid is a multiple of kXcds.
    const int64_t first = (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
    for (int64_t item = first; item < items; item += gridDim.x) {
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

// ---------------------------------------------------------------------------
// Merge of a pass's groups into the level state; finalize.
// ---------------------------------------------------------------------------
struct MergeParams {
    const ProblemDesc* descs;
    int level;
    int64_t batch, groups, total_tiles, sum_mp, sum_merge_blocks, nprob;
    double done_before;          // realisations already in the level state
    const void* part_mean;       // groups x sum_mp, PartT
    const double* part_m2;
    double* means;               // levels x sum_mp
    double* between;             // levels x sum_merge_blocks
    double* within;              // levels x nprob
};

// PartT: the sketch's accumulation type, in which it wrote the group means.
template <typename PartT>
__global__ __launch_bounds__(kMergeThreads) void merge_kernel(MergeParams prm)
{
    __shared__ double red[kMergeThreads];
    const int64_t pi = blockIdx.y;
    const ProblemDesc& Pd = prm.descs[pi];
    if ((int64_t)blockIdx.x >= Pd.merge_blocks) return;
    const int64_t mp = Pd.m * Pd.p;
    const int64_t e = (int64_t)blockIdx.x * kMergeThreads + threadIdx.x;
    double between = 0.0;
    if (e < mp) {
        double* mean = prm.means + prm.level * prm.sum_mp + Pd.mp_prefix;
        double mu = mean[e];
        double na = prm.done_before;
        const PartT* part = static_cast<const PartT*>(prm.part_mean) + Pd.mp_prefix + e;
        const uint32_t batch = (uint32_t)prm.batch, groups = (uint32_t)prm.groups;
        for (uint32_t g = 0; g < groups; ++g) {
            // group g holds realisations [g batch / groups, (g + 1) batch / groups)
            const double nb = (double)((g + 1) * batch / groups - g * batch / groups);
            const double n = na + nb;
            const double delta = (double)part[(int64_t)g * prm.sum_mp] - mu;
            mu += delta * (nb / n);
            between += delta * delta * (na * nb / n);
            na = n;
        }
        mean[e] = mu;
    }
    red[threadIdx.x] = between;
    __syncthreads();
    for (int half = kMergeThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) prm.between[prm.level * prm.sum_merge_blocks + Pd.between_prefix + blockIdx.x] += red[0];
    if (blockIdx.x == 0) {
        // within-group sums of this product: strided over the block, then a tree
        __syncthreads();
        double w = 0.0;
        const int64_t count = prm.groups * Pd.tiles;
        for (int64_t i = threadIdx.x; i < count; i += kMergeThreads)
            w += prm.part_m2[(i / Pd.tiles) * prm.total_tiles + Pd.tile_first + (i % Pd.tiles)];
        red[threadIdx.x] = w;
        __syncthreads();
        for (int half = kMergeThreads / 2; half > 0; half >>= 1) {
            if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
            __syncthreads();
        }
        if (threadIdx.x == 0) prm.within[prm.level * prm.nprob + pi] += red[0];
    }
}

struct FinalizeParams {
    const ProblemDesc* descs;
    int num_levels;
    int64_t sum_mp, sum_merge_blocks, nprob;
    double counts[32];
    const double* means;
    const double* between;       // levels x sum_merge_blocks
    const double* within;        // levels x nprob
    const double* tile_acc;      // levels x total_tiles (passes merged by the sketch)
    int64_t total_tiles;
    double* var;                 // levels x nprob
};

__global__ __launch_bounds__(kMergeThreads) void level_var_kernel(FinalizeParams prm)
{
    __shared__ double red[kMergeThreads];
    const int l = blockIdx.x;
    const int64_t pi = blockIdx.y;
    const ProblemDesc& Pd = prm.descs[pi];
    const double* bt = prm.between + l * prm.sum_merge_blocks + Pd.between_prefix;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < Pd.merge_blocks; b += kMergeThreads) s += bt[b];
    const double* ta = prm.tile_acc + l * prm.total_tiles + Pd.tile_first;
    for (int64_t t = threadIdx.x; t < Pd.tiles; t += kMergeThreads) s += ta[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int half = kMergeThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = prm.counts[l];
        prm.var[l * prm.nprob + pi] = n > 1.0 ? (red[0] + prm.within[l * prm.nprob + pi]) / (n - 1.0) : 0.0;
    }
}

__global__ __launch_bounds__(kMergeThreads) void telescope_kernel(FinalizeParams prm)
{
    const ProblemDesc& Pd = prm.descs[blockIdx.y];
    const int64_t mp = Pd.m * Pd.p;
    const int64_t e = (int64_t)blockIdx.x * kMergeThreads + threadIdx.x;
    if (e >= mp) return;
    double y = 0.0;
    for (int l = 0; l < prm.num_levels; ++l) {
        const double v = prm.means[l * prm.sum_mp + Pd.mp_prefix + e];
        y += v;
        if (Pd.level_means) Pd.level_means[l * mp + e] = v;
    }
    Pd.out[e] = y;
}

__global__ void fill_kernel(double* p, int64_t count, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Host side: plan, passes, finalize.
// ---------------------------------------------------------------------------
// kmem: the shortest padded realisation (FP8: 16 draws, whose MFMA step of
// 64 draws then reads zeros past them; the others pad to whole steps)
struct PolicyShape {
    int kstep, kpack, blk, elem, kmem;
};

static PolicyShape policy_shape(int prec)
{
    switch (prec) {
    case 0: return {PolicyF64::KSTEP, 1, PolicyF64::BLK, 8, PolicyF64::KSTEP};
    case 1: return {PolicyF32::KSTEP, 1, PolicyF32::BLK, 4, PolicyF32::KSTEP};
    case 2: return {PolicyBF16::KSTEP, PolicyBF16::KPACK, PolicyBF16::BLK, 2, PolicyBF16::KSTEP};
    default: return {PolicyFP8::KSTEP, PolicyFP8::KPACK, PolicyFP8::BLK, 1, 16};
    }
}

static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

static void level_padding(const MatmulPlan& plan, int64_t c, int64_t c_prev, int64_t& kc, int64_t& kpad)
{
    if (plan.func.kind == 0) {
        // the coarse weight is folded into the operands: the coarse and fine
        // draws are one run of positions, padded once, to a divisor of the
        // contraction step (FP8: 16 or 32 draws) or to whole steps
        kc = c_prev;
        kpad = round_up(c, plan.kmem);
        if (kpad > plan.kstep || plan.kstep % kpad != 0) kpad = round_up(kpad, plan.kstep);
        kpad = round_up(kpad, plan.kpack);
        return;
    }
    // a target function copies the accumulator where the coarse draws end:
    // that boundary falls on a contraction step
    kc = round_up(c_prev, plan.kstep);
    kpad = kc + round_up(c - c_prev, plan.kstep);
    // the packed layouts group 8 positions; the gather kernel writes whole groups
    kpad = round_up(kpad, plan.kpack);
}

// FP8 scale rule: the exponent s of the factor 2^s that each row of A (column
// of B) is multiplied by before its rounding to e4m3: the largest s with
// 2^s bound <= 256 (entries up to the bound sit in e4m3's top binades, below
// its largest value 448), clamped to [-20, 20], 0 for a zero bound.  Exact:
// bound = f 2^E with f in [1/2, 1) gives s = 8 - E, or 9 - E when f = 1/2.
__host__ __device__ inline int fp8_scale_exponent(double bound)
{
    if (!(bound > 0.0)) return 0;
    int E;
    const double f = frexp(bound, &E);
    int s = 8 - E + (f == 0.5 ? 1 : 0);
    return s < -20 ? -20 : (s > 20 ? 20 : s);
}

// Bound of the entries of an i.i.d. law: |loc| + 6 |scale| (normal, as
// fma(6, |scale|, |loc|)) or |loc| + |scale| (uniform); reparameterised laws
// take fma(6, |stdev|, |mean|) per entry, maximised over each row of A
// (column of B) on the device (fp8_bound_kernel).
static double fp8_iid_bound(const Law& law)
{
    if (law.kind == 0) return fma(6.0, fabs(law.scale), fabs(law.loc));
    return fabs(law.loc) + fabs(law.scale);
}

bool matmul_plan(const MatmulProblem* probs, int nprob, int prec, int num_levels, const int64_t* c,
                 const MatmulTuning* tune, const TargetFunc& func, const uint32_t* index_weights,
                 MatmulPlan& plan)
{
    plan = MatmulPlan();
    plan.func = func;
    plan.index_weights = index_weights;
    if (index_weights && (nprob != 1 || prec == 3)) return false;   // one product; not FP8 (range of 1/xi)
    if (nprob < 1) return false;
    plan.prec = prec;
    plan.num_levels = num_levels;
    plan.nprob = nprob;
    for (int l = 0; l < num_levels; ++l) plan.c[l] = c[l];
    const PolicyShape ps = policy_shape(prec);
    plan.kstep = ps.kstep;
    plan.kmem = ps.kmem;
    plan.kpack = ps.kpack;
    plan.elem = ps.elem;
    // workgroup tile: 128 (4 x 2 waves of 32 x 64) for the 32 x 32 MFMA
    // blocks unless tuned to 64 (2 x 2 waves of 32 x 32); f64 blocks are 16
    // wide and always use tile 64 (2 x 2 waves of 32 x 32 in 16 x 16 blocks)
    plan.nb = 2;
    int want_tile = tune && tune->tile > 0 ? tune->tile : 0;
    if (const char* env = getenv("MLMC_SKETCH_TILE")) {
        const int v = atoi(env);
        if (v == 64 || v == 128) want_tile = v;
    }
    if (want_tile > 0 && prec != 0) plan.nb = want_tile <= 2 * ps.blk ? 1 : 2;
    // a target function keeps the coarse sketch beside the fine one: the
    // 32 x 32-per-wave layout (tile 64) leaves room for the extra registers
    if (func.kind != 0 && prec != 0) plan.nb = 1;
    plan.tile = 2 * plan.nb * ps.blk;
    // f64: 2 x 2 waves of 32 x 32 (tile 64), or 4 x 4 such waves (tile 128:
    // twice the flops per byte staged, the same registers per wave)
    // (by default for products of at least 512 x 512, measured faster there)
    if (prec == 0) {
        bool large = true;
        for (int i = 0; i < nprob; ++i) large = large && probs[i].m >= 512 && probs[i].p >= 512;
        plan.tile = func.kind == 0 && (want_tile == 128 || (want_tile == 0 && large)) ? 128 : 64;
    }
    plan.kpad_max = 0;
    for (int l = 0; l < num_levels; ++l) {
        int64_t kc, kpad;
        level_padding(plan, c[l], l > 0 ? c[l - 1] : 0, kc, kpad);
        if (kpad > plan.kpad_max) plan.kpad_max = kpad;
    }
    plan.iid = true;
    plan.whole_tiles = true;
    plan.min_rows = probs[0].m + probs[0].p;
    for (int i = 1; i < nprob; ++i)
        if (probs[i].m + probs[i].p < plan.min_rows) plan.min_rows = probs[i].m + probs[i].p;
    for (int i = 0; i < nprob; ++i) {
        if (probs[i].A.kind >= 2 || probs[i].B.kind >= 2) plan.iid = false;   // column-dependent laws
        if (probs[i].m % plan.tile != 0 || probs[i].p % plan.tile != 0) plan.whole_tiles = false;
    }
    plan.descs.resize(nprob);
    plan.tile_owner.clear();
    plan.exp_host.clear();
    plan.fp8_reparam = false;
    int64_t rows = 0, mp = 0, mb = 0, tiles = 0;
    plan.max_mp = 0;
    plan.max_merge_blocks = 0;
    for (int i = 0; i < nprob; ++i) {
        const MatmulProblem& pr = probs[i];
        ProblemDesc& d = plan.descs[i];
        d.m = pr.m;
        d.n = pr.n;
        d.p = pr.p;
        d.m_pad = round_up(pr.m, plan.tile);
        d.p_pad = round_up(pr.p, plan.tile);
        d.A = pr.A;
        d.B = pr.B;
        d.sid_problem = pr.problem;
        d.tiles_n = ceil_div(pr.p, plan.tile);
        d.tiles = ceil_div(pr.m, plan.tile) * d.tiles_n;
        d.tile_first = tiles;
        d.rows_prefix = rows;
        d.mp_prefix = mp;
        d.merge_blocks = ceil_div(pr.m * pr.p, kMergeThreads);
        d.between_prefix = mb;
        // FP8: per-row (A) and per-column (B) exponents; an i.i.d. law has one
        // for all its rows, folded into its constants by the gather
        const int sa = prec == 3 && pr.A.kind != 2 ? fp8_scale_exponent(fp8_iid_bound(pr.A)) : 0;
        const int sb = prec == 3 && pr.B.kind != 2 ? fp8_scale_exponent(fp8_iid_bound(pr.B)) : 0;
        d.pre_a = (float)ldexp(1.0, sa);
        d.pre_b = (float)ldexp(1.0, sb);
        d.exp_a = d.exp_b = nullptr;     // set to the workspace tables by matmul_upload
        if (prec == 3) {
            plan.exp_host.insert(plan.exp_host.end(), (size_t)d.m_pad, (int8_t)sa);
            plan.exp_host.insert(plan.exp_host.end(), (size_t)d.p_pad, (int8_t)sb);
            if (pr.A.kind == 2 || pr.B.kind == 2) plan.fp8_reparam = true;
        }
        // both i.i.d. laws have mean loc: E[Z_0] = n loc_A loc_B in every entry
        d.mean0 = plan.iid ? (double)pr.n * pr.A.loc * pr.B.loc : 0.0;
        d.out = pr.out;
        d.level_means = pr.level_means;
        for (int64_t t = 0; t < d.tiles; ++t) plan.tile_owner.push_back(i);
        tiles += d.tiles;
        rows += d.m_pad + d.p_pad;
        mp += pr.m * pr.p;
        mb += d.merge_blocks;
        if (pr.m * pr.p > plan.max_mp) plan.max_mp = pr.m * pr.p;
        if (d.merge_blocks > plan.max_merge_blocks) plan.max_merge_blocks = d.merge_blocks;
    }
    plan.laws = law_pair_kind(probs[0].A.kind, probs[0].B.kind);
    for (int i = 1; i < nprob; ++i)
        if (law_pair_kind(probs[i].A.kind, probs[i].B.kind) != plan.laws) plan.laws = kLawsAny;
    // the laws of Sec. 4 have a gather of their own: every product uses them
    // for both operands, or none does; not with FP8 operands
    for (int i = 0; i < nprob; ++i) {
        const bool ea = probs[i].A.kind >= kLawExperimentFirst, eb = probs[i].B.kind >= kLawExperimentFirst;
        if ((ea || eb) && (plan.laws != kLawsExperiment || prec == 3)) return false;
    }
    plan.sum_rows = rows;
    plan.sum_mp = mp;
    plan.sum_merge_blocks = mb;
    plan.total_tiles = tiles;
    // the gathered operands of one pass stay within a budget (768 MiB by
    // default: larger passes mean fewer merges of the level state, measured
    // faster than a buffer sized for the 256 MB Infinity Cache; tunable,
    // MLMC_GATHER_BUDGET overrides); each level fills the buffer with as many
    // realisations as fit
    int64_t budget = (tune && tune->gather_budget > 0) ? tune->gather_budget : kGatherBudgetBytes;
    if (const char* env = getenv("MLMC_GATHER_BUDGET")) {
        const long long v = atoll(env);
        if (v > 0) budget = v;
    }
    const int64_t per_sample = plan.kpad_max * plan.sum_rows * plan.elem;
    if (budget < per_sample) budget = per_sample;
    plan.gather_bytes = budget;
    // about two rounds of resident workgroups: tile 64 runs 4 per CU, tile 128 runs 2
    const int64_t target = (tune && tune->target_blocks > 0) ? tune->target_blocks
                                                             : (plan.tile == 64 ? 2048 : 1024);
    plan.groups_max = ceil_div(target, plan.total_tiles);
    if (plan.groups_max > 65535) plan.groups_max = 65535;
    const int64_t L1 = num_levels;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    plan.off_means = off;      off = align(off + sizeof(double) * L1 * mp);
    plan.off_between = off;    off = align(off + sizeof(double) * L1 * mb);
    plan.off_within = off;     off = align(off + sizeof(double) * L1 * nprob);
    plan.off_tile_acc = off;   off = align(off + sizeof(double) * L1 * tiles);
    plan.off_var = off;        off = align(off + sizeof(double) * L1 * nprob);
    plan.off_norm = off;       off = align(off + sizeof(double));
    plan.state_doubles = (int64_t)(off / sizeof(double));
    plan.off_desc = off;       off = align(off + sizeof(ProblemDesc) * nprob);
    plan.off_tile_owner = off; off = align(off + sizeof(int32_t) * tiles);
    plan.off_cum = off;        off = align(off + (index_weights ? sizeof(uint64_t) * probs[0].n : 0));
    plan.off_exp = off;        off = align(off + (prec == 3 ? (size_t)rows : 0));
    // (FP8 always: the workspace query describes the shapes, not the laws)
    plan.off_bound = off;      off = align(off + (prec == 3 ? sizeof(double) * rows : 0));
    plan.off_gather = off;     off = align(off + (size_t)plan.gather_bytes);
    plan.off_part_mean = off;  off = align(off + sizeof(double) * plan.groups_max * mp);
    plan.off_part_m2 = off;    off = align(off + sizeof(double) * plan.groups_max * tiles);
    plan.total = off;
    return true;
}

double* matmul_level_var_ptr(const MatmulPlan& plan, char* ws)
{
    return reinterpret_cast<double*>(ws + plan.off_var);
}

hipError_t fill_doubles(double* p, int64_t count, double v, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = ceil_div(count, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, count, v);
    return hipGetLastError();
}

hipError_t matmul_upload(const MatmulPlan& plan, char* ws, hipStream_t stream)
{
    std::vector<ProblemDesc> descs(plan.descs);
    if (plan.prec == 3) {
        int8_t* tables = reinterpret_cast<int8_t*>(ws + plan.off_exp);
        for (ProblemDesc& d : descs) {
            d.exp_a = tables + d.rows_prefix;
            d.exp_b = tables + d.rows_prefix + d.m_pad;
        }
        hipError_t e = hipMemcpyAsync(tables, plan.exp_host.data(), plan.exp_host.size(), hipMemcpyHostToDevice,
                                      stream);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMemcpyAsync(ws + plan.off_desc, descs.data(), sizeof(ProblemDesc) * plan.nprob,
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(ws + plan.off_tile_owner, plan.tile_owner.data(), sizeof(int32_t) * plan.total_tiles,
                       hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    // the sources are pageable host memory owned by `plan`: wait until the
    // copies have consumed them
    return hipStreamSynchronize(stream);
}

// Sum of squares of `count` doubles into *out: one workgroup, strided
// per-thread sums then a tree (fixed order).
__global__ __launch_bounds__(kMergeThreads) void sum_squares_kernel(const double* x, int64_t count, double* out)
{
    __shared__ double red[kMergeThreads];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kMergeThreads) s = fma(x[i], x[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int half = kMergeThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

hipError_t matmul_level_norm2(const MatmulPlan& plan, char* ws, int level, hipStream_t stream)
{
    const double* means = reinterpret_cast<const double*>(ws + plan.off_means) + level * plan.sum_mp;
    hipLaunchKernelGGL(sum_squares_kernel, dim3(1), dim3(kMergeThreads), 0, stream, means,
                       plan.descs[0].m * plan.descs[0].p, reinterpret_cast<double*>(ws + plan.off_norm));
    return hipGetLastError();
}

double* matmul_norm_ptr(const MatmulPlan& plan, char* ws)
{
    return reinterpret_cast<double*>(ws + plan.off_norm);
}

// FP8 with reparameterised laws: the bound of every row of A (column of B),
// the maximum over the n columns (rows) j of fma(6, |stdev|, |mean|) in FP64,
// by an atomic maximum on the bit patterns (non-negative doubles order like
// their bits).  Grid: (ceil(count / 256), up to 4096 ranges of j of at least
// kBoundChunk); A's row i of column j sits at j ld + i, B's column q of row j
// at j ld + q, so both walk j.
constexpr int kBoundChunk = 256;

__global__ __launch_bounds__(256) void fp8_bound_kernel(const float* mean, const float* stdev, int64_t ld, int64_t n,
                                                        int64_t count, unsigned long long* bound)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const int64_t chunk = ceil_div(n, (int64_t)gridDim.y);
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    double b = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double v = fma(6.0, fabs((double)stdev[j * ld + i]), fabs((double)mean[j * ld + i]));
        b = v > b ? v : b;
    }
    atomicMax(bound + i, (unsigned long long)__double_as_longlong(b));
}

// The exponents of the rows (columns) of reparameterised operands from their bounds.
__global__ void fp8_exponent_kernel(const double* bound, int64_t count, int8_t* exps)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) exps[i] = (int8_t)fp8_scale_exponent(bound[i]);
}

hipError_t matmul_reset(const MatmulPlan& plan, char* ws, hipStream_t stream)
{
    // means, between, within and var are contiguous at the start of the workspace
    hipError_t e = fill_doubles(reinterpret_cast<double*>(ws), plan.state_doubles, 0.0, stream);
    if (e != hipSuccess || !plan.fp8_reparam) return e;
    // FP8 exponents of reparameterised operands, from the current means and scales
    double* bound = reinterpret_cast<double*>(ws + plan.off_bound);
    int8_t* tables = reinterpret_cast<int8_t*>(ws + plan.off_exp);
    for (const ProblemDesc& d : plan.descs) {
        for (int side = 0; side < 2; ++side) {
            const Law& law = side == 0 ? d.A : d.B;
            if (law.kind != 2) continue;
            const int64_t count = side == 0 ? d.m : d.p;
            const int64_t off = d.rows_prefix + (side == 0 ? 0 : d.m_pad);
            if ((e = fill_doubles(bound + off, count, 0.0, stream)) != hipSuccess) return e;
            int64_t chunks = ceil_div(d.n, (int64_t)kBoundChunk);
            if (chunks > 4096) chunks = 4096;
            hipLaunchKernelGGL(fp8_bound_kernel, dim3((unsigned)ceil_div(count, (int64_t)256), (unsigned)chunks),
                               dim3(256), 0, stream, law.mean, law.stdev, law.ld, d.n, count,
                               reinterpret_cast<unsigned long long*>(bound + off));
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(fp8_exponent_kernel, dim3((unsigned)ceil_div(count, (int64_t)256)), dim3(256), 0,
                               stream, bound + off, count, tables + off);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template <typename P, typename Compute, int WR, int WC, int NBR, int NBC, int WPE>
static hipError_t run_pass(const MatmulPlan& plan, const LevelRange& lr, int64_t k_first, int64_t batch,
                           int64_t done_before, int64_t kc, int64_t kpad, const StreamKeys& keys, char* ws,
                           hipStream_t stream, KernelTimer* timer)
{
    const ProblemDesc* descs = reinterpret_cast<const ProblemDesc*>(ws + plan.off_desc);
    GatherParams g;
    g.descs = descs;
    g.c = (uint32_t)lr.c;
    g.c_prev = (uint32_t)lr.c_prev;
    g.stride = (uint32_t)lr.stride;
    g.level_field = lr.level_field;
    g.kc = kc;
    g.kpad = kpad;
    g.batch = batch;
    g.key0 = keys.key0;
    g.key1 = keys.key1;
    g.k_first = (uint32_t)k_first;
    g.elem = plan.elem;
    g.gbuf = ws + plan.off_gather;
    {
        ScopedTiming t(timer, 1);
        // more position groups per block (lanes over (group, quad) items) when
        // some product has fewer than 1024 rows, while the grid still holds at
        // least 8192 blocks (eight waves per SIMD)
        int oct = 1;
        while (plan.min_rows < 1024 && oct < kGatherMaxOctets &&
               ceil_div(kpad, (int64_t)kGatherPositions * oct * 2) * batch * plan.nprob >= 8192)
            oct *= 2;
        g.octets = oct;
        // with a target function the sketch needs the coarse sum itself: no weight
        g.omega = lr.c_prev > 0 && plan.func.kind == 0 ? 1.0 - (double)lr.c / (double)lr.c_prev : 1.0;
        g.iw = plan.index_weights;
        g.cum = plan.index_weights ? reinterpret_cast<const uint64_t*>(ws + plan.off_cum) : nullptr;
        const dim3 grid((unsigned)ceil_div(kpad, (int64_t)kGatherPositions * oct), (unsigned)batch,
                        (unsigned)plan.nprob);
        if (plan.laws == kLawsExperiment) {
            if constexpr (sizeof(typename P::In) == 1) return hipErrorInvalidValue;   // not with FP8
            else hipLaunchKernelGGL((gather_experiment_kernel<Compute, typename P::In, P::KPACK>), grid,
                                    dim3(kGatherThreads), 0, stream, g);
        } else if (plan.value16) {
            if (plan.laws == kLawsNormal)
                hipLaunchKernelGGL((gather_kernel<Compute, typename P::In, P::KPACK, kLawsNormal, true>), grid,
                                   dim3(kGatherThreads), 0, stream, g);
            else if (plan.laws == kLawsUniform)
                hipLaunchKernelGGL((gather_kernel<Compute, typename P::In, P::KPACK, kLawsUniform, true>), grid,
                                   dim3(kGatherThreads), 0, stream, g);
            else
                hipLaunchKernelGGL((gather_kernel<Compute, typename P::In, P::KPACK, kLawsAny, true>), grid,
                                   dim3(kGatherThreads), 0, stream, g);
        } else if (plan.laws == kLawsNormal)
            hipLaunchKernelGGL((gather_kernel<Compute, typename P::In, P::KPACK, kLawsNormal, false>), grid,
                               dim3(kGatherThreads), 0, stream, g);
        else if (plan.laws == kLawsUniform)
            hipLaunchKernelGGL((gather_kernel<Compute, typename P::In, P::KPACK, kLawsUniform, false>), grid,
                               dim3(kGatherThreads), 0, stream, g);
        else
            hipLaunchKernelGGL((gather_kernel<Compute, typename P::In, P::KPACK, kLawsAny, false>), grid,
                               dim3(kGatherThreads), 0, stream, g);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;

    const int64_t groups = batch < plan.groups_max ? batch : plan.groups_max;
    SketchParams s;
    s.descs = descs;
    s.tile_owner = reinterpret_cast<const int32_t*>(ws + plan.off_tile_owner);
    s.total_tiles = plan.total_tiles;
    s.groups = groups;
    s.kc = kc;
    s.kpad = kpad;
    s.batch = batch;
    s.elem = plan.elem;
    s.c = (uint32_t)lr.c;
    s.c_prev = (uint32_t)lr.c_prev;
    s.func = plan.func;
    s.gbuf = g.gbuf;
    s.part_mean = ws + plan.off_part_mean;
    s.part_m2 = reinterpret_cast<double*>(ws + plan.off_part_m2);
    s.sum_mp = plan.sum_mp;
    s.fuse = groups == 1;
    s.done_before = (double)done_before;
    s.level_mean = reinterpret_cast<double*>(ws + plan.off_means) + lr.level * plan.sum_mp;
    s.tile_acc = reinterpret_cast<double*>(ws + plan.off_tile_acc) + lr.level * plan.total_tiles;
    int64_t blocks = plan.total_tiles * groups;
    if (blocks > kSketchMaxBlocks) blocks = kSketchMaxBlocks;
    blocks = ceil_div(blocks, kXcds) * kXcds;
    {
        ScopedTiming t(timer, 0);
        // shifted sums for i.i.d. laws (the mask-free form when every product
        // fills whole tiles), except in the 4 x 2-wave BF16/FP32 kernels,
        // where their extra live values spill (measured slower than Welford);
        // the masked form only where a lane holds at most 32 entries
        constexpr bool kShiftedFits = !(WR == 4 && WC == 2 && sizeof(typename P::In) >= 2);
        constexpr bool kMaskedFits = kShiftedFits && NBR * NBC * P::REGS <= 32;
        constexpr bool kDualForm = sizeof(typename P::In) <= 2;   // BF16, FP8: FP32 totals suffice
        const dim3 grid((unsigned)blocks), block(kWave * WR * WC);
        // the layouts a target function uses (2 x 2 waves; never the f64 4 x 4)
        constexpr bool kFuncForm = NBR * NBC * P::REGS <= 16 && WR * WC == 4;
        if (plan.func.kind != 0) {
            // the copied accumulators need more than 128 registers: two waves per SIMD
            if constexpr (kFuncForm) {
                // level 0 (no coarse sketch): the statistics fit the full occupancy
                if (lr.c_prev == 0 && plan.func.kind == 1)
                    hipLaunchKernelGGL((sketch_kernel<P, WR, WC, NBR, NBC, WPE, 6>), grid, block, 0, stream, s);
                else if (lr.c_prev == 0)
                    hipLaunchKernelGGL((sketch_kernel<P, WR, WC, NBR, NBC, WPE, 7>), grid, block, 0, stream, s);
                else if (plan.func.kind == 1)
                    hipLaunchKernelGGL((sketch_kernel<P, WR, WC, NBR, NBC, (WPE > 2 ? 2 : WPE), 4>), grid, block,
                                       0, stream, s);
                else
                    hipLaunchKernelGGL((sketch_kernel<P, WR, WC, NBR, NBC, (WPE > 2 ? 2 : WPE), 5>), grid, block,
                                       0, stream, s);
            } else
                return hipErrorInvalidConfiguration;   // matmul_plan picks tile 64 for a target function
        } else if (plan.iid && plan.whole_tiles && kDualForm && lr.c <= kDualMaxDraws)
            hipLaunchKernelGGL((sketch_kernel<P, WR, WC, NBR, NBC, WPE, kDualForm ? 3 : 0>), grid, block, 0,
                               stream, s);
        else if (plan.iid && kShiftedFits && plan.whole_tiles)
            hipLaunchKernelGGL((sketch_kernel<P, WR, WC, NBR, NBC, WPE, kShiftedFits ? 2 : 0>), grid, block, 0,
                               stream, s);
        else if (plan.iid && kMaskedFits)
            hipLaunchKernelGGL((sketch_kernel<P, WR, WC, NBR, NBC, WPE, kMaskedFits ? 1 : 0>), grid, block, 0,
                               stream, s);
        else
            hipLaunchKernelGGL((sketch_kernel<P, WR, WC, NBR, NBC, WPE, 0>), grid, block, 0, stream, s);
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;

    if (s.fuse) return hipSuccess;           // merged by the sketch epilogue
    MergeParams mg;
    mg.descs = descs;
    mg.level = lr.level;
    mg.batch = batch;
    mg.groups = groups;
    mg.total_tiles = plan.total_tiles;
    mg.sum_mp = plan.sum_mp;
    mg.sum_merge_blocks = plan.sum_merge_blocks;
    mg.nprob = plan.nprob;
    mg.done_before = (double)done_before;
    mg.part_mean = s.part_mean;
    mg.part_m2 = s.part_m2;
    mg.means = reinterpret_cast<double*>(ws + plan.off_means);
    mg.between = reinterpret_cast<double*>(ws + plan.off_between);
    mg.within = reinterpret_cast<double*>(ws + plan.off_within);
    {
        ScopedTiming t(timer, 2);
        hipLaunchKernelGGL((merge_kernel<typename P::Acc>), dim3((unsigned)plan.max_merge_blocks,
                           (unsigned)plan.nprob), dim3(kMergeThreads), 0, stream, mg);
    }
    return hipGetLastError();
}

template <typename P, typename Compute>
static hipError_t run_pass_nb(const MatmulPlan& plan, const LevelRange& lr, int64_t k_first, int64_t batch,
                              int64_t done_before, int64_t kc, int64_t kpad, const StreamKeys& keys, char* ws,
                              hipStream_t stream, KernelTimer* timer)
{
    // tile 64: 2 x 2 waves of 32 x 32.  Tile 128: 2 x 2 waves of 64 x 64
    // (two waves per SIMD; each fragment read from LDS feeds two MFMAs)
    if (plan.tile == 64)
        return run_pass<P, Compute, 2, 2, 1, 1, 4>(plan, lr, k_first, batch, done_before, kc, kpad, keys, ws, stream,
                                                   timer);
    return run_pass<P, Compute, 2, 2, 2, 2, 2>(plan, lr, k_first, batch, done_before, kc, kpad, keys, ws, stream,
                                               timer);
}

hipError_t matmul_level_run(const MatmulPlan& plan, const LevelRange& lr, int64_t done_before, const StreamKeys& keys,
                            char* ws, hipStream_t stream, KernelTimer* timer)
{
    int64_t kc, kpad;
    level_padding(plan, lr.c, lr.c_prev, kc, kpad);
    const int64_t per_sample = kpad * plan.sum_rows * plan.elem;
    int64_t level_batch = plan.gather_bytes / per_sample;
    if (level_batch < 1) level_batch = 1;
    if (level_batch > 65535) level_batch = 65535;
    // the sketch counts a group's padded positions in 32 bits
    if (level_batch > INT32_MAX / kpad) level_batch = INT32_MAX / kpad;
    for (int64_t b = 0; b < lr.count; b += level_batch) {
        const int64_t batch = (lr.count - b) < level_batch ? (lr.count - b) : level_batch;
        hipError_t err;
        const int64_t k_first = lr.k_begin + b, before = done_before + b;
        if (plan.prec == 0 && plan.tile == 128)
            err = run_pass<PolicyF64, double, 4, 4, 2, 2, 4>(plan, lr, k_first, batch, before, kc, kpad, keys, ws,
                                                             stream, timer);
        else if (plan.prec == 0)
            err = run_pass<PolicyF64, double, 2, 2, 2, 2, 2>(plan, lr, k_first, batch, before, kc, kpad, keys, ws,
                                                             stream, timer);
        else if (plan.prec == 1)
            err = run_pass_nb<PolicyF32, float>(plan, lr, k_first, batch, before, kc, kpad, keys, ws, stream, timer);
        else if (plan.prec == 2)
            err = run_pass_nb<PolicyBF16, float>(plan, lr, k_first, batch, before, kc, kpad, keys, ws, stream, timer);
        else
            err = run_pass_nb<PolicyFP8, float>(plan, lr, k_first, batch, before, kc, kpad, keys, ws, stream, timer);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t matmul_finalize(const MatmulPlan& plan, const int64_t* counts, char* ws, bool write_outputs,
                           hipStream_t stream)
{
    FinalizeParams f;
    f.descs = reinterpret_cast<const ProblemDesc*>(ws + plan.off_desc);
    f.num_levels = plan.num_levels;
    f.sum_mp = plan.sum_mp;
    f.sum_merge_blocks = plan.sum_merge_blocks;
    f.nprob = plan.nprob;
    for (int l = 0; l < 32; ++l) f.counts[l] = l < plan.num_levels ? (double)counts[l] : 0.0;
    f.means = reinterpret_cast<const double*>(ws + plan.off_means);
    f.between = reinterpret_cast<const double*>(ws + plan.off_between);
    f.within = reinterpret_cast<const double*>(ws + plan.off_within);
    f.tile_acc = reinterpret_cast<const double*>(ws + plan.off_tile_acc);
    f.total_tiles = plan.total_tiles;
    f.var = reinterpret_cast<double*>(ws + plan.off_var);
    hipLaunchKernelGGL(level_var_kernel, dim3((unsigned)plan.num_levels, (unsigned)plan.nprob), dim3(kMergeThreads),
                       0, stream, f);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || !write_outputs) return err;
    hipLaunchKernelGGL(telescope_kernel, dim3((unsigned)ceil_div(plan.max_mp, kMergeThreads), (unsigned)plan.nprob),
                       dim3(kMergeThreads), 0, stream, f);
    return hipGetLastError();
}

}  // namespace mlmc
