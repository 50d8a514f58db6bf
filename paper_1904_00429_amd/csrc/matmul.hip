// Matrix-product MLMC pipeline (Sec. 3; Alg. 1 per level, f = identity).
//
// Per pass over a batch of S realisations of one level l:
//   1. gather:  draw the c_l indices of every realisation (index stream) and
//      generate only the sampled columns a_t = A^(k)[:, r_t] and rows
//      b_t = B^(k)[r_t, :] (value stream, keyed by the column j = r_t), in the
//      operand precision, into a gathered buffer laid out for the MFMA
//      fragments.  Draws t < c_{l-1} (the coarse segment) and the remaining
//      draws (the fine segment) are each zero-padded to the contraction step.
//   2. sketch:  per output tile and group of realisations, the K loop runs
//      over the coarse segment, scales the accumulator by 1 - c_l / c_{l-1},
//      then continues over the fine segment: the result times n / c_l is
//      D_k = Z_l^(k) - Z_{l-1}^(k) (the coupled fine-minus-coarse sample of
//      Alg. 1) without ever forming either sketch.  Each entry's Welford
//      state over the group's realisations is kept in registers.
//   3. merge:   per entry, a fixed-order Chan merge of the group means into
//      the level's running mean (FP64); the between-group part of the sum of
//      squared deviations is reduced per block, the within-group parts are
//      summed by one thread.  V_l = (within + between) / (N_l - 1).
// After the last level, `finalize` forms V_l and the telescoping sum
// Y = sum_l Ybar_l (eq. (10)).
#include <hip/hip_bf16.h>
#include <stdlib.h>

#include "internal.hpp"

namespace mlmc {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kSketchThreads = 256;
constexpr int kMergeThreads = 256;
constexpr int kGatherThreads = 64;
constexpr int kGatherPositions = 8;
constexpr int64_t kGatherBudgetBytes = 192ll << 20;
constexpr int64_t kTargetSketchBlocks = 2048;

// ---------------------------------------------------------------------------
// Contraction policies: operand type, MFMA shape, wave tile, fragment layout.
// A workgroup is 2 x 2 waves, so its tile is 2 WM x 2 WN.
// ---------------------------------------------------------------------------
struct PolicyF64 {  // v_mfma_f64_16x16x4_f64: wave tile 32 x 32 = 2 x 2 blocks
    using In = double;
    using Acc = double;
    static constexpr int KSTEP = 4, KPACK = 1, BLK = 16, NB = 2, WM = 32, WN = 32;
    static constexpr int REGS = 4;  // accumulator elements per lane per block
    using AccVec = f64x4;
    // f64 results: lane l, register r holds row l / 16 + 4 r, column l % 16
    static __device__ __forceinline__ int row_of(int lane, int r) { return lane / 16 + 4 * r; }
    static __device__ __forceinline__ int col_of(int lane) { return lane % 16; }
};

struct PolicyF32 {  // v_mfma_f32_32x32x2_f32: wave tile 64 x 64 = 2 x 2 blocks
    using In = float;
    using Acc = float;
    static constexpr int KSTEP = 2, KPACK = 1, BLK = 32, NB = 2, WM = 64, WN = 64;
    static constexpr int REGS = 16;
    using AccVec = f32x16;
    static __device__ __forceinline__ int row_of(int lane, int r) { return 8 * (r / 4) + 4 * (lane / 32) + (r % 4); }
    static __device__ __forceinline__ int col_of(int lane) { return lane % 32; }
};

struct PolicyBF16 {  // v_mfma_f32_32x32x16_bf16: wave tile 64 x 64 = 2 x 2 blocks
    using In = __bf16;
    using Acc = float;
    static constexpr int KSTEP = 16, KPACK = 8, BLK = 32, NB = 2, WM = 64, WN = 64;
    static constexpr int REGS = 16;
    using AccVec = f32x16;
    static __device__ __forceinline__ int row_of(int lane, int r) { return 8 * (r / 4) + 4 * (lane / 32) + (r % 4); }
    static __device__ __forceinline__ int col_of(int lane) { return lane % 32; }
};

template <typename P> struct Frag;
template <> struct Frag<PolicyF64> { using T = double; };
template <> struct Frag<PolicyF32> { using T = float; };
template <> struct Frag<PolicyBF16> { using T = bf16x8; };

// Fragment of the gathered operand G (layout [kpad / KPACK][rows][KPACK]) for
// the MFMA block whose first row is `row0`, at padded draw `kk`.
__device__ __forceinline__ double load_frag(const PolicyF64&, const double* G, int64_t rows,
                                            int64_t row0, int64_t kk, int lane)
{
    const int64_t row = row0 + (lane % 16);
    const int64_t t = kk + lane / 16;
    return row < rows ? G[t * rows + row] : 0.0;
}

__device__ __forceinline__ float load_frag(const PolicyF32&, const float* G, int64_t rows,
                                           int64_t row0, int64_t kk, int lane)
{
    const int64_t row = row0 + (lane % 32);
    const int64_t t = kk + lane / 32;
    return row < rows ? G[t * rows + row] : 0.0f;
}

__device__ __forceinline__ bf16x8 load_frag(const PolicyBF16&, const __bf16* G, int64_t rows,
                                            int64_t row0, int64_t kk, int lane)
{
    const int64_t row = row0 + (lane % 32);
    const int64_t kb = kk / 8 + lane / 32;
    bf16x8 v;
    if (row < rows) {
        v = *reinterpret_cast<const bf16x8*>(G + (kb * rows + row) * 8);
    } else {
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.0f;
    }
    return v;
}

__device__ __forceinline__ f64x4 mma(const PolicyF64&, double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mma(const PolicyF32&, float a, float b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mma(const PolicyBF16&, bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Gather: only the sampled columns of the realisation are generated.
// ---------------------------------------------------------------------------
struct GatherParams {
    int64_t m, p;
    uint32_t n;
    uint32_t c, c_prev;
    int64_t kc, kpad;        // padded coarse length, padded total length
    uint32_t key0, key1, sid_index, sid_value;
    uint32_t k_first;        // realisation of batch slot 0
    Law A, B;
    void* GA;                // batch x [kpad / KPACK][m][KPACK]
    void* GB;                // batch x [kpad / KPACK][p][KPACK]
};

// Draw number t of padded position `pos`, or -1 for padding.
__device__ __forceinline__ int64_t draw_of_position(int64_t pos, int64_t kc, uint32_t c, uint32_t c_prev)
{
    if (pos < kc) return pos < (int64_t)c_prev ? pos : -1;
    const int64_t t = (int64_t)c_prev + (pos - kc);
    return t < (int64_t)c ? t : -1;
}

template <typename T> __device__ __forceinline__ T to_store(float v);
template <> __device__ __forceinline__ float to_store<float>(float v) { return v; }
template <> __device__ __forceinline__ __bf16 to_store<__bf16>(float v) { return (__bf16)v; }

template <typename Compute, typename Store, int KPACK>
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(GatherParams prm)
{
    __shared__ uint32_t cols[kGatherPositions];
    __shared__ int valid[kGatherPositions];
    const int64_t pos0 = (int64_t)blockIdx.x * kGatherPositions;
    const int64_t slot = blockIdx.y;
    const uint32_t k = prm.k_first + (uint32_t)slot;
    if (threadIdx.x < kGatherPositions) {
        const int64_t pos = pos0 + threadIdx.x;
        const int64_t t = pos < prm.kpad ? draw_of_position(pos, prm.kc, prm.c, prm.c_prev) : -1;
        valid[threadIdx.x] = t >= 0;
        cols[threadIdx.x] = t >= 0 ? draw_index((uint32_t)t, k, prm.sid_index, prm.key0, prm.key1, prm.n) : 0u;
    }
    __syncthreads();
    const int64_t rows = prm.m + prm.p;
    const int64_t quads = ceil_div(rows, 4);
    const bool normal = prm.A.kind != 1 || prm.B.kind != 1;
    const int npos = (int)((prm.kpad - pos0) < kGatherPositions ? (prm.kpad - pos0) : kGatherPositions);
    Store* GA = static_cast<Store*>(prm.GA) + slot * prm.kpad * prm.m;
    Store* GB = static_cast<Store*>(prm.GB) + slot * prm.kpad * prm.p;
    for (int64_t q = threadIdx.x; q < quads; q += kGatherThreads) {
        Store vals[kGatherPositions][4];
        for (int ip = 0; ip < kGatherPositions; ++ip) {
            if (ip >= npos || !valid[ip]) {
                for (int r = 0; r < 4; ++r) vals[ip][r] = (Store)0.0f;
                continue;
            }
            const uint32_t j = cols[ip];
            const Words4 w = philox4x32_10((uint32_t)q, k, j, prm.sid_value, prm.key0, prm.key1);
            Compute u[4], z[4];
            quad_values<Compute>(w, normal, u[0], u[1], u[2], u[3], z[0], z[1], z[2], z[3]);
            for (int r = 0; r < 4; ++r) {
                const int64_t e = 4 * q + r;
                Compute v = (Compute)0;
                if (e < prm.m) v = law_value<Compute>(prm.A, z[r], u[r], (int64_t)j * prm.A.ld + e);
                else if (e < rows) v = law_value<Compute>(prm.B, z[r], u[r], (int64_t)j * prm.B.ld + (e - prm.m));
                vals[ip][r] = (Store)v;
            }
        }
        for (int r = 0; r < 4; ++r) {
            const int64_t e = 4 * q + r;
            if (e >= rows) break;
            Store* G = e < prm.m ? GA : GB;
            const int64_t R = e < prm.m ? prm.m : prm.p;
            const int64_t row = e < prm.m ? e : e - prm.m;
            if constexpr (KPACK == 1) {
                for (int ip = 0; ip < npos; ++ip) G[(pos0 + ip) * R + row] = vals[ip][r];
            } else {
                // positions pos0 .. pos0+7 are one packed group of 8 draws
                Store pack[KPACK];
                for (int ip = 0; ip < KPACK; ++ip) pack[ip] = vals[ip][r];
                const int64_t kb = pos0 / KPACK;
                typedef Store vec_t __attribute__((ext_vector_type(KPACK)));
                vec_t vv;
                for (int ip = 0; ip < KPACK; ++ip) vv[ip] = pack[ip];
                *reinterpret_cast<vec_t*>(G + (kb * R + row) * KPACK) = vv;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Sketch + coupling + per-entry Welford over a group of realisations.
// ---------------------------------------------------------------------------
struct SketchParams {
    int64_t m, p;
    int64_t kc, kpad;
    int64_t batch;           // realisations in this pass
    int64_t tiles_n;
    double scale;            // n / c_l
    double omega;            // 1 - c_l / c_{l-1} (unused at level 0: kc == 0)
    const void* GA;
    const void* GB;
    double* part_mean;       // groups x m x p
    double* part_m2;         // groups x tiles
};

template <typename P>
__global__ __launch_bounds__(kSketchThreads) void sketch_kernel(SketchParams prm)
{
    using In = typename P::In;
    using Acc = typename P::Acc;
    using FragT = typename Frag<P>::T;
    constexpr int NE = P::NB * P::NB * P::REGS;  // entries per lane
    __shared__ double red[kSketchThreads / kWave];

    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int64_t tile = blockIdx.x;
    const int64_t group = blockIdx.y;
    const int64_t groups = gridDim.y;
    const int64_t tile_m = tile / prm.tiles_n, tile_n = tile % prm.tiles_n;
    const int64_t row0 = tile_m * (2 * P::WM) + (wave / 2) * P::WM;
    const int64_t col0 = tile_n * (2 * P::WN) + (wave % 2) * P::WN;
    const int64_t s_begin = group * prm.batch / groups;
    const int64_t s_end = (group + 1) * prm.batch / groups;
    const P pol{};

    Acc mean[NE], m2[NE];
    for (int e = 0; e < NE; ++e) { mean[e] = (Acc)0; m2[e] = (Acc)0; }
    Acc count = (Acc)0;
    const Acc scale = (Acc)prm.scale, omega = (Acc)prm.omega;

    for (int64_t s = s_begin; s < s_end; ++s) {
        const In* GA = static_cast<const In*>(prm.GA) + s * prm.kpad * prm.m;
        const In* GB = static_cast<const In*>(prm.GB) + s * prm.kpad * prm.p;
        typename P::AccVec acc[P::NB][P::NB];
        for (int bi = 0; bi < P::NB; ++bi)
            for (int bj = 0; bj < P::NB; ++bj)
                for (int r = 0; r < P::REGS; ++r) acc[bi][bj][r] = (Acc)0;
        for (int64_t kk = 0; kk < prm.kpad; kk += P::KSTEP) {
            if (kk == prm.kc && kk > 0) {
                // end of the coarse segment: fold in the coarse sketch weight
                for (int bi = 0; bi < P::NB; ++bi)
                    for (int bj = 0; bj < P::NB; ++bj)
                        for (int r = 0; r < P::REGS; ++r) acc[bi][bj][r] *= omega;
            }
            FragT a[P::NB], b[P::NB];
            for (int bi = 0; bi < P::NB; ++bi) a[bi] = load_frag(pol, GA, prm.m, row0 + bi * P::BLK, kk, lane);
            for (int bj = 0; bj < P::NB; ++bj) b[bj] = load_frag(pol, GB, prm.p, col0 + bj * P::BLK, kk, lane);
            for (int bi = 0; bi < P::NB; ++bi)
                for (int bj = 0; bj < P::NB; ++bj) acc[bi][bj] = mma(pol, a[bi], b[bj], acc[bi][bj]);
        }
        if (prm.kc == prm.kpad && prm.kc > 0) {
            for (int bi = 0; bi < P::NB; ++bi)
                for (int bj = 0; bj < P::NB; ++bj)
                    for (int r = 0; r < P::REGS; ++r) acc[bi][bj][r] *= omega;
        }
        count += (Acc)1;
        const Acc inv = (Acc)1 / count;
        int e = 0;
        for (int bi = 0; bi < P::NB; ++bi)
            for (int bj = 0; bj < P::NB; ++bj)
                for (int r = 0; r < P::REGS; ++r, ++e) {
                    const Acc d = scale * acc[bi][bj][r];
                    const Acc delta = d - mean[e];
                    mean[e] += delta * inv;
                    m2[e] += delta * (d - mean[e]);
                }
    }

    // group mean of every in-range entry, and the group's within sum of squares
    double m2_sum = 0.0;
    int e = 0;
    for (int bi = 0; bi < P::NB; ++bi)
        for (int bj = 0; bj < P::NB; ++bj)
            for (int r = 0; r < P::REGS; ++r, ++e) {
                const int64_t i = row0 + bi * P::BLK + P::row_of(lane, r);
                const int64_t j = col0 + bj * P::BLK + P::col_of(lane);
                if (i < prm.m && j < prm.p) {
                    prm.part_mean[(group * prm.m + i) * prm.p + j] = (double)mean[e];
                    m2_sum += (double)m2[e];
                }
            }
    for (int off = kWave / 2; off > 0; off >>= 1) m2_sum += __shfl_xor(m2_sum, off, kWave);
    if (lane == 0) red[wave] = m2_sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kSketchThreads / kWave; ++w) tot += red[w];
        prm.part_m2[group * gridDim.x + tile] = tot;
    }
}

// ---------------------------------------------------------------------------
// Merge of a pass's groups into the level state; finalize.
// ---------------------------------------------------------------------------
struct MergeParams {
    int64_t mp;
    int64_t batch, groups, tiles;
    double done_before;      // realisations already in the level state
    const double* part_mean;
    const double* part_m2;
    double* mean;            // level state: m x p
    double* between;         // level state: merge_blocks
    double* within;          // level state: 1
};

__global__ __launch_bounds__(kMergeThreads) void merge_kernel(MergeParams prm)
{
    __shared__ double red[kMergeThreads];
    const int64_t e = (int64_t)blockIdx.x * kMergeThreads + threadIdx.x;
    double between = 0.0;
    if (e < prm.mp) {
        double mu = prm.mean[e];
        double na = prm.done_before;
        for (int64_t g = 0; g < prm.groups; ++g) {
            const double nb = (double)((g + 1) * prm.batch / prm.groups - g * prm.batch / prm.groups);
            const double n = na + nb;
            const double delta = prm.part_mean[g * prm.mp + e] - mu;
            mu += delta * (nb / n);
            between += delta * delta * (na * nb / n);
            na = n;
        }
        prm.mean[e] = mu;
    }
    red[threadIdx.x] = between;
    __syncthreads();
    for (int half = kMergeThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        prm.between[blockIdx.x] += red[0];
        if (blockIdx.x == 0) {
            double w = 0.0;
            for (int64_t i = 0; i < prm.groups * prm.tiles; ++i) w += prm.part_m2[i];
            *prm.within += w;
        }
    }
}

struct FinalizeParams {
    int num_levels;
    int64_t merge_blocks;
    double counts[32];
    const double* between;   // levels x merge_blocks
    const double* within;    // levels
    double* var;             // levels
};

__global__ __launch_bounds__(kMergeThreads) void level_var_kernel(FinalizeParams prm)
{
    __shared__ double red[kMergeThreads];
    const int l = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < prm.merge_blocks; b += kMergeThreads) s += prm.between[l * prm.merge_blocks + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int half = kMergeThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = prm.counts[l];
        prm.var[l] = n > 1.0 ? (red[0] + prm.within[l]) / (n - 1.0) : 0.0;
    }
}

__global__ __launch_bounds__(kMergeThreads) void telescope_kernel(const double* means, int num_levels,
                                                                  int64_t mp, double* out,
                                                                  double* level_means)
{
    const int64_t e = (int64_t)blockIdx.x * kMergeThreads + threadIdx.x;
    if (e >= mp) return;
    double y = 0.0;
    for (int l = 0; l < num_levels; ++l) {
        const double v = means[l * mp + e];
        y += v;
        if (level_means) level_means[l * mp + e] = v;
    }
    out[e] = y;
}

__global__ void fill_kernel(double* p, int64_t count, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Host side: plan, passes, finalize.
// ---------------------------------------------------------------------------
static void policy_shape(int prec, int& kstep, int& kpack, int& tm, int& tn, int& elem)
{
    if (prec == 0) { kstep = PolicyF64::KSTEP; kpack = 1; tm = 2 * PolicyF64::WM; tn = 2 * PolicyF64::WN; elem = 8; }
    else if (prec == 1) { kstep = PolicyF32::KSTEP; kpack = 1; tm = 2 * PolicyF32::WM; tn = 2 * PolicyF32::WN; elem = 4; }
    else { kstep = PolicyBF16::KSTEP; kpack = PolicyBF16::KPACK; tm = 2 * PolicyBF16::WM; tn = 2 * PolicyBF16::WN; elem = 2; }
}

static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

static void level_padding(const MatmulPlan& plan, int64_t c, int64_t c_prev, int64_t& kc, int64_t& kpad)
{
    kc = round_up(c_prev, plan.kstep);
    kpad = kc + round_up(c - c_prev, plan.kstep);
    // the packed layout groups 8 positions; the gather kernel writes whole groups
    kpad = round_up(kpad, plan.kpack);
}

bool matmul_plan(int64_t m, int64_t n, int64_t p, int prec, int num_levels, const int64_t* c,
                 MatmulPlan& plan)
{
    plan = MatmulPlan();
    plan.m = m; plan.n = n; plan.p = p; plan.prec = prec; plan.num_levels = num_levels;
    for (int l = 0; l < num_levels; ++l) plan.c[l] = c[l];
    int elem = 8;
    policy_shape(prec, plan.kstep, plan.kpack, plan.tile_m, plan.tile_n, elem);
    if (plan.kpack > 1 && plan.kstep % plan.kpack != 0) return false;
    plan.tiles_m = ceil_div(m, plan.tile_m);
    plan.tiles_n = ceil_div(p, plan.tile_n);
    plan.kpad_max = 0;
    for (int l = 0; l < num_levels; ++l) {
        int64_t kc, kpad;
        level_padding(plan, c[l], l > 0 ? c[l - 1] : 0, kc, kpad);
        if (kpad > plan.kpad_max) plan.kpad_max = kpad;
    }
    const int64_t per_sample = plan.kpad_max * (m + p) * elem;
    // the gathered operands of one pass stay within a budget sized for the
    // 256 MB Infinity Cache; MLMC_GATHER_BUDGET (bytes) overrides it.  Each
    // level fills the buffer with as many realisations as fit.
    int64_t budget = kGatherBudgetBytes;
    if (const char* env = getenv("MLMC_GATHER_BUDGET")) {
        const long long v = atoll(env);
        if (v > 0) budget = v;
    }
    if (budget < per_sample) budget = per_sample;
    plan.elem = elem;
    plan.gather_bytes = budget;
    plan.batch = budget / per_sample;
    if (plan.batch > 65535) plan.batch = 65535;
    const int64_t tiles = plan.tiles_m * plan.tiles_n;
    plan.groups_max = ceil_div(kTargetSketchBlocks, tiles);
    if (plan.groups_max > 65535) plan.groups_max = 65535;
    plan.merge_blocks = ceil_div(m * p, kMergeThreads);
    const int64_t L1 = num_levels;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    plan.off_means = off;    off = align(off + sizeof(double) * L1 * m * p);
    plan.off_between = off;  off = align(off + sizeof(double) * L1 * plan.merge_blocks);
    plan.off_within = off;   off = align(off + sizeof(double) * L1);
    plan.off_var = off;      off = align(off + sizeof(double) * L1);
    // one buffer: the A part of a pass first, its B part right after it
    plan.off_gather_a = off; off = align(off + (size_t)plan.gather_bytes + 256);
    plan.off_gather_b = plan.off_gather_a;
    plan.off_part_mean = off; off = align(off + sizeof(double) * plan.groups_max * m * p);
    plan.off_part_m2 = off;  off = align(off + sizeof(double) * plan.groups_max * tiles);
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

hipError_t matmul_reset(const MatmulPlan& plan, char* ws, hipStream_t stream)
{
    // means, between, within and var are contiguous at the start of the workspace
    const int64_t doubles = (int64_t)(plan.off_gather_a / sizeof(double));
    return fill_doubles(reinterpret_cast<double*>(ws), doubles, 0.0, stream);
}

template <typename P, typename Compute>
static hipError_t run_pass(const MatmulPlan& plan, const LevelRange& lr, int64_t k_first,
                           int64_t batch, int64_t done_before, const Law& A, const Law& B,
                           const StreamKeys& keys, char* ws, hipStream_t stream, KernelTimer* timer)
{
    int64_t kc, kpad;
    level_padding(plan, lr.c, lr.c_prev, kc, kpad);
    GatherParams g;
    g.m = plan.m; g.p = plan.p; g.n = (uint32_t)plan.n;
    g.c = (uint32_t)lr.c; g.c_prev = (uint32_t)lr.c_prev;
    g.kc = kc; g.kpad = kpad;
    g.key0 = keys.key0; g.key1 = keys.key1;
    g.sid_index = stream_id(kTagIndex, lr.level_field, keys.problem);
    g.sid_value = stream_id(kTagValue, lr.level_field, keys.problem);
    g.k_first = (uint32_t)k_first;
    g.A = A; g.B = B;
    g.GA = ws + plan.off_gather_a;
    const size_t a_bytes = ((size_t)batch * kpad * plan.m * plan.elem + 255) & ~(size_t)255;
    g.GB = ws + plan.off_gather_a + a_bytes;
    const dim3 ggrid((unsigned)ceil_div(kpad, kGatherPositions), (unsigned)batch);
    {
        ScopedTiming t(timer, 1);
        hipLaunchKernelGGL((gather_kernel<Compute, typename P::In, P::KPACK>), ggrid, dim3(kGatherThreads), 0,
                           stream, g);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;

    const int64_t groups = batch < plan.groups_max ? batch : plan.groups_max;
    const int64_t tiles = plan.tiles_m * plan.tiles_n;
    SketchParams s;
    s.m = plan.m; s.p = plan.p; s.kc = kc; s.kpad = kpad; s.batch = batch;
    s.tiles_n = plan.tiles_n;
    s.scale = (double)plan.n / (double)lr.c;
    s.omega = lr.c_prev > 0 ? 1.0 - (double)lr.c / (double)lr.c_prev : 1.0;
    s.GA = g.GA; s.GB = g.GB;
    s.part_mean = reinterpret_cast<double*>(ws + plan.off_part_mean);
    s.part_m2 = reinterpret_cast<double*>(ws + plan.off_part_m2);
    {
        ScopedTiming t(timer, 0);
        hipLaunchKernelGGL(sketch_kernel<P>, dim3((unsigned)tiles, (unsigned)groups), dim3(kSketchThreads), 0,
                           stream, s);
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;

    const int64_t mp = plan.m * plan.p;
    MergeParams mg;
    mg.mp = mp; mg.batch = batch; mg.groups = groups; mg.tiles = tiles;
    mg.done_before = (double)done_before;
    mg.part_mean = s.part_mean; mg.part_m2 = s.part_m2;
    mg.mean = reinterpret_cast<double*>(ws + plan.off_means) + (int64_t)lr.level * mp;
    mg.between = reinterpret_cast<double*>(ws + plan.off_between) + (int64_t)lr.level * plan.merge_blocks;
    mg.within = reinterpret_cast<double*>(ws + plan.off_within) + lr.level;
    {
        ScopedTiming t(timer, 2);
        hipLaunchKernelGGL(merge_kernel, dim3((unsigned)plan.merge_blocks), dim3(kMergeThreads), 0, stream, mg);
    }
    return hipGetLastError();
}

hipError_t matmul_level_run(const MatmulPlan& plan, const LevelRange& lr, int64_t done_before,
                            const Law& A, const Law& B, const StreamKeys& keys, char* ws,
                            hipStream_t stream, KernelTimer* timer)
{
    int64_t kc, kpad;
    level_padding(plan, lr.c, lr.c_prev, kc, kpad);
    int64_t level_batch = plan.gather_bytes / (kpad * (plan.m + plan.p) * plan.elem + 512);
    if (level_batch < 1) level_batch = 1;
    if (level_batch > 65535) level_batch = 65535;
    for (int64_t b = 0; b < lr.count; b += level_batch) {
        const int64_t batch = (lr.count - b) < level_batch ? (lr.count - b) : level_batch;
        hipError_t err;
        if (plan.prec == 0)
            err = run_pass<PolicyF64, double>(plan, lr, lr.k_begin + b, batch, done_before + b, A, B, keys, ws, stream, timer);
        else if (plan.prec == 1)
            err = run_pass<PolicyF32, float>(plan, lr, lr.k_begin + b, batch, done_before + b, A, B, keys, ws, stream, timer);
        else
            err = run_pass<PolicyBF16, float>(plan, lr, lr.k_begin + b, batch, done_before + b, A, B, keys, ws, stream, timer);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t matmul_finalize(const MatmulPlan& plan, const int64_t* counts, char* ws, double* out,
                           double* level_means, hipStream_t stream)
{
    FinalizeParams f;
    f.num_levels = plan.num_levels;
    f.merge_blocks = plan.merge_blocks;
    for (int l = 0; l < 32; ++l) f.counts[l] = l < plan.num_levels ? (double)counts[l] : 0.0;
    f.between = reinterpret_cast<const double*>(ws + plan.off_between);
    f.within = reinterpret_cast<const double*>(ws + plan.off_within);
    f.var = reinterpret_cast<double*>(ws + plan.off_var);
    hipLaunchKernelGGL(level_var_kernel, dim3((unsigned)plan.num_levels), dim3(kMergeThreads), 0, stream, f);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int64_t mp = plan.m * plan.p;
    hipLaunchKernelGGL(telescope_kernel, dim3((unsigned)ceil_div(mp, kMergeThreads)), dim3(kMergeThreads), 0,
                       stream, reinterpret_cast<const double*>(ws + plan.off_means), plan.num_levels, mp, out,
                       level_means);
    return hipGetLastError();
}

}  // namespace mlmc
