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
#include "matmul_device.hpp"

namespace mlmc {

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
    const uint32_t* abandoned;   // single-launch form: its error flag (non-zero: the estimate is NaN), else NULL
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
    const bool lost = prm.abandoned && *prm.abandoned != 0u;
    double y = 0.0;
    for (int l = 0; l < prm.num_levels; ++l) {
        const double v = lost ? __builtin_nan("") : prm.means[l * prm.sum_mp + Pd.mp_prefix + e];
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

// Set form: open-addressing table of a realisation's distinct indices, at
// least twice as many slots as draws (a power of two), four words a slot.
static int64_t set_table_slots(int64_t c)
{
    int64_t t = 2;
    while (t < 2 * c) t <<= 1;
    return t;
}
static int64_t set_bytes_per_realisation(const MatmulPlan& plan, int64_t c, int64_t kpad)
{
    return plan.nprob * (set_table_slots(c) * 4 * (int64_t)sizeof(uint32_t) + kpad * (int64_t)sizeof(double));
}
constexpr int64_t kSetBudgetBytes = 256ll << 20;

// Realisations per pass of a level of padded length kpad: as many as the
// gathered operands' budget holds (and, in the set form, its tables' region).
static int64_t level_batch_of(const MatmulPlan& plan, int64_t c, int64_t kpad)
{
    const int64_t per_sample = kpad * plan.sum_rows * plan.elem;
    int64_t level_batch = plan.gather_bytes / per_sample;
    if (plan.set_form) {
        const int64_t by_set = plan.set_bytes / set_bytes_per_realisation(plan, c, kpad);
        if (by_set < level_batch) level_batch = by_set;
    }
    if (level_batch < 1) level_batch = 1;
    if (level_batch > 65535) level_batch = 65535;
    // the sketch counts a group's padded positions in 32 bits
    if (level_batch > INT32_MAX / kpad) level_batch = INT32_MAX / kpad;
    return level_batch;
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
    if (plan.persistent) {
        e = hipMemcpyAsync(ws + plan.off_passes, plan.passes.data(), sizeof(PassDesc) * plan.passes.size(),
                           hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
    }
    // the sources are pageable host memory owned by `plan`: wait until the
    // copies have consumed them
    return hipStreamSynchronize(stream);
}

void matmul_plan_persistent(MatmulPlan& plan, const LevelRange* ranges, int num_levels)
{
    plan.persistent = false;
    plan.passes.clear();
    // the forms the single-launch kernel is built for: products in whole
    // tiles (shifted sums), or at tile 128 any shapes (Welford, as the
    // launch-per-pass form takes them there)
    if (plan.func.kind != 0 || plan.index_weights || !plan.iid || plan.set_form) return;
    if (!plan.whole_tiles && plan.tile != 128) return;
    if (plan.laws != kLawsNormal && plan.laws != kLawsUniform) return;
    if (plan.prec == 0) return;        // FP64 keeps the launch-per-pass form
    if (plan.tile != 64 && plan.tile != 128) return;
    int64_t passes = 0;
    for (int l = 0; l < num_levels; ++l) {
        const LevelRange& lr = ranges[l];
        int64_t kc, kpad;
        level_padding(plan, lr.c, lr.c_prev, kc, kpad);
        // the batch of realisations per pass, as the launch-per-pass form takes it
        const int64_t level_batch = level_batch_of(plan, lr.c, kpad);
        for (int64_t b = 0; b < lr.count; b += level_batch) {
            const int64_t batch = (lr.count - b) < level_batch ? (lr.count - b) : level_batch;
            PassDesc d;
            d.level = lr.level;
            // two accumulators for short BF16 / FP8 realisations, shifted sums
            // otherwise; Welford where the tiles are ragged
            d.stats = !plan.whole_tiles ? 0 : (plan.elem <= 2 && lr.c <= kDualMaxDraws ? 3 : 2);
            d.c = (uint32_t)lr.c;
            d.c_prev = (uint32_t)lr.c_prev;
            d.stride = (uint32_t)lr.stride;
            d.level_field = lr.level_field;
            d.k_first = (uint32_t)(lr.k_begin + b);
            int oct = 1;
            while (plan.min_rows < 1024 && oct < kGatherMaxOctets &&
                   ceil_div(kpad, (int64_t)kGatherPositions * oct * 2) * batch * plan.nprob >= 8192)
                oct *= 2;
            d.octets = oct;
            d.kc = kc;
            d.kpad = kpad;
            d.batch = batch;
            d.gx = ceil_div(kpad, (int64_t)kGatherPositions * oct);
            d.units = d.gx * batch * plan.nprob;
            d.done_before = (double)b;
            d.omega = lr.c_prev > 0 ? 1.0 - (double)lr.c / (double)lr.c_prev : 1.0;
            plan.passes.push_back(d);
            ++passes;
        }
    }
    if (passes == 0 || passes > kPersistentMaxPasses) {
        plan.passes.clear();
        return;
    }
    plan.persistent = true;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = align(plan.total);
    plan.off_passes = off;  off = align(off + sizeof(PassDesc) * plan.passes.size());
    plan.sync_words = (passes + 1) * kPhaseWords + kSyncStride;
    plan.off_sync = off;    off = align(off + sizeof(uint32_t) * plan.sync_words);
    plan.off_gather2 = off; off = align(off + (size_t)plan.gather_bytes);
    plan.off_gather3 = off; off = align(off + (size_t)plan.gather_bytes);
    plan.total = off;
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

// ---------------------------------------------------------------------------
// Set form of a realisation (the note after Alg. 1 in Sec. 3.1).
// ---------------------------------------------------------------------------
void matmul_plan_set_form(MatmulPlan& plan)
{
    plan.set_form = true;
    int64_t need = 0, least = 0;
    for (int l = 0; l < plan.num_levels; ++l) {
        int64_t kc, kpad;
        level_padding(plan, plan.c[l], l > 0 ? plan.c[l - 1] : 0, kc, kpad);
        const int64_t one = set_bytes_per_realisation(plan, plan.c[l], kpad);
        int64_t batch = plan.gather_bytes / (kpad * plan.sum_rows * plan.elem);
        if (batch < 1) batch = 1;
        if (one * batch > need) need = one * batch;
        if (one > least) least = one;
    }
    plan.set_bytes = need < kSetBudgetBytes ? need : kSetBudgetBytes;
    if (plan.set_bytes < least) plan.set_bytes = least;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    plan.off_set = align(plan.total);
    plan.total = align(plan.off_set + (size_t)plan.set_bytes);
}

struct SetParams {
    const ProblemDesc* descs;
    uint32_t c, c_prev, stride, level_field;
    int64_t kc, kpad, batch;
    uint32_t k_first, key0, key1;
    double omega;               // weight of a coarse draw, 1 - c_l / c_{l-1}
    int64_t slots;              // table slots per realisation (a power of two)
    int shift;                  // 32 - log2(slots)
    uint32_t* tables;           // [product][slot of the batch] x 4 x slots words
    double* setw;               // [product][slot of the batch][kpad]
};

constexpr uint32_t kSetEmpty = 0xFFFFFFFFu;   // no index (an index is below n < 2^32 - 1)

// Slot of index j in a realisation's table (inserted when absent).  The table
// has more slots than the realisation has draws, so the probe ends.
__device__ __forceinline__ int64_t set_slot(uint32_t* key, int64_t slots, int shift, uint32_t j)
{
    int64_t s = (int64_t)((j * 2654435761u) >> shift);
    for (;;) {
        uint32_t cur = __hip_atomic_load(key + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == kSetEmpty) {
            uint32_t expected = kSetEmpty;
            if (__hip_atomic_compare_exchange_strong(key + s, &expected, j, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                return s;
            cur = expected;
        }
        if (cur == j) return s;
        s = (s + 1) & (slots - 1);
    }
}

// One workgroup per (realisation of the pass, product): the distinct indices
// of the realisation's draws, the number of coarse (positions < kc) and of
// other draws that took each, and the first position that drew it.  Every
// position then gets its weight: at the first position of an index, the sum
// of the weights of its draws (omega per coarse draw, 1 per other draw, as
// the gather folds them into a_t); 0 at every other position and at padding.
// The counts are integer atomics, so the weights do not depend on the order
// of the updates.
__global__ __launch_bounds__(256) void set_weights_kernel(SetParams prm)
{
    const int64_t slot = blockIdx.x, bz = blockIdx.y;
    const ProblemDesc& Pd = prm.descs[bz];
    const uint32_t n = (uint32_t)Pd.n;
    const uint32_t k = prm.k_first + (uint32_t)slot;
    const uint32_t sid_index = stream_id(kTagIndex, prm.level_field, Pd.sid_problem);
    uint32_t* key = prm.tables + (bz * prm.batch + slot) * 4 * prm.slots;
    uint32_t* cnt_other = key + prm.slots;
    uint32_t* cnt_coarse = cnt_other + prm.slots;
    uint32_t* first = cnt_coarse + prm.slots;
    for (int64_t i = threadIdx.x; i < prm.slots; i += blockDim.x) {
        key[i] = kSetEmpty;
        cnt_other[i] = 0u;
        cnt_coarse[i] = 0u;
        first[i] = 0xFFFFFFFFu;
    }
    __threadfence();
    __syncthreads();
    for (int64_t pos = threadIdx.x; pos < prm.kpad; pos += blockDim.x) {
        const int64_t t = draw_of_position(pos, prm.kc, prm.c, prm.c_prev, prm.stride);
        if (t < 0) continue;
        const uint32_t j = draw_index((uint32_t)t, k, sid_index, prm.key0, prm.key1, n);
        const int64_t s = set_slot(key, prm.slots, prm.shift, j);
        __hip_atomic_fetch_add(pos < prm.kc ? cnt_coarse + s : cnt_other + s, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_min(first + s, (uint32_t)pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    __syncthreads();
    double* w = prm.setw + (bz * prm.batch + slot) * prm.kpad;
    for (int64_t pos = threadIdx.x; pos < prm.kpad; pos += blockDim.x) {
        const int64_t t = draw_of_position(pos, prm.kc, prm.c, prm.c_prev, prm.stride);
        double v = 0.0;
        if (t >= 0) {
            const uint32_t j = draw_index((uint32_t)t, k, sid_index, prm.key0, prm.key1, n);
            const int64_t s = set_slot(key, prm.slots, prm.shift, j);
            if (__hip_atomic_load(first + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)pos) {
                const uint32_t other = __hip_atomic_load(cnt_other + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t coarse = __hip_atomic_load(cnt_coarse + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v = (double)other + prm.omega * (double)coarse;
            }
        }
        w[pos] = v;
    }
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
    g.setw = nullptr;
    if (plan.set_form) {
        // the distinct indices of every realisation of the pass and the
        // weights of the positions that generate them
        SetParams sp;
        sp.descs = descs;
        sp.c = (uint32_t)lr.c;
        sp.c_prev = (uint32_t)lr.c_prev;
        sp.stride = (uint32_t)lr.stride;
        sp.level_field = lr.level_field;
        sp.kc = kc;
        sp.kpad = kpad;
        sp.batch = batch;
        sp.k_first = (uint32_t)k_first;
        sp.key0 = keys.key0;
        sp.key1 = keys.key1;
        sp.omega = lr.c_prev > 0 ? 1.0 - (double)lr.c / (double)lr.c_prev : 1.0;
        sp.slots = set_table_slots(lr.c);
        int lg = 0;
        while ((int64_t)1 << lg < sp.slots) ++lg;
        sp.shift = 32 - lg;
        sp.tables = reinterpret_cast<uint32_t*>(ws + plan.off_set);
        sp.setw = reinterpret_cast<double*>(ws + plan.off_set + (size_t)(plan.nprob * batch * 4 * sp.slots) *
                                                                    sizeof(uint32_t));
        {
            ScopedTiming t(timer, 1);
            hipLaunchKernelGGL(set_weights_kernel, dim3((unsigned)batch, (unsigned)plan.nprob), dim3(256), 0, stream,
                               sp);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        g.setw = sp.setw;
    }
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
        // with a target function the sketch needs the coarse sum itself: no
        // weight; in the set form the position weights already hold it
        g.omega = lr.c_prev > 0 && plan.func.kind == 0 && !plan.set_form ? 1.0 - (double)lr.c / (double)lr.c_prev
                                                                          : 1.0;
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
    const int64_t level_batch = level_batch_of(plan, lr.c, kpad);
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
    f.abandoned = plan.persistent ? reinterpret_cast<const uint32_t*>(ws + plan.off_sync) +
                                        (int64_t)(plan.passes.size() + 1) * kPhaseWords
                                  : nullptr;
    hipLaunchKernelGGL(level_var_kernel, dim3((unsigned)plan.num_levels, (unsigned)plan.nprob), dim3(kMergeThreads),
                       0, stream, f);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || !write_outputs) return err;
    hipLaunchKernelGGL(telescope_kernel, dim3((unsigned)ceil_div(plan.max_mp, kMergeThreads), (unsigned)plan.nprob),
                       dim3(kMergeThreads), 0, stream, f);
    return hipGetLastError();
}

}  // namespace mlmc
