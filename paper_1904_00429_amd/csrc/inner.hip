// Inner-product level sampling (Sec. 2; Alg. 1 with m = p = 1).
//
// A level sample of realisation k is
//   D_k = (n / c) * ( (1 - c / c_prev) * sum_{t < c_prev} x_{r_t} y_{r_t}
//                     + sum_{c_prev <= t < c} x_{r_t} y_{r_t} ),
// the fine sketch (eq. (1) with xi = 1/n over c draws) minus the coarse sketch
// over the first c_prev of the same draws; at level 0 (c_prev = 0) the fine
// sketch alone.  Nothing is read from memory except reparameterised
// means/scales: indices and values are regenerated from the counter-based
// stream, so the kernel is bound by VALU issue (Philox is 90% of the work).
// Separate instantiations (template flags, so the plain kernel is unchanged)
// give the other forms: a target function f (FN: f of both sketches), weighted
// index draws (IW: per-draw factor 1 / (n xi_j)), the stride coupling (ST: the
// coarse draws are every M-th draw) and 32-bit index words (W32).
//
// One launch covers every level of a phase (the pilot, or the extension):
// workgroups are dealt to levels in proportion to each level's draw count, so
// the whole GPU works on all levels at once and no level runs a grid too small
// to fill the chip.  Inside a level, a group of G lanes (a power of two, up to
// the whole 256-lane workgroup) owns one realisation at a time; its lanes take
// draw pairs (2q, 2q+1), which share one Philox call of the index stream (with
// 32-bit index words, draw quads 4g .. 4g+3 share one call).  G is chosen so
// every lane gets at least eight pairs, which amortises the per-realisation
// reduction (a butterfly of cross-lane shuffles, plus an LDS step when the
// group spans several waves).
//
// Statistics: every lane of a group holds D_k after the reduction and updates
// FP64 sums shifted by the group's first sample K (n, S1 = sum (D - K),
// S2 = sum (D - K)^2: no division per sample, no cancellation since K is a
// draw of the same law).  At the end each group turns them into (n, mean, M2),
// a fixed-order Chan tree in LDS merges the groups of the workgroup, and a
// one-block-per-level kernel folds the workgroup partials into the level's
// running state in a fixed order, so results are bitwise reproducible.
#include "internal.hpp"

namespace mlmc {

constexpr int kInnerBlock = 256;
constexpr int kInnerMaxBlocks = 8192;
constexpr int64_t kInnerTargetBlocks = 8192;
constexpr int64_t kInnerMinPairsPerBlock = 2048;

struct InnerLevel {
    uint32_t c, c_prev, k_begin, count;
    uint32_t g_log2;          // lanes per realisation = 1 << g_log2, at most 256
    uint32_t block_begin, blocks;
    uint32_t sid_index, sid_value;
    uint32_t stride;          // stride coupling M: the coarse draws are M - 1, 2M - 1, ... (0: prefix)
    double scale;             // n / c
    double scale_c;           // n / c_prev (0 at level 0)
    double omega;             // 1 - c / c_prev, weight of the first c_prev draws
};

struct InnerMultiParams {
    uint32_t n;
    uint32_t n_shift;         // 32 - log2(n) when n is a power of two <= 2^32, else 0xFFFFFFFF
    uint32_t key0, key1;
    int32_t num_levels;
    Law x, y;
    TargetFunc f;             // applied to both sketches (FN kernels)
    const uint32_t* iw;       // index weights (IW kernels): xi_j = w_j / W
    const uint64_t* cum;      // their cumulative sums, W = cum[n - 1]
    Moments* partials;        // one per workgroup
    uint32_t total_blocks;    // workgroups with work (a larger grid's others leave at once)
    InnerLevel lev[32];
};

// One block per level: fold that level's workgroup partials (thread i takes
// partials i, i + 256, ... in order, then a tree), then append the result to
// the level's running state.
struct InnerFoldParams {
    int32_t num_levels;
    uint32_t block_begin[32];
    uint32_t blocks[32];
    const Moments* partials;
    Moments* level_state;
};

// The parameters of a phase's level launch and fold, in device memory: the
// kernels read them from there, so a launch whose partition the device
// computes (after eq. (28) on the device) is enqueued like any other.
struct InnerSlot {
    InnerMultiParams multi;
    InnerFoldParams fold;
    uint32_t arrivals;        // fold workgroups done (the last one runs the fold's tail)
};

// Index from its two Philox words; a power-of-two n is the top bits of the
// 64-bit word, floor(x n / 2^64) = hi >> (32 - log2 n), which is the same value.
__device__ __forceinline__ uint32_t inner_index(uint32_t lo, uint32_t hi, const InnerMultiParams& prm)
{
    if (prm.n_shift != 0xFFFFFFFFu) return prm.n_shift >= 32 ? 0u : hi >> prm.n_shift;
    return index_from_words(lo, hi, prm.n);
}

template <typename T, int LAWS>
__device__ __forceinline__ T inner_product_term(const InnerMultiParams& prm, uint32_t k, uint32_t j,
                                                uint32_t sid_value)
{
    if constexpr (LAWS == kLawsExperiment) {
        // x_j is element 0 and y_j element 1 of the column vector v_j, each
        // from its own call of the experiment stream
        const uint32_t sid_exp = (sid_value & 0x0FFFFFFFu) | (kTagExperiment << 28);
        const T xv = (T)experiment_value(prm.x.kind, prm.x.loc, prm.x.scale, prm.x.aux, 0u, k, j, sid_exp,
                                         prm.key0, prm.key1);
        const T yv = (T)experiment_value(prm.y.kind, prm.y.loc, prm.y.scale, prm.y.aux, 1u, k, j, sid_exp,
                                         prm.key0, prm.key1);
        return xv * yv;
    }
    const Words4 w = philox4x32_10(0u, k, j, sid_value, prm.key0, prm.key1);
    const T u0 = unit<T>(w.w0);
    const T u1 = unit<T>(w.w1);
    if (LAWS == kLawsUniform) {
        const T xv = fma(u0, (T)(2.0 * prm.x.scale), (T)(prm.x.loc - prm.x.scale));
        const T yv = fma(u1, (T)(2.0 * prm.y.scale), (T)(prm.y.loc - prm.y.scale));
        return xv * yv;
    }
    T z0, z1;
    box_muller(u0, u1, z0, z1);
    if (LAWS == kLawsNormal) {
        const T xv = fma(z0, (T)prm.x.scale, (T)prm.x.loc);
        const T yv = fma(z1, (T)prm.y.scale, (T)prm.y.loc);
        return xv * yv;
    }
    const T xv = law_value<T>(prm.x, z0, u0, (int64_t)j);
    const T yv = law_value<T>(prm.y, z1, u1, (int64_t)j);
    return xv * yv;
}

// W32: the four product terms of draw quad g (draws 4g .. 4g + 3) of
// realisation k from one Philox call of the index stream, r = w >> (32 -
// log2 n) for each 32-bit word (n a power of two); draws past c give 0.
template <typename T, int LAWS>
__device__ __forceinline__ void quad_terms(const InnerMultiParams& prm, const InnerLevel& L, uint32_t g, uint32_t k,
                                           T (&v)[4])
{
    const Words4 w = philox4x32_10(g, k, 0u, L.sid_index, prm.key0, prm.key1);
    const uint32_t r[4] = {w.w0, w.w1, w.w2, w.w3};
    const uint32_t sh = prm.n_shift;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t j = sh >= 32u ? 0u : r[i] >> sh;
        v[i] = (4u * g + (uint32_t)i < L.c) ? inner_product_term<T, LAWS>(prm, k, j, L.sid_value) : (T)0;
    }
}

// Sum of the product terms of quads g0, g0 + G, ... below g_end into acc.
template <typename T, int LAWS>
__device__ __forceinline__ void sum_quads(const InnerMultiParams& prm, const InnerLevel& L, uint32_t g0,
                                          uint32_t g_end, uint32_t G, uint32_t k, T& acc)
{
    for (uint32_t g = g0; g < g_end; g += G) {
        T v[4];
        quad_terms<T, LAWS>(prm, L, g, k, v);
        acc += (v[0] + v[1]) + (v[2] + v[3]);
    }
}

// The two product terms of draw pair q (draws 2q and 2q + 1) of realisation k;
// IW: weighted draws, each term times 1 / (n xi_j) (eq. (18) with a general xi).
template <typename T, int LAWS, bool IW>
__device__ __forceinline__ void pair_terms(const InnerMultiParams& prm, const InnerLevel& L, uint32_t q,
                                           uint32_t k, T& v0, T& v1)
{
    const Words4 w = philox4x32_10(q, k, 0u, L.sid_index, prm.key0, prm.key1);
    if constexpr (IW) {
        const uint64_t total = prm.cum[prm.n - 1];
        const uint32_t r0 = index_from_cumulative(w.w0, w.w1, prm.cum, prm.n, total);
        const uint32_t r1 = index_from_cumulative(w.w2, w.w3, prm.cum, prm.n, total);
        const double tn = (double)total / (double)prm.n;
        v0 = inner_product_term<T, LAWS>(prm, k, r0, L.sid_value) * (T)(tn / (double)prm.iw[r0]);
        v1 = (2u * q + 1u < L.c)
                 ? inner_product_term<T, LAWS>(prm, k, r1, L.sid_value) * (T)(tn / (double)prm.iw[r1])
                 : (T)0;
    } else {
        const uint32_t r0 = inner_index(w.w0, w.w1, prm);
        const uint32_t r1 = inner_index(w.w2, w.w3, prm);
        v0 = inner_product_term<T, LAWS>(prm, k, r0, L.sid_value);
        v1 = (2u * q + 1u < L.c) ? inner_product_term<T, LAWS>(prm, k, r1, L.sid_value) : (T)0;
    }
}

// Sum of the product terms of pairs q0, q0 + G, q0 + 2G, ... below q_end into
// acc, in increasing q; two pairs per iteration give the scheduler two
// independent Philox chains to interleave.
template <typename T, int LAWS, bool IW>
__device__ __forceinline__ void sum_pairs(const InnerMultiParams& prm, const InnerLevel& L, uint32_t q0,
                                          uint32_t q_end, uint32_t G, uint32_t k, T& acc)
{
    uint32_t q = q0;
    for (; q + G < q_end; q += 2u * G) {
        T a0, a1, b0, b1;
        pair_terms<T, LAWS, IW>(prm, L, q, k, a0, a1);
        pair_terms<T, LAWS, IW>(prm, L, q + G, k, b0, b1);
        acc += a0 + a1;
        acc += b0 + b1;
    }
    if (q < q_end) {
        T a0, a1;
        pair_terms<T, LAWS, IW>(prm, L, q, k, a0, a1);
        acc += a0 + a1;
    }
}

// FN: a target function f other than the identity.  The level sample is then
// f(Z_l) - f(Z_{l-1}) with Z_l = (n / c_l)(C + F) and Z_{l-1} = (n / c_{l-1}) C,
// C and F the sums over the coarse and the remaining draws, so both sums are
// reduced over the group instead of their weighted combination.
// ST: stride coupling.  Every pair is summed, and each of its two draws goes
// to the coarse sum when its number t has (t + 1) % M == 0, else to the fine
// sum (a separate instantiation, so the prefix kernels are unchanged).
// W32: 32-bit index words, the lane walks draw quads instead of pairs (same
// coarse range / straddling unit / fine range split, or the stride predicate).
template <typename T, int LAWS, bool FN, bool IW, bool ST, bool W32>
__global__ __launch_bounds__(kInnerBlock) void inner_multi_kernel(const InnerMultiParams* __restrict__ pp)
{
    const InnerMultiParams& prm = *pp;
    if (blockIdx.x >= prm.total_blocks) return;
    __shared__ double wave_sum[kInnerBlock / kWave];
    __shared__ double wave_sum_c[FN ? kInnerBlock / kWave : 1];
    __shared__ Moments slots[kInnerBlock];

    int l = 0;
    while (l + 1 < prm.num_levels && blockIdx.x >= prm.lev[l].block_begin + prm.lev[l].blocks) ++l;
    const InnerLevel& L = prm.lev[l];
    const uint32_t g = L.g_log2;
    const int G = 1 << g;
    const int groups = G >= kInnerBlock ? 1 : kInnerBlock / G;
    const int gi = threadIdx.x >> g;
    const int lane_g = threadIdx.x & (G - 1);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const uint64_t bl = blockIdx.x - L.block_begin;
    const uint32_t s_lo = (uint32_t)(bl * L.count / L.blocks);
    const uint32_t s_hi = (uint32_t)((bl + 1) * L.count / L.blocks);
    const uint32_t iters = (s_hi - s_lo + groups - 1) / groups;
    const uint32_t pairs = (L.c + 1u) >> 1;
    const uint32_t coarse_pairs = L.c_prev >> 1;   // pairs whose two draws are both < c_prev
    const bool odd_prev = (L.c_prev & 1u) != 0u;
    const T omega = (T)L.omega;

    double n = 0.0, K = 0.0, S1 = 0.0, S2 = 0.0;
    for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t s = s_lo + (uint32_t)gi + it * (uint32_t)groups;
        const bool active = s < s_hi;
        const uint32_t k = L.k_begin + (active ? s : s_lo);
        // Pairs below coarse_pairs hold two coarse draws; with an odd c_prev
        // the next pair straddles (its first draw is coarse, its second
        // fine); the rest are fine.  The lane takes pairs q = lane_g (mod G).
        T acc_coarse = (T)0, acc_fine = (T)0;
        if constexpr (W32) {
            const uint32_t quads = (L.c + 3u) >> 2;
            if constexpr (ST) {
                const uint32_t M = L.stride;
                for (uint32_t g4 = (uint32_t)lane_g; g4 < quads; g4 += (uint32_t)G) {
                    T v[4];
                    quad_terms<T, LAWS>(prm, L, g4, k, v);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (M != 0u && (4u * g4 + (uint32_t)i + 1u) % M == 0u) acc_coarse += v[i];
                        else acc_fine += v[i];
                    }
                }
            } else {
                // quads below cq hold four coarse draws; with c_prev % 4 = rem > 0
                // quad cq straddles (its first rem draws are coarse)
                const uint32_t cq = L.c_prev >> 2, rem = L.c_prev & 3u;
                sum_quads<T, LAWS>(prm, L, (uint32_t)lane_g, cq, (uint32_t)G, k, acc_coarse);
                if (rem != 0u && (cq & (uint32_t)(G - 1)) == (uint32_t)lane_g) {
                    T v[4];
                    quad_terms<T, LAWS>(prm, L, cq, k, v);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if ((uint32_t)i < rem) acc_coarse += v[i];
                        else acc_fine += v[i];
                    }
                }
                const uint32_t fine_begin = cq + (rem != 0u ? 1u : 0u);
                const uint32_t g_fine = fine_begin + (((uint32_t)lane_g - fine_begin) & (uint32_t)(G - 1));
                sum_quads<T, LAWS>(prm, L, g_fine, quads, (uint32_t)G, k, acc_fine);
            }
        } else if constexpr (ST) {
            // L.stride >= 2 above level 0 (c_l >= 2 c_{l-1}); 0 at level 0 (no coarse draws)
            const uint32_t M = L.stride;
            for (uint32_t q = (uint32_t)lane_g; q < pairs; q += (uint32_t)G) {
                T a0, a1;
                pair_terms<T, LAWS, IW>(prm, L, q, k, a0, a1);
                const bool c0 = M != 0u && (2u * q + 1u) % M == 0u;
                const bool c1 = M != 0u && (2u * q + 2u) % M == 0u;
                if (c0) acc_coarse += a0; else acc_fine += a0;
                if (c1) acc_coarse += a1; else acc_fine += a1;
            }
        } else {
            sum_pairs<T, LAWS, IW>(prm, L, (uint32_t)lane_g, coarse_pairs, (uint32_t)G, k, acc_coarse);
            if (odd_prev && (coarse_pairs & (uint32_t)(G - 1)) == (uint32_t)lane_g) {
                T a0, a1;
                pair_terms<T, LAWS, IW>(prm, L, coarse_pairs, k, a0, a1);
                acc_coarse += a0;
                acc_fine += a1;
            }
            const uint32_t fine_begin = coarse_pairs + (odd_prev ? 1u : 0u);
            const uint32_t q_fine = fine_begin + (((uint32_t)lane_g - fine_begin) & (uint32_t)(G - 1));
            sum_pairs<T, LAWS, IW>(prm, L, q_fine, pairs, (uint32_t)G, k, acc_fine);
        }
        T part = FN ? acc_fine : omega * acc_coarse + acc_fine;
        T part_c = acc_coarse;
        const int width = G < kWave ? G : kWave;
        for (int off = width >> 1; off > 0; off >>= 1) {
            part += __shfl_xor(part, off, kWave);
            if constexpr (FN) part_c += __shfl_xor(part_c, off, kWave);
        }
        double total = (double)part, total_c = (double)part_c;
        if (G > kWave) {
            // the group spans G / 64 waves: add their sums in wave order
            if (lane == 0) {
                wave_sum[wave] = total;
                if constexpr (FN) wave_sum_c[wave] = total_c;
            }
            __syncthreads();
            const int first = (gi * G) / kWave;
            total = 0.0;
            total_c = 0.0;
            for (int w = 0; w < G / kWave; ++w) {
                total += wave_sum[first + w];
                if constexpr (FN) total_c += wave_sum_c[first + w];
            }
            __syncthreads();
        }
        if (active) {
            double d;
            if constexpr (FN) {
                d = target_value(prm.f.kind, L.scale * (total_c + total), prm.f.theta0, prm.f.theta1);
                if (L.c_prev > 0u) d -= target_value(prm.f.kind, L.scale_c * total_c, prm.f.theta0, prm.f.theta1);
            } else {
                d = L.scale * total;
            }
            if (n == 0.0) K = d;
            n += 1.0;
            const double dev = d - K;
            S1 += dev;
            S2 = fma(dev, dev, S2);
        }
    }
    if (lane_g == 0) {
        Moments m = {0.0, 0.0, 0.0};
        if (n > 0.0) {
            m.n = n;
            m.mean = K + S1 / n;
            m.m2 = fmax(S2 - S1 * (S1 / n), 0.0);
        }
        slots[gi] = m;
    }
    __syncthreads();
    for (int half = groups >> 1; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) slots[threadIdx.x] = chan_merge(slots[threadIdx.x], slots[threadIdx.x + half]);
        __syncthreads();
    }
    if (threadIdx.x == 0) prm.partials[blockIdx.x] = slots[0];
}

__global__ void inner_telescope_kernel(const Moments* level_state, int num_levels, double* out,
                                       double* level_means, double* level_var)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double y = 0.0;
    for (int l = 0; l < num_levels; ++l) {
        const Moments st = level_state[l];
        y += st.mean;
        if (level_means) level_means[l] = st.mean;
        level_var[l] = st.n > 1.0 ? st.m2 / (st.n - 1.0) : 0.0;
    }
    *out = y;
}

size_t inner_partials_capacity() { return kInnerMaxBlocks; }

// Lanes per realisation: at least eight draw pairs per lane, at most a workgroup.
__host__ __device__ inline uint32_t lanes_log2_for(int64_t c)
{
    const int64_t pairs = (c + 1) / 2;
    uint32_t g = 0;
    while (g < 8 && (int64_t(8) << (g + 1)) <= pairs) ++g;
    return g;
}

// The partition of a phase's launch over its levels (host for the pilot and
// fixed phases, device for the extension that eq. (28) schedules there):
// workgroups dealt to levels in proportion to their draw pairs, at most
// kInnerMaxBlocks in all.  Fills the level fields of prm and the fold's
// ranges; returns the number of workgroups with work.
__host__ __device__ inline uint32_t inner_partition(const LevelRange* ranges, int num_levels, int64_t n,
                                                    uint32_t problem, InnerMultiParams& prm, InnerFoldParams& fold)
{
    double work[32], total = 0.0;
    for (int i = 0; i < num_levels; ++i) {
        work[i] = ranges[i].count > 0 ? (double)ranges[i].count * (double)((ranges[i].c + 1) / 2) : 0.0;
        total += work[i];
    }
    double target = total / (double)kInnerMinPairsPerBlock;
    if (target > (double)kInnerTargetBlocks) target = (double)kInnerTargetBlocks;
    if (target < 1.0) target = 1.0;
    uint32_t next = 0;
    fold.num_levels = num_levels;
    for (int i = 0; i < num_levels; ++i) {
        const LevelRange& lr = ranges[i];
        InnerLevel& L = prm.lev[i];
        L.c = (uint32_t)lr.c;
        L.c_prev = (uint32_t)lr.c_prev;
        L.k_begin = (uint32_t)lr.k_begin;
        L.count = (uint32_t)(lr.count > 0 ? lr.count : 0);
        L.g_log2 = lanes_log2_for(lr.c);
        L.sid_index = stream_id(kTagIndex, lr.level_field, problem);
        L.sid_value = stream_id(kTagValue, lr.level_field, problem);
        L.scale = (double)n / (double)lr.c;
        L.scale_c = lr.c_prev > 0 ? (double)n / (double)lr.c_prev : 0.0;
        L.omega = lr.c_prev > 0 ? 1.0 - (double)lr.c / (double)lr.c_prev : 0.0;
        L.stride = (uint32_t)lr.stride;
        int64_t blocks = 0;
        if (L.count > 0 && total > 0.0) {
            const int64_t groups = (int64_t)1 << (L.g_log2 >= 8 ? 0 : 8 - L.g_log2);
            const int64_t most = ceil_div(L.count, groups);
            blocks = (int64_t)(target * work[i] / total + 0.5);
            if (blocks < 1) blocks = 1;
            if (blocks > most) blocks = most;
        }
        L.block_begin = next;
        L.blocks = (uint32_t)blocks;
        fold.block_begin[i] = next;
        fold.blocks[i] = (uint32_t)blocks;
        next += (uint32_t)blocks;
    }
    if (next > (uint32_t)kInnerMaxBlocks) {
        // scale every level down proportionally (at least one block each)
        uint32_t again = 0;
        for (int i = 0; i < num_levels; ++i) {
            int64_t b = prm.lev[i].blocks;
            if (b > 0) {
                b = (int64_t)((double)b * (kInnerMaxBlocks - num_levels) / (double)next);
                if (b < 1) b = 1;
            }
            prm.lev[i].block_begin = again;
            prm.lev[i].blocks = (uint32_t)b;
            fold.block_begin[i] = again;
            fold.blocks[i] = (uint32_t)b;
            again += (uint32_t)b;
        }
        next = again;
    }
    prm.total_blocks = next;
    return next;
}

// Copies a phase's parameters into their device slot (a kernel, so that the
// copy is captured like any launch); with `zero`, also clears the first
// `levels` level states (the start of an estimate).
__global__ void inner_store_kernel(InnerSlot src, InnerSlot* dst, Moments* zero, int levels)
{
    const uint32_t* a = reinterpret_cast<const uint32_t*>(&src);
    uint32_t* b = reinterpret_cast<uint32_t*>(dst);
    for (uint32_t i = threadIdx.x; i < sizeof(InnerSlot) / 4; i += blockDim.x) b[i] = a[i];
    if (zero && (int)threadIdx.x < levels) zero[threadIdx.x] = Moments{0.0, 0.0, 0.0};
}

// eq. (28) on the device after the pilot: V_l of every level (the telescope's
// formula), N_l by schedule_counts (the host's arithmetic), and the extension's
// partition into the parameter slot; counts[l] = the realisations level l has
// after the extension (the pilot's when the schedule fails, whose code goes to
// status).  One thread.
struct InnerScheduleParams {
    InnerMultiParams base;           // the laws, keys and partials of the launch
    int32_t num_levels;
    double eps;
    int64_t pilot, max_total_draws, n;
    uint32_t problem;
    int64_t c[32];
    uint32_t level_field[32], stride[32];
    const Moments* level_state;
    InnerSlot* slot;
    int64_t* counts;
    int32_t* status;                 // schedule_counts' code, then its level
    double* status_value;
};

// eq. (28) on the device into `out` (the extension's parameters).  One thread.
__device__ inline void inner_schedule(const InnerScheduleParams& sp, InnerSlot& out)
{
    const int L1 = sp.num_levels;
    double var[32];
    int64_t N[32];
    for (int l = 0; l < L1; ++l) {
        const Moments st = sp.level_state[l];
        var[l] = st.n > 1.0 ? st.m2 / (st.n - 1.0) : 0.0;
    }
    int bad_level = 0;
    double bad_value = 0.0;
    const int code = schedule_counts(sp.eps, sp.c, var, L1, sp.pilot, sp.max_total_draws, N, &bad_level, &bad_value);
    LevelRange ranges[32];
    for (int l = 0; l < L1; ++l) {
        LevelRange& r = ranges[l];
        r.level = l;
        r.level_field = sp.level_field[l];
        r.c = sp.c[l];
        r.c_prev = l > 0 ? sp.c[l - 1] : 0;
        r.k_begin = sp.pilot;
        r.count = code == 0 ? N[l] - sp.pilot : 0;
        r.stride = sp.stride[l];
        sp.counts[l] = code == 0 ? N[l] : sp.pilot;
    }
    out.multi = sp.base;
    inner_partition(ranges, L1, sp.n, sp.problem, out.multi, out.fold);
    out.fold.partials = sp.base.partials;
    out.fold.level_state = const_cast<Moments*>(sp.level_state);
    sp.status[0] = code;
    sp.status[1] = bad_level;
    *sp.status_value = bad_value;
}

// What the fold kernel does after folding: nothing, eq. (28) for the next
// phase (its parameters into the slot the fold has read), or the telescoping
// sum with the level means and variances.
struct InnerTail {
    InnerScheduleParams sched;       // TAIL 1
    double* out;                     // TAIL 2: Y, then level means (nullable) and V_l
    double* level_means;
    double* level_var;
};

// One workgroup per level folds that level's workgroup partials (thread i
// takes partials i, i + 256, ... in order, then a tree in LDS) and appends the
// result to the level's running state; the last workgroup to finish (an
// arrival counter in the slot, released and acquired at agent scope) runs the
// tail and clears the counter.
template <int TAIL>
__global__ __launch_bounds__(kInnerBlock) void inner_fold_kernel(InnerSlot* slot, InnerTail tail)
{
    __shared__ Moments slots[kInnerBlock];
    __shared__ InnerSlot next[1];
    __shared__ int last;
    const InnerFoldParams& prm = slot->fold;
    const int l = blockIdx.x;
    const int L1 = prm.num_levels;
    const Moments* part = prm.partials + prm.block_begin[l];
    const uint32_t blocks = prm.blocks[l];
    Moments st = {0.0, 0.0, 0.0};
    for (uint32_t i = threadIdx.x; i < blocks; i += kInnerBlock) st = chan_merge(st, part[i]);
    slots[threadIdx.x] = st;
    __syncthreads();
    for (int half = kInnerBlock >> 1; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) slots[threadIdx.x] = chan_merge(slots[threadIdx.x], slots[threadIdx.x + half]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && blocks > 0) prm.level_state[l] = chan_merge(prm.level_state[l], slots[0]);
    if constexpr (TAIL == 0) return;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t ticket = __hip_atomic_fetch_add(&slot->arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = ticket == (uint32_t)L1 - 1u;
        if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (!last) return;
    if constexpr (TAIL == 1) {
        // every other workgroup is done with the slot: thread 0 schedules the
        // next phase into LDS (its counter cleared), then the workgroup
        // writes the slot
        if (threadIdx.x == 0) {
            inner_schedule(tail.sched, next[0]);
            next[0].arrivals = 0u;
        }
        __syncthreads();
        const uint32_t* a = reinterpret_cast<const uint32_t*>(&next[0]);
        uint32_t* b = reinterpret_cast<uint32_t*>(slot);
        for (uint32_t i = threadIdx.x; i < sizeof(InnerSlot) / 4; i += blockDim.x) b[i] = a[i];
    }
    if constexpr (TAIL == 2) {
        if (threadIdx.x == 0) {
            double y = 0.0;
            for (int v = 0; v < L1; ++v) {
                const Moments sv = prm.level_state[v];
                y += sv.mean;
                if (tail.level_means) tail.level_means[v] = sv.mean;
                tail.level_var[v] = sv.n > 1.0 ? sv.m2 / (sv.n - 1.0) : 0.0;
            }
            *tail.out = y;
            __hip_atomic_store(&slot->arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename T, bool FN, bool IW, bool ST>
static void launch_inner(int laws, dim3 grid, hipStream_t stream, const InnerMultiParams* prm)
{
    const dim3 block(kInnerBlock);
    if (laws == kLawsUniform)
        hipLaunchKernelGGL((inner_multi_kernel<T, kLawsUniform, FN, IW, ST, false>), grid, block, 0, stream, prm);
    else if (laws == kLawsNormal)
        hipLaunchKernelGGL((inner_multi_kernel<T, kLawsNormal, FN, IW, ST, false>), grid, block, 0, stream, prm);
    else if (laws == kLawsExperiment)
        hipLaunchKernelGGL((inner_multi_kernel<T, kLawsExperiment, FN, IW, ST, false>), grid, block, 0, stream, prm);
    else
        hipLaunchKernelGGL((inner_multi_kernel<T, kLawsAny, FN, IW, ST, false>), grid, block, 0, stream, prm);
}

// 32-bit index words: uniform draws and the classic laws only (the host checks)
template <typename T, bool FN, bool ST>
static void launch_inner_w32(int laws, dim3 grid, hipStream_t stream, const InnerMultiParams* prm)
{
    const dim3 block(kInnerBlock);
    if (laws == kLawsUniform)
        hipLaunchKernelGGL((inner_multi_kernel<T, kLawsUniform, FN, false, ST, true>), grid, block, 0, stream, prm);
    else if (laws == kLawsNormal)
        hipLaunchKernelGGL((inner_multi_kernel<T, kLawsNormal, FN, false, ST, true>), grid, block, 0, stream, prm);
    else
        hipLaunchKernelGGL((inner_multi_kernel<T, kLawsAny, FN, false, ST, true>), grid, block, 0, stream, prm);
}

template <typename T>
static void launch_inner_forms(int laws, dim3 grid, hipStream_t stream, const InnerMultiParams* prm, bool fn,
                               bool iw, bool st, bool w32)
{
    if (w32) {
        if (fn && st) launch_inner_w32<T, true, true>(laws, grid, stream, prm);
        else if (fn) launch_inner_w32<T, true, false>(laws, grid, stream, prm);
        else if (st) launch_inner_w32<T, false, true>(laws, grid, stream, prm);
        else launch_inner_w32<T, false, false>(laws, grid, stream, prm);
        return;
    }
    if (st) {
        // the stride coupling: one instantiation per precision, law pair and form
        if (fn && iw) launch_inner<T, true, true, true>(laws, grid, stream, prm);
        else if (fn) launch_inner<T, true, false, true>(laws, grid, stream, prm);
        else if (iw) launch_inner<T, false, true, true>(laws, grid, stream, prm);
        else launch_inner<T, false, false, true>(laws, grid, stream, prm);
        return;
    }
    if (fn && iw) launch_inner<T, true, true, false>(laws, grid, stream, prm);
    else if (fn) launch_inner<T, true, false, false>(laws, grid, stream, prm);
    else if (iw) launch_inner<T, false, true, false>(laws, grid, stream, prm);
    else launch_inner<T, false, false, false>(laws, grid, stream, prm);
}

// The parameters of a launch that do not depend on the levels.
static InnerMultiParams inner_base(int64_t n, const Law& x, const Law& y, const TargetFunc& f, const IndexWeights& iw,
                                   const StreamKeys& keys, int num_levels, Moments* partials)
{
    InnerMultiParams prm;
    prm.f = f;
    prm.iw = iw.w;
    prm.cum = iw.cum;
    prm.n = (uint32_t)n;
    prm.n_shift = 0xFFFFFFFFu;
    if ((n & (n - 1)) == 0) {
        uint32_t lg = 0;
        while ((int64_t(1) << lg) < n) ++lg;
        prm.n_shift = 32u - lg;     // n = 1 gives a shift of 32: every index is 0
    }
    prm.key0 = keys.key0;
    prm.key1 = keys.key1;
    prm.num_levels = num_levels;
    prm.x = x;
    prm.y = y;
    prm.partials = partials;
    prm.total_blocks = 0;
    return prm;
}

// The level launch (grid workgroups, parameters in the slot), then the fold
// with its tail.
template <int TAIL>
static hipError_t inner_launch(dim3 grid, int num_levels, const Law& x, const Law& y, const TargetFunc& f,
                               const IndexWeights& iw, int prec, bool stride, bool index_word32, int64_t n,
                               InnerSlot* slot, const InnerTail& tail, hipStream_t stream, KernelTimer* timer)
{
    const int laws = law_pair_kind(x.kind, y.kind);
    // the laws of Sec. 4 pair only with each other
    if (laws != kLawsExperiment && (x.kind >= kLawExperimentFirst || y.kind >= kLawExperimentFirst))
        return hipErrorInvalidValue;
    // 32-bit index words: power-of-two n, uniform draws, classic laws
    if (index_word32 && ((n & (n - 1)) != 0 || iw.w || laws == kLawsExperiment)) return hipErrorInvalidValue;
    {
        ScopedTiming t(timer, 0);
        const InnerMultiParams* pp = &slot->multi;
        if (prec == 0) launch_inner_forms<double>(laws, grid, stream, pp, f.kind != 0, iw.w != nullptr, stride,
                                                  index_word32);
        else launch_inner_forms<float>(laws, grid, stream, pp, f.kind != 0, iw.w != nullptr, stride, index_word32);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ScopedTiming t(timer, TAIL == 0 ? 2 : 3);
        hipLaunchKernelGGL((inner_fold_kernel<TAIL>), dim3((unsigned)num_levels), dim3(kInnerBlock), 0, stream, slot,
                           tail);
    }
    return hipGetLastError();
}

// The slot of a host-partitioned phase, stored by a kernel (which also clears
// the level states at the start of an estimate).
static hipError_t inner_store(const LevelRange* ranges, int num_levels, int64_t n, const Law& x, const Law& y,
                              const TargetFunc& f, const IndexWeights& iw, const StreamKeys& keys, Moments* partials,
                              Moments* level_state, InnerSlot* slot, bool zero_state, uint32_t* next, bool* stride,
                              hipStream_t stream, KernelTimer* timer)
{
    InnerSlot host;
    host.multi = inner_base(n, x, y, f, iw, keys, num_levels, partials);
    *next = inner_partition(ranges, num_levels, n, keys.problem, host.multi, host.fold);
    host.fold.partials = partials;
    host.fold.level_state = level_state;
    host.arrivals = 0u;
    *stride = false;   // some level uses the stride coupling
    for (int i = 0; i < num_levels; ++i) *stride = *stride || ranges[i].stride != 0;
    ScopedTiming t(timer, 3);
    hipLaunchKernelGGL(inner_store_kernel, dim3(1), dim3(256), 0, stream, host, slot, zero_state ? level_state : nullptr,
                       num_levels);
    return hipGetLastError();
}

hipError_t inner_levels_run(const LevelRange* ranges, int num_levels, int64_t n, const Law& x, const Law& y,
                            const TargetFunc& f, const IndexWeights& iw, int prec, bool index_word32,
                            const StreamKeys& keys, Moments* partials, Moments* level_state, InnerSlot* slot,
                            bool zero_state, const InnerTelescope* tele, hipStream_t stream, KernelTimer* timer)
{
    uint32_t next = 0;
    bool stride = false;
    hipError_t e = inner_store(ranges, num_levels, n, x, y, f, iw, keys, partials, level_state, slot, zero_state, &next,
                               &stride, stream, timer);
    if (e != hipSuccess) return e;
    InnerTail tail = {};
    if (!tele)
        return inner_launch<0>(dim3(next > 0 ? next : 1), num_levels, x, y, f, iw, prec, stride, index_word32, n,
                               slot, tail, stream, timer);
    tail.out = tele->out;
    tail.level_means = tele->level_means;
    tail.level_var = tele->level_var;
    return inner_launch<2>(dim3(next > 0 ? next : 1), num_levels, x, y, f, iw, prec, stride, index_word32, n, slot,
                           tail, stream, timer);
}

hipError_t inner_target_run(const InnerScheduleInputs& s, const LevelRange* pilot, int num_levels, int64_t n,
                            const Law& x, const Law& y, const TargetFunc& f, const IndexWeights& iw, int prec,
                            bool index_word32, const StreamKeys& keys, Moments* partials, Moments* level_state,
                            InnerSlot* slot, const InnerTelescope& tele, hipStream_t stream, KernelTimer* timer)
{
    uint32_t next = 0;
    bool stride = false;
    hipError_t e = inner_store(pilot, num_levels, n, x, y, f, iw, keys, partials, level_state, slot, true, &next,
                               &stride, stream, timer);
    if (e != hipSuccess) return e;
    InnerTail tail = {};
    InnerScheduleParams& sp = tail.sched;
    sp.base = inner_base(n, x, y, f, iw, keys, num_levels, partials);
    sp.num_levels = num_levels;
    sp.eps = s.eps;
    sp.pilot = s.pilot;
    sp.max_total_draws = s.max_total_draws;
    sp.n = n;
    sp.problem = keys.problem;
    for (int l = 0; l < num_levels; ++l) {
        sp.c[l] = s.c[l];
        sp.level_field[l] = s.level_field[l];
        sp.stride[l] = s.stride[l];
    }
    sp.level_state = level_state;
    sp.slot = slot;
    sp.counts = s.counts;
    sp.status = s.status;
    sp.status_value = s.status_value;
    // the pilot, then its fold, which runs eq. (28) and writes the extension's slot
    e = inner_launch<1>(dim3(next > 0 ? next : 1), num_levels, x, y, f, iw, prec, stride, index_word32, n, slot,
                        tail, stream, timer);
    if (e != hipSuccess) return e;
    // the extension's partition is known on the device only: the largest
    // grid, whose workgroups past it leave at once; then the fold with the
    // telescoping sum
    InnerTail last = {};
    last.out = tele.out;
    last.level_means = tele.level_means;
    last.level_var = tele.level_var;
    return inner_launch<2>(dim3(kInnerMaxBlocks), num_levels, x, y, f, iw, prec, stride, index_word32, n, slot, last,
                           stream, timer);
}

size_t inner_slot_bytes() { return sizeof(InnerSlot); }

hipError_t inner_telescope(const Moments* level_state, int num_levels, double* out, double* level_means,
                           double* level_var, hipStream_t stream)
{
    hipLaunchKernelGGL(inner_telescope_kernel, dim3(1), dim3(64), 0, stream, level_state, num_levels, out,
                       level_means, level_var);
    return hipGetLastError();
}

}  // namespace mlmc
