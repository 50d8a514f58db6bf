// Inner-product level kernel (Sec. 2; Alg. 1 with m = p = 1, f = identity).
//
// A level sample of realisation k is
//   D_k = (n / c) * ( (1 - c / c_prev) * sum_{t < c_prev} x_{r_t} y_{r_t}
//                     + sum_{c_prev <= t < c} x_{r_t} y_{r_t} ),
// which is the fine sketch (eq. (1) with xi = 1/n over c draws) minus the
// coarse sketch over the first c_prev of the same draws; at level 0
// (c_prev = 0) it is the fine sketch alone.  Nothing is read from memory
// except reparameterised means/scales: indices and values are regenerated
// from the counter-based stream, so the kernel is bound by integer VALU work
// (Philox) and the roofline that matters is the VALU issue rate.
//
// Work mapping: a group of G lanes (a power of two <= 64) owns one
// realisation at a time; its lanes take draw pairs (2q, 2q+1), which share one
// Philox call of the index stream.  The group's partial sums meet in a
// butterfly of cross-lane shuffles, every lane of the group then holds D_k and
// updates its Welford state in FP64.  At the end the groups of a workgroup
// are combined by a fixed-order Chan tree in LDS and one Moments per
// workgroup goes to global memory; a single-workgroup kernel folds those into
// the level's running state, again in a fixed order.
#include "internal.hpp"

namespace mlmc {

struct InnerParams {
    uint32_t n, c, c_prev;
    uint32_t key0, key1, sid_index, sid_value;
    uint32_t k_begin, num_samples;
    uint32_t group_log2;
    double scale;   // n / c
    double omega;   // 1 - c / c_prev, weight of the first c_prev draws
    Law x, y;
    Moments* partials;
};

constexpr int kInnerBlock = 256;
constexpr int kInnerMaxBlocks = 4096;

template <typename T>
__device__ __forceinline__ void inner_draw_values(const InnerParams& prm, uint32_t k, uint32_t j,
                                                  bool normal, T& xv, T& yv)
{
    const Words4 w = philox4x32_10(0u, k, j, prm.sid_value, prm.key0, prm.key1);
    const T u0 = unit<T>(w.w0);
    const T u1 = unit<T>(w.w1);
    T z0 = (T)0, z1 = (T)0;
    if (normal) box_muller(u0, u1, z0, z1);
    xv = law_value<T>(prm.x, z0, u0, (int64_t)j);
    yv = law_value<T>(prm.y, z1, u1, (int64_t)j);
}

template <typename T>
__global__ __launch_bounds__(kInnerBlock) void inner_level_kernel(InnerParams prm)
{
    __shared__ Moments slots[kInnerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int G = 1 << prm.group_log2;
    const int lane_g = lane & (G - 1);
    const int groups_per_wave = kWave >> prm.group_log2;
    const int groups_per_block = (kInnerBlock / kWave) * groups_per_wave;
    const int slot = wave * groups_per_wave + (lane >> prm.group_log2);
    const int64_t stride = (int64_t)gridDim.x * groups_per_block;
    const uint32_t pairs = (prm.c + 1u) >> 1;
    const bool normal = prm.x.kind != 1 || prm.y.kind != 1;

    Moments st = {0.0, 0.0, 0.0};
    for (int64_t s = (int64_t)blockIdx.x * groups_per_block + slot;; s += stride) {
        // every lane of a wave runs the same number of iterations, so the
        // cross-lane shuffles below always see their whole group
        const bool active = s < (int64_t)prm.num_samples;
        if (!__any(active)) break;
        const uint32_t k = prm.k_begin + (uint32_t)(active ? s : 0);
        T acc_coarse = (T)0, acc_fine = (T)0;
        for (uint32_t q = lane_g; q < pairs; q += G) {
            uint32_t r0, r1;
            draw_index_pair(q, k, prm.sid_index, prm.key0, prm.key1, prm.n, r0, r1);
            const uint32_t t0 = 2u * q;
            T xv, yv;
            inner_draw_values<T>(prm, k, r0, normal, xv, yv);
            if (t0 < prm.c_prev) acc_coarse += xv * yv;
            else acc_fine += xv * yv;
            if (t0 + 1u < prm.c) {
                inner_draw_values<T>(prm, k, r1, normal, xv, yv);
                if (t0 + 1u < prm.c_prev) acc_coarse += xv * yv;
                else acc_fine += xv * yv;
            }
        }
        for (int off = G >> 1; off > 0; off >>= 1) {
            acc_coarse += __shfl_xor(acc_coarse, off, kWave);
            acc_fine += __shfl_xor(acc_fine, off, kWave);
        }
        if (active) {
            const double d = prm.scale * (prm.omega * (double)acc_coarse + (double)acc_fine);
            st.n += 1.0;
            const double delta = d - st.mean;
            st.mean += delta / st.n;
            st.m2 += delta * (d - st.mean);
        }
    }
    if (lane_g == 0) slots[slot] = st;
    __syncthreads();
    for (int half = groups_per_block >> 1; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) slots[threadIdx.x] = chan_merge(slots[threadIdx.x], slots[threadIdx.x + half]);
        __syncthreads();
    }
    if (threadIdx.x == 0) prm.partials[blockIdx.x] = slots[0];
}

// Folds `count` workgroup partials, then the level's earlier state, in a
// fixed order: thread i merges partials i, i + 256, ..., then a tree.
__global__ __launch_bounds__(kInnerBlock) void inner_fold_kernel(const Moments* partials, int count,
                                                                 Moments* level_state)
{
    __shared__ Moments slots[kInnerBlock];
    Moments st = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < count; i += kInnerBlock) st = chan_merge(st, partials[i]);
    slots[threadIdx.x] = st;
    __syncthreads();
    for (int half = kInnerBlock >> 1; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) slots[threadIdx.x] = chan_merge(slots[threadIdx.x], slots[threadIdx.x + half]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *level_state = chan_merge(*level_state, slots[0]);
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

static uint32_t group_log2_for(int64_t c)
{
    const int64_t pairs = (c + 1) / 2;
    uint32_t g = 0;
    while ((int64_t(1) << g) < pairs && g < 6) ++g;
    return g;
}

hipError_t inner_level_run(const LevelRange& lr, int64_t n, const Law& x, const Law& y, int prec,
                           const StreamKeys& keys, Moments* partials, Moments* level_state,
                           hipStream_t stream, KernelTimer* timer)
{
    if (lr.count <= 0) return hipSuccess;
    InnerParams prm;
    prm.n = (uint32_t)n;
    prm.c = (uint32_t)lr.c;
    prm.c_prev = (uint32_t)lr.c_prev;
    prm.key0 = keys.key0;
    prm.key1 = keys.key1;
    prm.sid_index = stream_id(kTagIndex, lr.level_field, keys.problem);
    prm.sid_value = stream_id(kTagValue, lr.level_field, keys.problem);
    prm.k_begin = (uint32_t)lr.k_begin;
    prm.num_samples = (uint32_t)lr.count;
    prm.group_log2 = group_log2_for(lr.c);
    prm.scale = (double)n / (double)lr.c;
    prm.omega = lr.c_prev > 0 ? 1.0 - (double)lr.c / (double)lr.c_prev : 0.0;
    prm.x = x;
    prm.y = y;
    prm.partials = partials;
    const int64_t groups_per_block = (kInnerBlock / kWave) * (kWave >> prm.group_log2);
    int64_t blocks = ceil_div(lr.count, groups_per_block);
    if (blocks > kInnerMaxBlocks) blocks = kInnerMaxBlocks;
    {
        ScopedTiming t(timer, 0);
        if (prec == 0)
            hipLaunchKernelGGL(inner_level_kernel<double>, dim3((unsigned)blocks), dim3(kInnerBlock), 0,
                               stream, prm);
        else
            hipLaunchKernelGGL(inner_level_kernel<float>, dim3((unsigned)blocks), dim3(kInnerBlock), 0,
                               stream, prm);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ScopedTiming t(timer, 2);
        hipLaunchKernelGGL(inner_fold_kernel, dim3(1), dim3(kInnerBlock), 0, stream,
                           (const Moments*)partials, (int)blocks, level_state + lr.level);
    }
    return hipGetLastError();
}

hipError_t inner_telescope(const Moments* level_state, int num_levels, double* out,
                           double* level_means, double* level_var, hipStream_t stream)
{
    hipLaunchKernelGGL(inner_telescope_kernel, dim3(1), dim3(64), 0, stream, level_state,
                       num_levels, out, level_means, level_var);
    return hipGetLastError();
}

}  // namespace mlmc
