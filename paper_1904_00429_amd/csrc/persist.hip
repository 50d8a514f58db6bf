// Single-launch form of a fixed-N_l matrix-product estimate over a table of
// products (Sec. 3, Alg. 1 per level): every level's passes run in one
// persistent kernel.  A pass is a batch of realisations of one level; step p
// of the launch gathers the sampled columns of pass p into one of three
// buffers and sketches pass p - 1 from another, so the VALU-bound generation
// of one pass overlaps the MFMA-bound contraction of the previous one, and the
// work of a step is claimed from queues rather than dealt by a grid:
//
//   * a step's work lists are the chunks of 16 gather units of pass p (a unit
//     is one wave's block of positions of one realisation of one product) and
//     the sketch tiles of pass p - 1 (a tile over the whole batch);
//   * each list is split into one contiguous queue per XCD (a product's tiles
//     stay together, so their operand rows are shared through that XCD's L2);
//     a workgroup drains the queue of its own XCD, then the others';
//   * between the two lists of step p a workgroup waits at barrier p - 1,
//     where every workgroup arrives after the sketch of step p - 1: every
//     thread releases its writes at agent scope, one thread per workgroup
//     arrives on the barrier's counter; the waiter polls it for the whole
//     grid, then acquires.  The grid never exceeds the workgroups the device
//     holds at once, and the wait is bounded: past its limit the launch raises
//     an error flag and every workgroup leaves.
//
// Sketches of consecutive passes of one level are in consecutive steps, each
// behind the barrier after the previous one, so their merges into the level
// state (the fused Chan merge of the sketch epilogue) keep the order of the
// launch-per-pass form; passes of different levels touch different state.
// The arithmetic is that of the launch-per-pass form (the same device
// functions on the same passes), so both give the same estimate.
#include "matmul_device.hpp"
#include "mlmc.h"

namespace mlmc {

constexpr int64_t kUnitsPerItem = 16;   // gather units per queue item

struct PersistParams {
    const ProblemDesc* descs;
    const int32_t* tile_owner;
    int64_t total_tiles;
    const PassDesc* passes;
    int32_t num_passes;
    int32_t elem;
    char* gbuf[3];               // gather buffer of pass p: gbuf[p % 3]
    int64_t sum_mp;
    double* level_mean;          // levels x sum_mp
    double* tile_acc;            // levels x total_tiles
    uint32_t key0, key1;
    uint32_t* sync;              // (num_passes + 1) steps x kPhaseWords, then the error flag
    int64_t timeout_ticks;       // wall-clock ticks a workgroup may wait at a barrier
};

// Sketch item `item` (an output tile over the whole batch) of pass `pass`.
template <typename P, int WR, int WC, int NBR, int NBC>
__device__ __attribute__((always_inline)) void sketch_of_pass(
    const PersistParams& prm, const PassDesc& d, int pass, int64_t item,
    typename SketchStage<P, WR, WC, NBR, NBC>::Buf& lds0, typename SketchStage<P, WR, WC, NBR, NBC>::Buf& lds1,
    double* red)
{
    SketchParams s = {};
    s.descs = prm.descs;
    s.tile_owner = prm.tile_owner;
    s.total_tiles = prm.total_tiles;
    s.groups = 1;
    s.kc = d.kc;
    s.kpad = d.kpad;
    s.batch = d.batch;
    s.elem = prm.elem;
    s.c = d.c;
    s.c_prev = d.c_prev;
    s.gbuf = prm.gbuf[pass % 3];
    s.sum_mp = prm.sum_mp;
    s.fuse = 1;
    s.done_before = d.done_before;
    s.level_mean = prm.level_mean + (int64_t)d.level * prm.sum_mp;
    s.tile_acc = prm.tile_acc + (int64_t)d.level * prm.total_tiles;
    // ragged tiles (tile 128 only): Welford
    if constexpr (NBR == 2) {
        if (d.stats == 0) {
            sketch_item<P, WR, WC, NBR, NBC, 0>(s, item, lds0, lds1, red);
            return;
        }
    }
    // BF16 and FP8 take the two-accumulator statistics for short realisations
    if constexpr (sizeof(typename P::In) <= 2) {
        if (d.stats == 3) {
            sketch_item<P, WR, WC, NBR, NBC, 3>(s, item, lds0, lds1, red);
            return;
        }
    }
    sketch_item<P, WR, WC, NBR, NBC, 2>(s, item, lds0, lds1, red);
}

// Gather item `item` of pass `pass`: kUnitsPerItem units, one wave each.
template <typename P, typename Compute, int WAVES, int LAWS, bool V16>
__device__ __attribute__((always_inline)) void gather_of_pass(const PersistParams& prm, const PassDesc& d, int pass,
                                                               int64_t item, int wave, int lane, uint32_t* cols,
                                                               Compute* colf)
{
    GatherParams g = {};
    g.descs = prm.descs;
    g.c = d.c;
    g.c_prev = d.c_prev;
    g.level_field = d.level_field;
    g.kc = d.kc;
    g.kpad = d.kpad;
    g.batch = d.batch;
    g.octets = d.octets;
    g.omega = d.omega;
    g.stride = d.stride;
    g.key0 = prm.key0;
    g.key1 = prm.key1;
    g.k_first = d.k_first;
    g.elem = prm.elem;
    g.gbuf = prm.gbuf[pass % 3];
    const int64_t units = d.units, gx = d.gx, per_prob = d.gx * d.batch;
    const int64_t u0 = item * kUnitsPerItem;
    const int64_t u1 = u0 + kUnitsPerItem < units ? u0 + kUnitsPerItem : units;
    for (int64_t u = u0 + wave; u < u1; u += WAVES) {
        const int64_t bz = u / per_prob, r = u - bz * per_prob;
        const int64_t by = r / gx, bx = r - by * gx;
        gather_unit<Compute, typename P::In, P::KPACK, LAWS, V16>(g, (uint32_t)bx, (uint32_t)by, (uint32_t)bz, lane,
                                                                  kWave, cols, colf);
    }
}

// Claims the items [0, n) of one work list from its per-XCD queues (counters
// at `counters`, kSyncStride apart) and runs `work` on each: the queue of the
// workgroup's own XCD first, then the others'.
template <typename Work>
__device__ __attribute__((always_inline)) void drain_queues(uint32_t* counters, int64_t n, int home,
                                                             int64_t* claimed, Work&& work)
{
    for (int qi = 0; qi < kXcds; ++qi) {
        const int q = (home + qi) % kXcds;
        const int64_t first = n * q / kXcds, len = n * (q + 1) / kXcds - first;
        if (len == 0) continue;
        for (;;) {
            if (threadIdx.x == 0)
                *claimed = (int64_t)__hip_atomic_fetch_add(counters + q * kSyncStride, 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const int64_t i = *claimed;
            __syncthreads();
            if (i >= len) break;
            work(first + i);
        }
    }
}

template <typename P, typename Compute, int WR, int WC, int NBR, int NBC, int WPE, int LAWS, bool V16>
__global__ __launch_bounds__(kWave * WR * WC, WPE) void persistent_kernel(PersistParams prm)
{
    using St = SketchStage<P, WR, WC, NBR, NBC>;
    constexpr int WAVES = WR * WC;
    __shared__ __align__(16) typename St::Buf lds0;
    __shared__ __align__(16) typename St::Buf lds1;
    __shared__ double red[WAVES];
    __shared__ uint32_t cols[WAVES][kGatherMaxPos];
    __shared__ Compute colf[WAVES][kGatherMaxPos];
    __shared__ int64_t claimed;
    __shared__ int phase_ok;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int home = (int)(blockIdx.x % kXcds);    // workgroups are dealt to the XCDs round-robin
    uint32_t* const error = prm.sync + (int64_t)(prm.num_passes + 1) * kPhaseWords;

    // Step ph: gather pass ph; wait at barrier ph - 1; sketch pass ph - 1;
    // arrive at barrier ph.  The gather of pass ph overwrites the buffer that
    // the sketch of pass ph - 3 read, which every workgroup finished before
    // arriving at barrier ph - 2, and this workgroup waited there in step
    // ph - 1: so a workgroup gathers as soon as it has sketched, and the wait
    // for the slowest workgroup of a barrier overlaps the next gather.
    for (int ph = 0; ph <= prm.num_passes; ++ph) {
        uint32_t* const words = prm.sync + (int64_t)ph * kPhaseWords;
        if (ph < prm.num_passes)
            drain_queues(words + kXcds * kSyncStride, ceil_div(prm.passes[ph].units, kUnitsPerItem), home, &claimed,
                         [&](int64_t item) {
                             gather_of_pass<P, Compute, WAVES, LAWS, V16>(prm, prm.passes[ph], ph, item, wave, lane,
                                                                          cols[wave], colf[wave]);
                         });
        if (ph > 0) {
            // barrier ph - 1: the gather of pass ph - 1 and the sketch of
            // pass ph - 2 (the level state this one merges into) are done
            if (threadIdx.x == 0) {
                const uint32_t* const arrive = words - kPhaseWords + 2 * kXcds * kSyncStride;
                const int64_t t0 = wall_clock64();
                int ok = 1;
                while (__hip_atomic_load(arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
                    if (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                        wall_clock64() - t0 > prm.timeout_ticks) {
                        __hip_atomic_store(error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                phase_ok = ok;
            }
            __syncthreads();
            if (!phase_ok) return;
            drain_queues(words, prm.total_tiles, home, &claimed, [&](int64_t item) {
                sketch_of_pass<P, WR, WC, NBR, NBC>(prm, prm.passes[ph - 1], ph - 1, item, lds0, lds1, red);
            });
        }
        // arrive at barrier ph (the last one has no waiter: the launch's end
        // orders the finalisation after it)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(words + 2 * kXcds * kSyncStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

namespace {

// Workgroups the device holds at once for `kernel` (all of them take part in
// every barrier), or 0 when the query fails.
template <typename K>
int64_t resident_capacity(K kernel, int threads)
{
    int device = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&device) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), threads, 0) !=
        hipSuccess)
        return 0;
    return (int64_t)cus * per_cu;
}

template <typename P, typename Compute, int WR, int WC, int NBR, int NBC, int WPE, int LAWS, bool V16>
hipError_t launch_persistent(const MatmulPlan& plan, const StreamKeys& keys, char* ws, hipStream_t stream)
{
    auto kernel = persistent_kernel<P, Compute, WR, WC, NBR, NBC, WPE, LAWS, V16>;
    constexpr int threads = kWave * WR * WC;
    int64_t grid = resident_capacity(kernel, threads);
    if (grid < kXcds) return hipErrorInvalidConfiguration;
    grid -= grid % kXcds;
    int device = 0, rate_khz = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device);
    if (e != hipSuccess) return e;
    PersistParams prm;
    prm.descs = reinterpret_cast<const ProblemDesc*>(ws + plan.off_desc);
    prm.tile_owner = reinterpret_cast<const int32_t*>(ws + plan.off_tile_owner);
    prm.total_tiles = plan.total_tiles;
    prm.passes = reinterpret_cast<const PassDesc*>(ws + plan.off_passes);
    prm.num_passes = (int32_t)plan.passes.size();
    prm.elem = plan.elem;
    prm.gbuf[0] = ws + plan.off_gather;
    prm.gbuf[1] = ws + plan.off_gather2;
    prm.gbuf[2] = ws + plan.off_gather3;
    prm.sum_mp = plan.sum_mp;
    prm.level_mean = reinterpret_cast<double*>(ws + plan.off_means);
    prm.tile_acc = reinterpret_cast<double*>(ws + plan.off_tile_acc);
    prm.key0 = keys.key0;
    prm.key1 = keys.key1;
    prm.sync = reinterpret_cast<uint32_t*>(ws + plan.off_sync);
    // a step lasts milliseconds; ten seconds means some workgroup never ran
    prm.timeout_ticks = (int64_t)rate_khz * 1000 * 10;
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), 0, stream, prm);
    return hipGetLastError();
}

template <typename P, typename Compute, int WR, int WC, int NBR, int NBC, int WPE>
hipError_t launch_laws(const MatmulPlan& plan, const StreamKeys& keys, char* ws, hipStream_t stream)
{
    const bool normal = plan.laws == kLawsNormal;
    if (plan.value16)
        return normal ? launch_persistent<P, Compute, WR, WC, NBR, NBC, WPE, kLawsNormal, true>(plan, keys, ws, stream)
                      : launch_persistent<P, Compute, WR, WC, NBR, NBC, WPE, kLawsUniform, true>(plan, keys, ws, stream);
    return normal ? launch_persistent<P, Compute, WR, WC, NBR, NBC, WPE, kLawsNormal, false>(plan, keys, ws, stream)
                  : launch_persistent<P, Compute, WR, WC, NBR, NBC, WPE, kLawsUniform, false>(plan, keys, ws, stream);
}

}  // namespace

hipError_t matmul_persistent_run(const MatmulPlan& plan, const StreamKeys& keys, char* ws, hipStream_t stream,
                                 KernelTimer* timer)
{
    if (!plan.persistent) return hipErrorInvalidValue;
    hipError_t e;
    {
        // the claim and arrival counters of every step and the error flag start at zero
        ScopedTiming t(timer, MLMC_KERNEL_FINAL);
        e = fill_doubles(reinterpret_cast<double*>(ws + plan.off_sync), ceil_div(plan.sync_words, 2), 0.0, stream);
    }
    if (e != hipSuccess) return e;
    ScopedTiming t(timer, MLMC_KERNEL_SAMPLE);
    // the workgroup shapes of the launch-per-pass form: tile 64 is 2 x 2 waves
    // of one MFMA block, tile 128 2 x 2 waves of 2 x 2 blocks; the gather and
    // the sketch share one register allocation, which fits three waves per
    // SIMD at tile 64 (measured faster than four, where more of it spills)
    // and two at tile 128
    switch (plan.prec) {
    case 1:
        return plan.tile == 128 ? launch_laws<PolicyF32, float, 2, 2, 2, 2, 2>(plan, keys, ws, stream)
                                : launch_laws<PolicyF32, float, 2, 2, 1, 1, 3>(plan, keys, ws, stream);
    case 2:
        return plan.tile == 128 ? launch_laws<PolicyBF16, float, 2, 2, 2, 2, 2>(plan, keys, ws, stream)
                                : launch_laws<PolicyBF16, float, 2, 2, 1, 1, 3>(plan, keys, ws, stream);
    case 3:
        return plan.tile == 128 ? launch_laws<PolicyFP8, float, 2, 2, 2, 2, 2>(plan, keys, ws, stream)
                                : launch_laws<PolicyFP8, float, 2, 2, 1, 1, 3>(plan, keys, ws, stream);
    default:
        return hipErrorInvalidValue;   // FP64 keeps the launch-per-pass form
    }
}

hipError_t matmul_persistent_status(const MatmulPlan& plan, char* ws, hipStream_t stream, bool* failed)
{
    *failed = false;
    if (!plan.persistent) return hipSuccess;
    uint32_t flag = 0;
    const uint32_t* dev = reinterpret_cast<const uint32_t*>(ws + plan.off_sync) +
                          (int64_t)(plan.passes.size() + 1) * kPhaseWords;
    hipError_t e = hipMemcpyAsync(&flag, dev, sizeof(flag), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    *failed = flag != 0u;
    return e;
}

}  // namespace mlmc
