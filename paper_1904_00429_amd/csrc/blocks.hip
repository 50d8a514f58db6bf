// Building blocks exported for testing: raw Philox words, the index draws and
// the sampled columns exactly as the estimators produce them.
#include <hip/hip_bf16.h>

#include "internal.hpp"

namespace mlmc {

__global__ void philox_batch_kernel(int64_t count, const uint32_t* ctr, uint32_t key0, uint32_t key1,
                                    uint32_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const Words4 w = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key0, key1);
    out[4 * i] = w.w0;
    out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2;
    out[4 * i + 3] = w.w3;
}

__global__ void sample_indices_kernel(uint32_t key0, uint32_t key1, uint32_t sid_index, uint32_t k0,
                                      int64_t num_samples, int64_t c, uint32_t n, int32_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pairs = (c + 1) / 2;
    if (i >= num_samples * pairs) return;
    const int64_t s = i / pairs;
    const uint32_t q = (uint32_t)(i % pairs);
    uint32_t r0, r1;
    draw_index_pair(q, k0 + (uint32_t)s, sid_index, key0, key1, n, r0, r1);
    out[s * c + 2 * q] = (int32_t)r0;
    if (2 * (int64_t)q + 1 < c) out[s * c + 2 * q + 1] = (int32_t)r1;
}

// cum[j] = w_0 + ... + w_j: each thread sums a contiguous segment, a scan of
// the segment sums in LDS, then each thread writes its segment's running sums
// (exact integer arithmetic: the order does not matter).
constexpr int kCumThreads = 1024;

__global__ __launch_bounds__(kCumThreads) void cumulative_kernel(const uint32_t* w, int64_t n, uint64_t* cum)
{
    __shared__ uint64_t part[kCumThreads];
    const int64_t per = (n + kCumThreads - 1) / kCumThreads;
    const int64_t b = (int64_t)threadIdx.x * per;
    const int64_t e = b + per < n ? b + per : n;
    uint64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += w[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kCumThreads; off <<= 1) {
        const uint64_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    for (int64_t i = b; i < e; ++i) {
        run += w[i];
        cum[i] = run;
    }
}

__global__ void sample_indices_weighted_kernel(uint32_t key0, uint32_t key1, uint32_t sid_index, uint32_t k0,
                                               int64_t num_samples, int64_t c, uint32_t n, const uint64_t* cum,
                                               int32_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pairs = (c + 1) / 2;
    if (i >= num_samples * pairs) return;
    const int64_t s = i / pairs;
    const uint32_t q = (uint32_t)(i % pairs);
    const uint64_t total = cum[n - 1];
    const Words4 w = philox4x32_10(q, k0 + (uint32_t)s, 0u, sid_index, key0, key1);
    out[s * c + 2 * q] = (int32_t)index_from_cumulative(w.w0, w.w1, cum, n, total);
    if (2 * (int64_t)q + 1 < c) out[s * c + 2 * q + 1] = (int32_t)index_from_cumulative(w.w2, w.w3, cum, n, total);
}

// Theorem 3.1's xi**: s_j = sqrt(EA_j) sqrt(EB_j), EA_j = sum_i (mean_ij^2 +
// stdev_ij^2) accumulated in FP64 for i = 0, 1, ... (the mean's square first;
// the squares of FP32 values are exact in FP64, so fused and separate
// multiply-adds agree), likewise EB_j over row j of B.
__global__ void column_moments_kernel(int64_t m, int64_t n, int64_t p, Law A, Law B, double* s)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double ea = 0.0, eb = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        const double mu = (double)A.mean[j * A.ld + i], sd = (double)A.stdev[j * A.ld + i];
        ea = ea + mu * mu;
        ea = ea + sd * sd;
    }
    for (int64_t q = 0; q < p; ++q) {
        const double mu = (double)B.mean[j * B.ld + q], sd = (double)B.stdev[j * B.ld + q];
        eb = eb + mu * mu;
        eb = eb + sd * sd;
    }
    s[j] = sqrt(ea) * sqrt(eb);
}

__global__ __launch_bounds__(256) void max_kernel(const double* s, int64_t n, double* out)
{
    __shared__ double red[256];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) v = s[i] > v ? s[i] : v;
    red[threadIdx.x] = v;
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half && red[threadIdx.x + half] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// w_j = max(1, floor(2^24 s_j / max s)); uniform laws (s == NULL): 2^24
__global__ void quantise_weights_kernel(const double* s, const double* smax, int64_t n, uint32_t* w)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (!s) {
        w[j] = 1u << 24;
        return;
    }
    const double mx = *smax;
    const double v = mx > 0.0 ? floor(s[j] / mx * 16777216.0) : 1.0;
    w[j] = v < 1.0 ? 1u : (uint32_t)v;
}

template <typename Compute, bool ROUND_BF16>
__global__ void gather_f64_kernel(int64_t m, int64_t p, uint32_t n, Law A, Law B, uint32_t key0,
                                  uint32_t key1, uint32_t sid_index, uint32_t sid_value, uint32_t k0,
                                  int64_t num_samples, int64_t c, double* AS, double* BS)
{
    const int64_t quads = ceil_div(m + p, 4);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= num_samples * c * quads) return;
    const int64_t q = i % quads;
    const int64_t t = (i / quads) % c;
    const int64_t s = i / (quads * c);
    const uint32_t k = k0 + (uint32_t)s;
    const uint32_t j = draw_index((uint32_t)t, k, sid_index, key0, key1, n);
    if (A.kind >= kLawExperimentFirst) {
        // the laws of Sec. 4 (both operands): one experiment-stream call per element
        const uint32_t sid_exp = (sid_value & 0x0FFFFFFFu) | (kTagExperiment << 28);
        for (int r = 0; r < 4; ++r) {
            const int64_t e = 4 * q + r;
            if (e >= m + p) break;
            const Law& L = e < m ? A : B;
            const Compute v = (Compute)experiment_value(L.kind, L.loc, L.scale, L.aux, (uint32_t)e, k, j, sid_exp,
                                                        key0, key1);
            double out = (double)v;
            if (ROUND_BF16) out = (double)(float)(__bf16)(float)v;
            if (e < m) AS[(s * c + t) * m + e] = out;
            else BS[(s * c + t) * p + (e - m)] = out;
        }
        return;
    }
    const Words4 w = philox4x32_10((uint32_t)q, k, j, sid_value, key0, key1);
    const bool normal = A.kind != 1 || B.kind != 1;
    Compute u[4], z[4];
    quad_values<Compute>(w, normal, u[0], u[1], u[2], u[3], z[0], z[1], z[2], z[3]);
    for (int r = 0; r < 4; ++r) {
        const int64_t e = 4 * q + r;
        if (e >= m + p) break;
        Compute v;
        if (e < m) v = law_value<Compute>(A, z[r], u[r], (int64_t)j * A.ld + e);
        else v = law_value<Compute>(B, z[r], u[r], (int64_t)j * B.ld + (e - m));
        double out = (double)v;
        if (ROUND_BF16) out = (double)(float)(__bf16)(float)v;
        if (e < m) AS[(s * c + t) * m + e] = out;
        else BS[(s * c + t) * p + (e - m)] = out;
    }
}

hipError_t philox_batch(int64_t count, const uint32_t* ctr, uint32_t key0, uint32_t key1, uint32_t* out,
                        hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_batch_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, stream, count,
                       ctr, key0, key1, out);
    return hipGetLastError();
}

hipError_t sample_indices(const StreamKeys& keys, uint32_t level_field, uint32_t k0, int64_t num_samples,
                          int64_t c, int64_t n, int32_t* out, hipStream_t stream)
{
    const int64_t work = num_samples * ((c + 1) / 2);
    if (work <= 0) return hipSuccess;
    hipLaunchKernelGGL(sample_indices_kernel, dim3((unsigned)ceil_div(work, 256)), dim3(256), 0, stream,
                       keys.key0, keys.key1, stream_id(kTagIndex, level_field, keys.problem), k0, num_samples, c,
                       (uint32_t)n, out);
    return hipGetLastError();
}

hipError_t build_cumulative(const uint32_t* w, int64_t n, uint64_t* cum, hipStream_t stream)
{
    hipLaunchKernelGGL(cumulative_kernel, dim3(1), dim3(kCumThreads), 0, stream, w, n, cum);
    return hipGetLastError();
}

hipError_t sample_indices_weighted(const StreamKeys& keys, uint32_t level_field, uint32_t k0, int64_t num_samples,
                                   int64_t c, int64_t n, const uint64_t* cum, int32_t* out, hipStream_t stream)
{
    const int64_t work = num_samples * ((c + 1) / 2);
    if (work <= 0) return hipSuccess;
    hipLaunchKernelGGL(sample_indices_weighted_kernel, dim3((unsigned)ceil_div(work, 256)), dim3(256), 0, stream,
                       keys.key0, keys.key1, stream_id(kTagIndex, level_field, keys.problem), k0, num_samples, c,
                       (uint32_t)n, cum, out);
    return hipGetLastError();
}

hipError_t optimal_weights(int64_t m, int64_t n, int64_t p, const Law& A, const Law& B, uint32_t* w,
                           double* scratch, hipStream_t stream)
{
    const dim3 grid((unsigned)ceil_div(n, 256));
    if (A.kind >= kLawExperimentFirst || B.kind >= kLawExperimentFirst) return hipErrorInvalidValue;
    if (A.kind != 2 || B.kind != 2) {
        hipLaunchKernelGGL(quantise_weights_kernel, grid, dim3(256), 0, stream, nullptr, nullptr, n, w);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(column_moments_kernel, grid, dim3(256), 0, stream, m, n, p, A, B, scratch);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, stream, scratch, n, scratch + n);
    hipLaunchKernelGGL(quantise_weights_kernel, grid, dim3(256), 0, stream, scratch, scratch + n, n, w);
    return hipGetLastError();
}

hipError_t gather_columns_f64(int64_t m, int64_t n, int64_t p, const Law& A, const Law& B,
                              const StreamKeys& keys, uint32_t level_field, uint32_t k0, int64_t num_samples,
                              int64_t c, int prec, double* AS, double* BS, hipStream_t stream)
{
    const int64_t work = num_samples * c * ceil_div(m + p, 4);
    if (work <= 0) return hipSuccess;
    if ((A.kind >= kLawExperimentFirst) != (B.kind >= kLawExperimentFirst)) return hipErrorInvalidValue;
    const uint32_t si = stream_id(kTagIndex, level_field, keys.problem);
    const uint32_t sv = stream_id(kTagValue, level_field, keys.problem);
    const dim3 grid((unsigned)ceil_div(work, 256));
    if (prec == 0)
        hipLaunchKernelGGL((gather_f64_kernel<double, false>), grid, dim3(256), 0, stream, m, p, (uint32_t)n, A, B,
                           keys.key0, keys.key1, si, sv, k0, num_samples, c, AS, BS);
    else if (prec == 1)
        hipLaunchKernelGGL((gather_f64_kernel<float, false>), grid, dim3(256), 0, stream, m, p, (uint32_t)n, A, B,
                           keys.key0, keys.key1, si, sv, k0, num_samples, c, AS, BS);
    else
        hipLaunchKernelGGL((gather_f64_kernel<float, true>), grid, dim3(256), 0, stream, m, p, (uint32_t)n, A, B,
                           keys.key0, keys.key1, si, sv, k0, num_samples, c, AS, BS);
    return hipGetLastError();
}

}  // namespace mlmc
