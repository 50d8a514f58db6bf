// Adjoint of the matrix estimator for reparameterised laws
//   A = M_A + S_A o Z,  B = M_B + S_B o W  (Z, W standard normal, entrywise).
//
// The estimate is Y = sum_l (1/N_l) sum_k D_{l,k} with
// D_{l,k} = (n / c_l) sum_t w_t a_t b_t^T (w_t = 1 - c_l / c_{l-1} for the c_{l-1}
// coarse draws, 1 otherwise; Alg. 1 with the prefix coupling, the first
// c_{l-1} draws, or the stride coupling, draws M - 1, 2M - 1, ...).  Y is bilinear
// in (a_t, b_t), so for an upstream gradient G = dL/dY (m x p)
//   dL/da_t = kappa_t G b_t,   dL/db_t = kappa_t G^T a_t,   kappa_t = (n / c_l) w_t / N_l,
// and the chain rule through a_t = M_A[:, r_t] + S_A[:, r_t] o z_t gives
//   dM_A[:, r_t] += dL/da_t,  dS_A[:, r_t] += dL/da_t o z_t   (likewise for B).
// Nothing of the forward pass is stored: the indices and normals of every
// realisation are regenerated from the counter-based stream, exactly as the
// forward drew them, and the sampled columns are regenerated from M and S.
//
// Every draw adds into the gradient column of its index, and many draws hit
// the same column (a few per column and level at the differentiation
// workload's sizes, thousands with a skewed index law).  The draws of a pass
// (a batch of realisations of one level) are therefore put in column order
// first, and each column's sum is formed in that order by one owner; nothing
// is added atomically, so the gradients are the same bits on every run.
//
// Per pass (E = S c_l draws, flat draw number e = s c_l + t):
//   adj_keys:     the column r of every draw, drawn as the forward drew it;
//   adj_radix_*:  a stable LSD radix sort of the draw numbers by column
//                 (8-bit digits: histogram, scan, scatter), so the draws of
//                 one column are adjacent and in draw order;
//   adj_gather:   in sorted order, each draw's regenerated a_t and b_t
//                 (position-major rows, FP32 or BF16), its normals and kappa_t;
//   adj_tile:     U^T = B_S G^T (E x m) and V = A_S^T G (E x p) on MFMA, one
//                 workgroup per 64 sorted draws x 128 gradient columns; the
//                 rows scaled by kappa_t (dM), and also by the normal (dS), are
//                 summed down each column segment in LDS; a segment inside the
//                 tile is added to its gradient row by a plain read-modify-
//                 write, a segment that crosses the tile's edge leaves its
//                 partial sum in a carry slot;
//   adj_fixup:    each crossing segment's partials, summed in tile order and
//                 added once.
#include <type_traits>

#include "internal.hpp"

namespace mlmc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kAdjThreads = 256;
constexpr int kAdjRows = 64;              // sorted draws per tile
constexpr int kAdjCols = 128;             // gradient columns per tile
constexpr int64_t kAdjBudget = 4ll << 30;    // pass buffers at most
constexpr uint32_t kNoKey = 0xFFFFFFFFu;  // past the ends of the sorted list (n < 2^32)

constexpr int kSortThreads = 256;         // one thread per digit value
constexpr int kSortItems = 16;
constexpr int kSortBlock = kSortThreads * kSortItems;
constexpr int kSortScanThreads = 1024;

static int64_t round_up_adj(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Draw t is one of the coarse draws of its level sample.
__device__ __forceinline__ bool coarse_draw(uint32_t t, uint32_t c_prev, uint32_t stride)
{
    return stride ? (t + 1u) % stride == 0u : t < c_prev;
}

// ---- the draws of a pass ------------------------------------------------------
// The draws of every level are numbered in one sequence (level by level,
// realisation by realisation, t = 0 .. c_l - 1); a pass takes a contiguous
// range of it, so that a pass may hold whole levels or parts of several.
constexpr int kAdjMaxLevels = 32;

struct AdjLevelTable {
    int32_t nlev;
    int64_t first[kAdjMaxLevels + 1];     // number of each level's first draw; first[nlev]: all draws
    uint32_t c[kAdjMaxLevels], c_prev[kAdjMaxLevels], stride[kAdjMaxLevels];
    uint32_t sid_index[kAdjMaxLevels], sid_value[kAdjMaxLevels];
    float kappa_coarse[kAdjMaxLevels], kappa_fine[kAdjMaxLevels];
};

struct AdjDraw {
    int l;
    uint32_t k, t;                        // realisation and position in it
};

__device__ __forceinline__ AdjDraw adj_draw(const AdjLevelTable& lt, int64_t g)
{
    int l = 0;
    while (l + 1 < lt.nlev && g >= lt.first[l + 1]) ++l;
    const int64_t r = g - lt.first[l];
    AdjDraw d;
    d.l = l;
    d.k = (uint32_t)(r / lt.c[l]);
    d.t = (uint32_t)(r % lt.c[l]);
    return d;
}

struct AdjKeyParams {
    AdjLevelTable lt;
    int64_t g0, E;                        // the pass: draws g0 .. g0 + E - 1
    uint32_t n;
    uint32_t key0, key1;
    const uint64_t* cum;                  // cumulative index weights (NULL: uniform draws)
    uint32_t* keys;
    uint32_t* vals;
};

__global__ __launch_bounds__(256) void adj_keys_kernel(AdjKeyParams prm)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= prm.E) return;
    const AdjDraw d = adj_draw(prm.lt, prm.g0 + e);
    const uint32_t sid = prm.lt.sid_index[d.l];
    prm.keys[e] = prm.cum ? draw_index_weighted(d.t, d.k, sid, prm.key0, prm.key1, prm.cum, prm.n, prm.cum[prm.n - 1])
                          : draw_index(d.t, d.k, sid, prm.key0, prm.key1, prm.n);
    prm.vals[e] = (uint32_t)e;
}

// ---- stable LSD radix sort by column (8-bit digits) ---------------------------
// counts[d * nb + b]: draws of block b whose digit is d (integer LDS atomics:
// the counts do not depend on their order).
__global__ __launch_bounds__(kSortThreads) void adj_radix_hist_kernel(const uint32_t* keys, int64_t E, int shift,
                                                                       uint32_t* counts, int64_t nb)
{
    __shared__ uint32_t h[kSortThreads];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t e = base + (int64_t)i * kSortThreads + threadIdx.x;
        if (e < E) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Exclusive prefix sum of the digit-major counts, in place (one workgroup):
// each wave takes a contiguous segment, sums it (coalesced), the waves'
// totals give each segment's offset, and the wave scans its segment 64
// entries at a time with lane shuffles.
__global__ __launch_bounds__(kSortScanThreads) void adj_radix_scan_kernel(uint32_t* counts, int64_t len)
{
    constexpr int W = kSortScanThreads / kWave;
    __shared__ uint32_t wsum[W];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t per = (len + W - 1) / W;
    const int64_t b = (int64_t)wave * per;
    const int64_t e = b + per < len ? b + per : len;
    uint32_t s = 0u;
    for (int64_t i = b + lane; i < e; i += kWave) s += counts[i];
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) wsum[wave] = s;
    __syncthreads();
    uint32_t run = 0u;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (int64_t base = b; base < e; base += kWave) {
        const int64_t i = base + lane;
        const uint32_t c = i < e ? counts[i] : 0u;
        uint32_t x = c;                                    // inclusive scan over the 64 entries
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (i < e) counts[i] = run + x - c;
        run += __shfl(x, kWave - 1);
    }
}

// Block b places its draws, in their order, after every draw of a smaller
// digit and after the draws of the same digit in blocks before b.  Inside the
// block the draws go in rounds of 256 (round-major, then thread order, which
// is their order): a wave finds the lanes that share its digit with eight
// ballots, and the waves' counts per digit, kept in LDS, order the waves.
__global__ __launch_bounds__(kSortThreads) void adj_radix_scatter_kernel(const uint32_t* kin, const uint32_t* vin,
                                                                          uint32_t* kout, uint32_t* vout, int64_t E,
                                                                          int shift, const uint32_t* offsets,
                                                                          int64_t nb)
{
    constexpr int W = kSortThreads / kWave;
    __shared__ uint32_t run[kSortThreads];
    __shared__ uint32_t wcnt[W][kSortThreads];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    run[threadIdx.x] = offsets[(int64_t)threadIdx.x * nb + blockIdx.x];
    for (int w = 0; w < W; ++w) wcnt[w][threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t e = base + (int64_t)i * kSortThreads + threadIdx.x;
        const bool ok = e < E;
        uint32_t key = 0u, val = 0u, d = 0u;
        if (ok) {
            key = kin[e];
            val = vin[e];
            d = (key >> shift) & 255u;
        }
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (ok && rank == 0u) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (ok) {
            uint32_t pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t tot = 0u;
        for (int w = 0; w < W; ++w) {
            tot += wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = 0u;
        }
        run[threadIdx.x] += tot;
        __syncthreads();
    }
}

// ---- regeneration of the sampled columns, in sorted order --------------------
// The contraction's t operand is stored tile-blocked, so that each K-chunk
// of a tile is one contiguous block that the tile kernel copies straight into
// LDS: FP32 values at [tile][k][row] (k < Kc, row < 64), BF16 at
// [tile][k / 8][row][k % 8]; Kc is K rounded up to kAdjKc, and the rows past
// K and the draws past the end of the last tile hold zeros.  The normals stay
// position-major ([draw][row], row stride m or p rounded up to 8): the
// epilogue reads them along the gradient columns.
constexpr int kAdjKc = 128;               // four chunks of either precision

struct AdjGatherParams {
    AdjLevelTable lt;
    int64_t m, p, g0, E;
    int64_t kca, kcb;             // K of the two operand blocks: m and p rounded up to kAdjKc
    uint32_t n;
    uint32_t key0, key1;
    Law A, B;
    const uint32_t* keys;         // sorted columns
    const uint32_t* vals;         // sorted draw numbers (within the pass)
    const uint32_t* iw;           // index weights (NULL: uniform): kappa_t also times 1 / (n xi_j)
    const uint64_t* cum;
    void* VA;                     // tiles x kca x 64: values of a_t (FP32, or BF16 in the same region)
    void* VB;                     // tiles x kcb x 64: values of b_t
    float* kap;                   // E
    uint2* info;                  // E: (realisation, value stream) of each sorted draw
    bool value16;                 // the forward's values came from 16-bit uniforms
};

// Uniforms and normals of rows 4q .. 4q+3 of [a; b] for draw column j of
// realisation k, as the forward generated them.
__device__ __forceinline__ void adj_quad(bool value16, uint32_t q, uint32_t k, uint32_t j, uint32_t sid, uint32_t key0,
                                         uint32_t key1, float (&u)[4], float (&z)[4])
{
    if (value16) {
        // rows 4q .. 4q+3 are halves of words 2 (q & 1) and 2 (q & 1) + 1
        // of the call for rows 8 (q / 2) .. 8 (q / 2) + 7
        const Words4 w = philox4x32_10(q >> 1, k, j, sid, key0, key1);
        const uint32_t a = (q & 1u) ? w.w2 : w.w0, b = (q & 1u) ? w.w3 : w.w1;
        u[0] = unit16<float>(a & 0xFFFFu);
        u[1] = unit16<float>(a >> 16);
        u[2] = unit16<float>(b & 0xFFFFu);
        u[3] = unit16<float>(b >> 16);
        box_muller(u[0], u[1], z[0], z[1]);
        box_muller(u[2], u[3], z[2], z[3]);
    } else {
        const Words4 w = philox4x32_10(q, k, j, sid, key0, key1);
        quad_values<float>(w, true, u[0], u[1], u[2], u[3], z[0], z[1], z[2], z[3]);
    }
}

// Element (k, row) of a tile block of K-extent kc.
__device__ __forceinline__ int64_t adj_blk_f32(int64_t T, int64_t kc, int64_t k, int row)
{
    return (T * kc + k) * kAdjRows + row;
}
__device__ __forceinline__ int64_t adj_blk_bf16(int64_t T, int64_t kc, int64_t k, int row)
{
    return ((T * (kc / 8) + k / 8) * kAdjRows + row) * 8 + (k % 8);
}

// One workgroup per tile of 64 sorted draws.  The rows of each operand are
// taken in blocks of 64 (k0 .. k0 + 63 of a or of b, up to the padded K): for
// a block, every (Philox quad of rows, group of four draws) pair generates
// its values and normals, the normals go straight to global memory
// (position-major, a quad's four rows adjacent) and the values into an LDS
// tile [row][draw]; the tile is then written out in the blocked layout with
// whole 16-byte vectors (FP32: a row's 64 draws, 256 bytes; BF16: eight
// rows of one draw).  Rows past K and draws past the pass hold zeros.
constexpr int kAdjGatherBlock = 64;

template <bool BF16>
__global__ __launch_bounds__(kAdjThreads) void adj_gather_kernel(AdjGatherParams prm)
{
    __shared__ uint32_t cols[kAdjRows];
    __shared__ uint32_t reals[kAdjRows];
    __shared__ uint32_t sids[kAdjRows];
    __shared__ __align__(16) float tile[kAdjGatherBlock][kAdjRows];   // [row of the block][draw]
    const int64_t T = blockIdx.x;
    const int64_t e_first = T * kAdjRows;
    const int64_t left = prm.E - e_first;
    const int nvalid = left < kAdjRows ? (int)left : kAdjRows;
    if (threadIdx.x < kAdjRows) {
        const int64_t e = e_first + threadIdx.x;
        uint32_t j = 0u, k = 0u, sid = 0u;
        if ((int)threadIdx.x < nvalid) {
            const AdjDraw d = adj_draw(prm.lt, prm.g0 + prm.vals[e]);
            j = prm.keys[e];
            k = d.k;
            sid = prm.lt.sid_value[d.l];
            float kappa = coarse_draw(d.t, prm.lt.c_prev[d.l], prm.lt.stride[d.l]) ? prm.lt.kappa_coarse[d.l]
                                                                                     : prm.lt.kappa_fine[d.l];
            if (prm.iw) kappa *= (float)((double)prm.cum[prm.n - 1] / ((double)prm.n * (double)prm.iw[j]));
            prm.kap[e] = kappa;
            prm.info[e] = make_uint2(k, sid);
        }
        cols[threadIdx.x] = j;
        reals[threadIdx.x] = k;
        sids[threadIdx.x] = sid;
    }
    const int64_t m = prm.m, rows = prm.m + prm.p;
    const int ngroups = (nvalid + 3) / 4;                 // groups of four draws with a valid one
    // reparameterised laws whose rows allow 16-byte loads of four means / scales
    auto vec_law = [](const Law& l) {
        return l.kind == 2 && (l.ld & 3) == 0 && ((uintptr_t)l.mean & 15) == 0 && ((uintptr_t)l.stdev & 15) == 0;
    };
    const bool vec_ms[2] = {vec_law(prm.A), vec_law(prm.B)};
    for (int part = 0; part < 2; ++part) {
        const int64_t K = part ? prm.p : m;               // rows of the operand
        const int64_t kc = part ? prm.kcb : prm.kca;      // its padded K
        const int64_t off = part ? m : 0;                 // its first row in [a; b]
        for (int64_t k0 = 0; k0 < kc; k0 += kAdjGatherBlock) {
            __syncthreads();                              // the tile is free (and the draw table written)
            // rows k0 .. k1 - 1 of the operand are real; the rest of the tile is zero
            const int64_t k1 = K < k0 + kAdjGatherBlock ? K : k0 + kAdjGatherBlock;
            for (int i = threadIdx.x; i < kAdjGatherBlock * kAdjRows; i += kAdjThreads) {
                const int rr = i / kAdjRows, d = i % kAdjRows;
                if (k0 + rr >= k1 || d >= nvalid) tile[rr][d] = 0.0f;
            }
            if (k0 < k1) {
                // quads of [a; b] rows covering rows off + k0 .. off + k1 - 1
                const int64_t q_lo = (off + k0) / 4, q_hi = (off + k1 - 1) / 4;
                const int nq = (int)(q_hi - q_lo + 1);
                for (int item = threadIdx.x; item < nq * ngroups; item += kAdjThreads) {
                    const int g = item / nq;
                    const int64_t q = q_lo + item % nq;
                    const int64_t e0 = 4 * q;
                    for (int dd = 0; dd < 4; ++dd) {
                        const int r = 4 * g + dd;
                        if (r >= nvalid) break;
                        const uint32_t j = cols[r], kr = reals[r], sid = sids[r];
                        float u[4], z[4];
                        adj_quad(prm.value16, (uint32_t)q, kr, j, sid, prm.key0, prm.key1, u, z);
                        // the quad's rows that lie in this block of this operand
                        const Law& law = part ? prm.B : prm.A;
                        const bool whole = e0 >= off + k0 && e0 + 3 < off + k1 && ((e0 - off) & 3) == 0;
                        if (whole && vec_ms[part]) {
                            // a whole aligned quad of a reparameterised law: the
                            // four means and scales as two 16-byte loads
                            const int64_t k = e0 - off, idx = (int64_t)j * law.ld + k;
                            const float4 mu = *reinterpret_cast<const float4*>(law.mean + idx);
                            const float4 sd = *reinterpret_cast<const float4*>(law.stdev + idx);
                            tile[k - k0][r] = fmaf(sd.x, z[0], mu.x);
                            tile[k - k0 + 1][r] = fmaf(sd.y, z[1], mu.y);
                            tile[k - k0 + 2][r] = fmaf(sd.z, z[2], mu.z);
                            tile[k - k0 + 3][r] = fmaf(sd.w, z[3], mu.w);
                        } else {
                            for (int i2 = 0; i2 < 4; ++i2) {
                                const int64_t e = e0 + i2;
                                if (e < off + k0 || e >= off + k1 || e >= rows) continue;
                                const int64_t k = e - off;
                                tile[k - k0][r] = law_value<float>(law, z[i2], u[i2], (int64_t)j * law.ld + k);
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // write the block out
            if constexpr (!BF16) {
                float* V = static_cast<float*>(part ? prm.VB : prm.VA);
                for (int i = threadIdx.x; i < kAdjGatherBlock * kAdjRows / 4; i += kAdjThreads) {
                    const int rr = i / (kAdjRows / 4), d4 = i % (kAdjRows / 4);
                    *reinterpret_cast<float4*>(V + adj_blk_f32(T, kc, k0 + rr, 4 * d4)) =
                        *reinterpret_cast<const float4*>(&tile[rr][4 * d4]);
                }
            } else {
                __bf16* V = static_cast<__bf16*>(part ? prm.VB : prm.VA);
                for (int i = threadIdx.x; i < (kAdjGatherBlock / 8) * kAdjRows; i += kAdjThreads) {
                    const int g8 = i / kAdjRows, d = i % kAdjRows;
                    bf16x8 v;
#pragma unroll
                    for (int i2 = 0; i2 < 8; ++i2) v[i2] = (__bf16)tile[8 * g8 + i2][d];
                    *reinterpret_cast<bf16x8*>(V + adj_blk_bf16(T, kc, k0 + 8 * g8, d)) = v;
                }
            }
        }
    }
}

// ---- contraction tiles and the segmented sums --------------------------------
typedef __attribute__((address_space(1))) void* AdjGlobalPtr;   // operands of global_load_lds
typedef __attribute__((address_space(3))) void* AdjLdsPtr;

struct AdjTileParams {
    int64_t m, p, E;
    int64_t kca, kcb;             // K extents of the t operand blocks (of a_t and of b_t)
    int64_t xpad_m, xpad_p;       // m, p rounded up to 128
    const void* XU;               // x operand of U = B_S G^T: FP32 [kcb][xpad_m] (G^T), BF16 blocked
    const void* XV;               // x operand of V = A_S^T G: FP32 [kca][xpad_p] (G), BF16 blocked
    const void* VA;               // t operand of V (values of a_t), tile-blocked
    const void* VB;               // t operand of U (values of b_t)
    const float* kap;
    const uint2* info;            // (realisation, value stream) of each sorted draw
    const uint32_t* keys;
    uint32_t key0, key1;
    bool value16;
    int64_t tiles;                // row tiles (64 sorted draws each)
    int64_t tiles_u, tiles_v;     // column tiles of U; those of V follow
    float* dMA; float* dSA; int64_t lda;
    float* dMB; float* dSB; int64_t ldb;
    float* carry;                 // tiles x 2 (first, last) x 2 (dM, dS) x (m + p)
};

// K-chunk of a stage: 16 (FP32) or 32 (BF16) k; a stage holds the chunk's t
// block (64 rows, 4 KB) and x block (128 columns, 8 KB); kAdjStages stages
// keep two chunks' loads in flight during the MFMAs of a third.
constexpr int kAdjStages = 4;
constexpr int kAdjStageBytes = 12 * 1024;
constexpr size_t kAdjSums = kAdjRows * kAdjCols * sizeof(float);
constexpr size_t kAdjLds = (size_t)kAdjStages * kAdjStageBytes > kAdjSums ? (size_t)kAdjStages * kAdjStageBytes
                                                                            : kAdjSums;
constexpr int kAdjBatch = 8;              // gradient read-modify-writes in flight per thread
static_assert(kAdjKc % (4 * 32) == 0, "the padded K holds a whole number of four-chunk steps");
constexpr int kAdjXcds = 8;               // accelerator complex dies of an MI355X, each with its own L2

struct AdjTileShape {
    int64_t T;                    // tile of sorted draws
    bool is_u;
    int xt;                       // column tile (of U or of V)
    int xb;                       // first gradient column of the tile
    int X;                        // gradient columns
    int wt, wx;                   // the wave's 32 x 64 block inside the tile
};

// Workgroups are dealt to the XCDs in turn (workgroup i to XCD i % 8); the
// tiles are numbered so that each XCD takes a contiguous range of them, and
// the column tiles of one row tile are adjacent: the workgroups that read
// the same t block then run on one XCD at about the same time and share it
// through that XCD's L2.
__device__ __forceinline__ AdjTileShape adj_shape(const AdjTileParams& prm)
{
    // the grid has fewer than 2^31 workgroups: 32-bit arithmetic
    const uint32_t xt = (uint32_t)(prm.tiles_u + prm.tiles_v);
    const uint32_t total = (uint32_t)prm.tiles * xt;
    const uint32_t i = blockIdx.x;
    const uint32_t xcd = i % kAdjXcds, local = i / kAdjXcds;
    const uint32_t q = total / kAdjXcds, rem = total % kAdjXcds;
    const uint32_t li = xcd * q + (xcd < rem ? xcd : rem) + local;
    AdjTileShape s;
    s.T = li / xt;
    int64_t ct = li % xt;
    s.is_u = ct < prm.tiles_u;
    if (!s.is_u) ct -= prm.tiles_u;
    s.xt = (int)ct;
    s.xb = (int)ct * kAdjCols;
    s.X = (int)(s.is_u ? prm.m : prm.p);
    const int wave = threadIdx.x / kWave;
    s.wt = (wave / 2) * 32;
    s.wx = (wave % 2) * 64;
    return s;
}

// Segments of the tile's rows, the same for every column: skey[0] is the
// column of the draw before the tile, skey[1 + r] row r's, skey[65] the one
// after the tile (kNoKey past either end); fin[0 .. nfin) lists the rows that
// close a segment lying inside the tile (finished here); the first segment
// goes to carry slot 0 when it began in an earlier tile, the last to slot 1
// when it continues into the next.
struct AdjSegments {
    uint32_t skey[kAdjRows + 2];
    float kap[kAdjRows];          // kappa_t of the tile's rows (0 past the end)
    uint2 info[kAdjRows];         // (realisation, value stream) of the tile's rows
    uint64_t ends;                // bit r: row r closes a segment
    int began;                    // the first segment began in an earlier tile
    int cont;                     // the last segment continues into the next tile
    uint8_t fin[kAdjRows];
    int nfin;
    float part[kAdjCols];         // the walk's upper-half share of a segment across rows 31 | 32
};

__device__ __forceinline__ void adj_load_keys(const AdjTileParams& prm, int64_t T, AdjSegments& sg)
{
    const int64_t r0 = T * kAdjRows;
    if (threadIdx.x < kAdjRows + 2) {
        const int64_t e = r0 - 1 + threadIdx.x;
        sg.skey[threadIdx.x] = (e >= 0 && e < prm.E) ? prm.keys[e] : kNoKey;
    }
    if (threadIdx.x < kAdjRows) {
        const int64_t e = r0 + threadIdx.x;
        sg.kap[threadIdx.x] = e < prm.E ? prm.kap[e] : 0.0f;
        sg.info[threadIdx.x] = e < prm.E ? prm.info[e] : make_uint2(0u, 0u);
    }
}

__device__ __forceinline__ void adj_segments(AdjSegments& sg, int rows)
{
    int n = 0, start = 0;
    uint64_t ends = 0ull;
    sg.began = sg.skey[0] == sg.skey[1];
    sg.cont = rows == kAdjRows && sg.skey[kAdjRows + 1] == sg.skey[kAdjRows];
    for (int r = 0; r < rows; ++r) {
        if (r == rows - 1 || sg.skey[r + 2] != sg.skey[r + 1]) {
            ends |= 1ull << r;
            const bool began = start == 0 && sg.began;
            const bool cont = r == rows - 1 && sg.cont;
            if (!began && !cont) sg.fin[n++] = (uint8_t)r;
            start = r + 1;
        }
    }
    sg.ends = ends;
    sg.nfin = n;
}

// Row t of the epilogue's 64 x 128 sums lives in one of three stage arrays
// (24 rows each).
struct AdjRows {
    float* s0;
    float* s1;
    float* s2;
    __device__ __forceinline__ float* row(int t) const
    {
        return t < 24 ? s0 + t * kAdjCols : t < 48 ? s1 + (t - 24) * kAdjCols : s2 + (t - 48) * kAdjCols;
    }
};

// The accumulators (lane l, register r of block bj: row 8(r/4) + 4(l/32) + r%4,
// column 32 bj + l%32 of the wave's block) times kappa_t (dM), then times
// kappa_t z_t (dS), each in turn through LDS.  The walk down the rows is
// split in two halves, rows 0 .. 31 and 32 .. 63, each walked by 128 threads
// (one per column): a segment that runs across row 31 | 32 is finished from
// the two halves' partial sums (upper + lower) after a barrier.  A finished
// segment's sum is left in the row that closes it (or in its carry slot);
// then all threads add the finished sums into the gradient rows, kAdjBatch
// independent read-modify-writes at a time.
__device__ __forceinline__ void adj_epilogue(const AdjTileParams& prm, const AdjTileShape& sh, const f32x16 (&acc)[2],
                                             const AdjRows& sv, AdjSegments& sg)
{
    constexpr int H = kAdjRows / 2;
    const int lane = threadIdx.x % kWave;
    const int64_t r0 = sh.T * kAdjRows;
    const int64_t left = prm.E - r0;
    const int rows = left < kAdjRows ? (int)left : kAdjRows;
    if (threadIdx.x == 0) adj_segments(sg, rows);
    const int64_t ld = sh.is_u ? prm.lda : prm.ldb;
    const int64_t cw = prm.m + prm.p;
    const bool lower = threadIdx.x >= kAdjCols;            // walks rows H .. rows - 1
    const int xl = threadIdx.x % kAdjCols, x = sh.xb + xl;
    const int64_t ccol = (sh.is_u ? 0 : prm.m) + x;
    for (int which = 0; which < 2; ++which) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int xw = sh.wx + bj * 32 + lane % 32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int t = sh.wt + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
                sv.row(t)[xw] = sg.kap[t] * acc[bj][r];
            }
        }
        __syncthreads();
        if (which) {
            // the normals of the tile's columns, regenerated from the draws'
            // streams (one Philox quad of rows per item), multiply in place
            const int64_t off = sh.is_u ? 0 : prm.m;        // the columns' first row in [a; b]
            const int x_end = sh.xb + kAdjCols < sh.X ? sh.xb + kAdjCols : sh.X;
            const int64_t q_lo = (off + sh.xb) / 4, q_hi = (off + x_end - 1) / 4;
            const int nq = (int)(q_hi - q_lo + 1);
            for (int item = threadIdx.x; item < rows * nq; item += kAdjThreads) {
                const int t = item / nq;
                const int64_t q = q_lo + item % nq;
                const uint2 inf = sg.info[t];
                float u[4], z[4];
                adj_quad(prm.value16, (uint32_t)q, inf.x, sg.skey[t + 1], inf.y, prm.key0, prm.key1, u, z);
                float* row = sv.row(t);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t c = 4 * q + i - off;            // gradient column
                    if (c >= sh.xb && c < x_end) row[c - sh.xb] *= z[i];
                }
            }
            __syncthreads();
        }
        // segment ends are the same for every column (uniform branches)
        const uint64_t ends = sg.ends;
        const bool span = rows > H && !((ends >> (H - 1)) & 1ull);   // a segment runs across H - 1 | H
        const bool span_began = span && sg.began && (ends & ((1ull << H) - 1ull)) == 0ull;
        float held = 0.0f;                                 // the lower half's share of that segment
        int held_row = -1;
        auto finish = [&](int r, float sum, bool began) {
            const bool cont = r == rows - 1 && sg.cont;
            if (began || cont)
                prm.carry[((sh.T * 2 + (began ? 0 : 1)) * 2 + which) * cw + ccol] = sum;
            else
                sv.row(r)[xl] = sum;
        };
        if (x < sh.X) {
            const int r_begin = lower ? H : 0;
            const int r_end = lower ? rows : (rows < H ? rows : H);
            float sum = 0.0f;
            bool first = true;
#pragma unroll 1
            for (int r = r_begin; r < r_end; ++r) {
                float* cell = sv.row(r) + xl;
                sum += *cell;
                if ((ends >> r) & 1ull) {
                    if (lower && first && span) {
                        held = sum;
                        held_row = r;
                    } else {
                        finish(r, sum, first && (lower ? false : sg.began));
                    }
                    sum = 0.0f;
                    first = false;
                }
            }
            if (!lower && span) sg.part[xl] = sum;        // the upper half's share
        }
        __syncthreads();
        if (lower && x < sh.X && held_row >= 0) finish(held_row, sg.part[xl] + held, span_began);
        __syncthreads();
        float* grad = sh.is_u ? (which ? prm.dSA : prm.dMA) : (which ? prm.dSB : prm.dMB);
        const int items = sg.nfin * kAdjCols;
        for (int base = 0; base < items; base += kAdjThreads * kAdjBatch) {
            float* ptr[kAdjBatch];
            float v[kAdjBatch], g[kAdjBatch];
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u) {
                const int i = base + u * kAdjThreads + (int)threadIdx.x;
                const int r = i < items ? sg.fin[i / kAdjCols] : 0;
                const int xl = i % kAdjCols, x = sh.xb + xl;
                ptr[u] = nullptr;
                if (i < items && x < sh.X) {
                    ptr[u] = grad + (int64_t)sg.skey[r + 1] * ld + x;
                    v[u] = sv.row(r)[xl];
                }
            }
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u)
                if (ptr[u]) g[u] = *ptr[u];
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u)
                if (ptr[u]) *ptr[u] = g[u] + v[u];
        }
        __syncthreads();
    }
}

// U^T = B_S G^T (rows: the tile's sorted draws, columns i) or V = A_S^T G
// (columns q).  FP32: v_mfma_f32_32x32x2_f32, chunks of 16 k; BF16:
// v_mfma_f32_32x32x16_bf16 (FP32 accumulation), chunks of 32 k.  A chunk's t
// block (4 KB) and x block (8 KB) go straight from global memory into one of
// four LDS stage arrays (global_load_lds_dwordx4: lane i's 16 bytes land at
// the wave's base plus 16 i, which is the stored layout), so no registers
// hold them; the chunks c + 1 and c + 2 are in flight while the MFMAs run on
// chunk c, and the loads of chunk c + 3 are issued once every wave is past
// chunk c - 1.  The stage arrays are separate objects so that the fragment
// reads of one are not made to wait for the loads into the others.  2 x 2
// waves, each 32 x 64 (two blocks sharing the t fragment).
template <bool BF16>
__global__ __launch_bounds__(kAdjThreads) void adj_tile_kernel(AdjTileParams prm)
{
    constexpr int C = BF16 ? 32 : 16;                  // k per chunk
    constexpr int kLoads = 3;                          // global_load_lds per thread per chunk
    __shared__ __align__(16) char st0[kAdjStageBytes];
    __shared__ __align__(16) char st1[kAdjStageBytes];
    __shared__ __align__(16) char st2[kAdjStageBytes];
    __shared__ __align__(16) char st3[kAdjStageBytes];
    __shared__ AdjSegments sg;
    const AdjTileShape sh = adj_shape(prm);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    adj_load_keys(prm, sh.T, sg);
    const int64_t kc = sh.is_u ? prm.kcb : prm.kca;    // padded contraction length (multiple of 4 C)
    const int64_t esz = BF16 ? 2 : 4;
    // the tile's t block: kc x 64 values, 4 KB per chunk
    const char* tsrc = static_cast<const char*>(sh.is_u ? prm.VB : prm.VA) + sh.T * kc * kAdjRows * esz;
    const char* xsrc = static_cast<const char*>(sh.is_u ? prm.XU : prm.XV);
    const int64_t xpad = sh.is_u ? prm.xpad_m : prm.xpad_p;
    if constexpr (BF16) xsrc += (int64_t)sh.xt * kc * kAdjCols * esz;   // blocked: [tile][k/8][128][8]

    auto issue = [&](int c, char* st) {
        __builtin_amdgcn_global_load_lds((AdjGlobalPtr)(tsrc + (int64_t)c * 4096 + threadIdx.x * 16),
                                         (AdjLdsPtr)(st + wave * 1024), 16, 0, 0);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int vid = threadIdx.x + v * kAdjThreads;
            const char* src;
            if constexpr (BF16) {
                src = xsrc + (int64_t)c * 8192 + vid * 16;
            } else {
                const int k = vid / 32, x4 = vid % 32;  // [k][128] floats
                src = xsrc + (((int64_t)c * C + k) * xpad + sh.xb + 4 * x4) * 4;
            }
            __builtin_amdgcn_global_load_lds((AdjGlobalPtr)src, (AdjLdsPtr)(st + 4096 + (v * kAdjThreads + wave * kWave) * 16),
                                             16, 0, 0);
        }
    };
    f32x16 acc[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[bj][r] = 0.0f;
    auto compute = [&](const char* st) {
        if constexpr (BF16) {
            const __bf16* A = reinterpret_cast<const __bf16*>(st);          // [4][64][8]
            const __bf16* B = reinterpret_cast<const __bf16*>(st + 4096);   // [4][128][8]
#pragma unroll
            for (int kk = 0; kk < C; kk += 16) {
                const int g = kk / 8 + lane / 32;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(A + (g * kAdjRows + sh.wt + lane % 32) * 8);
                const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(B + (g * kAdjCols + sh.wx + lane % 32) * 8);
                const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(B + (g * kAdjCols + sh.wx + 32 + lane % 32) * 8);
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc[1], 0, 0, 0);
            }
        } else {
            const float* A = reinterpret_cast<const float*>(st);            // [16][64]
            const float* B = reinterpret_cast<const float*>(st + 4096);     // [16][128]
#pragma unroll
            for (int kk = 0; kk < C; kk += 2) {
                const float a = A[(kk + lane / 32) * kAdjRows + sh.wt + lane % 32];
                const float b0 = B[(kk + lane / 32) * kAdjCols + sh.wx + lane % 32];
                const float b1 = B[(kk + lane / 32) * kAdjCols + sh.wx + 32 + lane % 32];
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc[1], 0, 0, 0);
            }
        }
    };
    // Every step issues one chunk (past the last one, the last chunk again,
    // into a stage that is not read any more), so at the wait for chunk c
    // exactly the loads of the two chunks after it are younger: vmcnt counts
    // the outstanding loads in issue order.
    auto wait_chunk = [&]() {
        // s_waitcnt: vmcnt in bits 3:0 (and 15:14), lgkmcnt 11:8 at 0 (this
        // wave's fragment reads are done), expcnt 6:4 left at its maximum
        __builtin_amdgcn_s_waitcnt(0x0070 | (2 * kLoads));
    };
    // The stage handover needs only the workgroup barrier: each wave has
    // waited for its own loads of the chunk (vmcnt), and the LDS reads of the
    // stage it overwrites next were consumed by MFMAs before the barrier.
    // __syncthreads would also fence global memory, i.e. wait for every load
    // still in flight.
    auto handover = [&]() { asm volatile("s_barrier" ::: "memory"); };
    const int chunks = (int)(kc / C);                  // a multiple of 4
    issue(0, st0);
    issue(1, st1);
    issue(2, st2);
    auto next = [&](int c) { return c < chunks ? c : chunks - 1; };
    for (int c = 0; c < chunks; c += 4) {
        wait_chunk();
        handover();
        issue(next(c + 3), st3);
        compute(st0);
        wait_chunk();
        handover();
        issue(next(c + 4), st0);
        compute(st1);
        wait_chunk();
        handover();
        issue(next(c + 5), st1);
        compute(st2);
        wait_chunk();
        handover();
        issue(next(c + 6), st2);
        compute(st3);
    }
    __syncthreads();                                   // the repeated last loads have landed
    adj_epilogue(prm, sh, acc, AdjRows{reinterpret_cast<float*>(st0), reinterpret_cast<float*>(st1),
                                       reinterpret_cast<float*>(st2)}, sg);
}

// A column segment that crosses tile edges: its first tile T (whose last
// segment continues and began in T) adds T's partial and those of the tiles
// it runs through, in tile order, and writes the gradient row once.
struct AdjFixParams {
    int64_t m, p, E;
    const uint32_t* keys;
    const float* carry;
    float* dMA; float* dSA; int64_t lda;
    float* dMB; float* dSB; int64_t ldb;
};

__device__ __forceinline__ bool adj_continues(const uint32_t* keys, int64_t E, int64_t T)
{
    const int64_t l = T * kAdjRows + kAdjRows - 1;
    return l + 1 < E && keys[l] == keys[l + 1];
}

__global__ __launch_bounds__(kAdjThreads) void adj_fixup_kernel(AdjFixParams prm)
{
    const int64_t T = blockIdx.x;
    const uint32_t* keys = prm.keys;
    if (!adj_continues(keys, prm.E, T)) return;
    const int64_t f = T * kAdjRows;
    const bool whole = keys[f] == keys[f + kAdjRows - 1];
    const bool began = T > 0 && keys[f - 1] == keys[f];
    if (whole && began) return;                           // inside a chain that starts earlier
    const uint32_t j = keys[f + kAdjRows - 1];
    const int64_t cw = prm.m + prm.p;
    for (int64_t ci = threadIdx.x; ci < 2 * cw; ci += kAdjThreads) {
        const int which = ci >= cw;
        const int64_t col = ci - which * cw;
        float sum = prm.carry[((T * 2 + 1) * 2 + which) * cw + col];
        for (int64_t t2 = T + 1;; ++t2) {
            sum += prm.carry[((t2 * 2 + 0) * 2 + which) * cw + col];
            const int64_t f2 = t2 * kAdjRows;
            if (!(adj_continues(keys, prm.E, t2) && keys[f2] == keys[f2 + kAdjRows - 1])) break;
        }
        float* g = col < prm.m ? (which ? prm.dSA : prm.dMA) + (int64_t)j * prm.lda + col
                               : (which ? prm.dSB : prm.dMB) + (int64_t)j * prm.ldb + (col - prm.m);
        *g += sum;
    }
}

// ---- G, workspace and the pass loop -------------------------------------------
// The x operands from G = dL/dY (FP64, m x p row-major), with zeros in the
// padding: FP32 G^T as [kcb][xpad_m] and G as [kca][xpad_p]; BF16 (round to
// nearest even) blocked per column tile, [tile][k / 8][128][k % 8]: for U,
// column x = i and k = q (the value G[i][q]); for V, x = q and k = i.
struct AdjXOperands {
    int64_t m, p, kca, kcb, xpad_m, xpad_p;
    const double* grad;
    void* XU;
    void* XV;
};

template <bool BF16>
__global__ __launch_bounds__(256) void adj_x_operands_kernel(AdjXOperands o)
{
    const int64_t nu = o.kcb * o.xpad_m, nv = o.kca * o.xpad_p;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nu + nv) return;
    const bool u = e < nu;
    const int64_t f = u ? e : e - nu;
    const int64_t kc = u ? o.kcb : o.kca;
    int64_t k, x;
    if constexpr (BF16) {
        // f = ((tile * (kc / 8) + k / 8) * 128 + x % 128) * 8 + k % 8
        const int64_t k8 = f % 8, xl = (f / 8) % kAdjCols, g = f / (8 * kAdjCols);
        k = (g % (kc / 8)) * 8 + k8;
        x = (g / (kc / 8)) * kAdjCols + xl;
    } else {
        const int64_t xpad = u ? o.xpad_m : o.xpad_p;
        k = f / xpad;
        x = f % xpad;
    }
    // U: x = i < m, k = q < p; V: x = q < p, k = i < m
    const int64_t i = u ? x : k, q = u ? k : x;
    const float v = (i < o.m && q < o.p) ? (float)o.grad[i * o.p + q] : 0.0f;
    if constexpr (BF16) static_cast<__bf16*>(u ? o.XU : o.XV)[f] = (__bf16)v;
    else static_cast<float*>(u ? o.XU : o.XV)[f] = v;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct AdjDims {
    int64_t kca, kcb, xpad_m, xpad_p;
};

static AdjDims adj_dims(int64_t m, int64_t p)
{
    AdjDims d;
    d.kca = round_up_adj(m, kAdjKc);
    d.kcb = round_up_adj(p, kAdjKc);
    d.xpad_m = round_up_adj(m, kAdjCols);
    d.xpad_p = round_up_adj(p, kAdjCols);
    return d;
}

// Head of the workspace: the two x operands (FP32 sizes; BF16 uses half).
static size_t adj_head_bytes(int64_t m, int64_t p)
{
    const AdjDims d = adj_dims(m, p);
    return align256((size_t)(d.kcb * d.xpad_m) * 4) + align256((size_t)(d.kca * d.xpad_p) * 4);
}

// The buffers of a pass of E draws (values sized for FP32, which BF16 halves).
struct AdjPassLayout {
    size_t keys0, vals0, keys1, vals1, counts, VA, VB, info, kap, carry, total;
};

static AdjPassLayout adj_pass_layout(int64_t E, int64_t m, int64_t p)
{
    const AdjDims d = adj_dims(m, p);
    const int64_t nb = ceil_div(E, kSortBlock), tiles = ceil_div(E, kAdjRows);
    AdjPassLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t at = off; off = align256(off + bytes); return at; };
    L.keys0 = take(4 * (size_t)E);
    L.vals0 = take(4 * (size_t)E);
    L.keys1 = take(4 * (size_t)E);
    L.vals1 = take(4 * (size_t)E);
    L.counts = take(4 * (size_t)kSortThreads * (size_t)nb);
    L.VA = take(4 * (size_t)(tiles * kAdjRows * d.kca));
    L.VB = take(4 * (size_t)(tiles * kAdjRows * d.kcb));
    L.info = take(8 * (size_t)E);
    L.kap = take(4 * (size_t)E);
    L.carry = take(4 * (size_t)(tiles * 4 * (m + p)));
    L.total = off;
    return L;
}

// Draws per pass: all of them when their buffers fit the budget, else the
// most that fit (at least 64); at most 2^30 draws and a tile grid below 2^31
// workgroups.
static int64_t adj_pass_draws(int64_t m, int64_t p, size_t budget, int64_t draws)
{
    const int64_t xt = ceil_div(m, kAdjCols) + ceil_div(p, kAdjCols);
    int64_t cap = ((1ll << 31) - 1) / xt * kAdjRows;
    if (cap > (1ll << 30)) cap = 1ll << 30;
    if (draws <= cap && adj_pass_layout(draws, m, p).total <= budget) return draws;
    const size_t per = adj_pass_layout(kAdjRows, m, p).total / kAdjRows + 1;
    int64_t E = (int64_t)(budget / per);
    if (E > cap) E = cap;
    E = E / kAdjRows * kAdjRows;
    if (E < kAdjRows) E = kAdjRows;
    while (E > kAdjRows && adj_pass_layout(E, m, p).total > budget) E -= kAdjRows;
    return E;
}

// Pass buffers: room for every draw of the call, or kAdjBudget when that is
// less (N NULL: kAdjBudget); always room for one 64-draw pass.
static size_t adj_budget(int64_t m, int64_t p, int num_levels, const int64_t* c, const int64_t* N)
{
    size_t need = (size_t)kAdjBudget;
    if (N) {
        int64_t draws = 0;
        for (int l = 0; l < num_levels; ++l) draws += N[l] * c[l];
        const size_t all = adj_pass_layout(draws, m, p).total;
        if (all < need) need = all;
    }
    const size_t one = adj_pass_layout(kAdjRows, m, p).total;
    return need > one ? need : one;
}

size_t adjoint_workspace_size(int64_t m, int64_t n, int64_t p, int num_levels, const int64_t* c, const int64_t* N,
                              bool weighted)
{
    size_t total = adj_budget(m, p, num_levels, c, N) + adj_head_bytes(m, p);
    if (weighted) total += align256((size_t)n * sizeof(uint64_t));
    return total;
}

size_t adjoint_workspace_min(int64_t m, int64_t n, int64_t p, bool weighted)
{
    size_t total = adj_pass_layout(kAdjRows, m, p).total + adj_head_bytes(m, p);
    if (weighted) total += align256((size_t)n * sizeof(uint64_t));
    return total;
}

hipError_t adjoint_run(int64_t m, int64_t n, int64_t p, const Law& A, const Law& B, int num_levels,
                       const int64_t* c, const int64_t* N, const StreamKeys& keys, bool shared,
                       const double* grad, float* dMA, float* dSA, float* dMB, float* dSB,
                       const uint32_t* index_weights, char* ws, size_t ws_bytes, bool bf16, bool stride,
                       bool value16, hipStream_t stream, KernelTimer* timer)
{
    const AdjDims dims = adj_dims(m, p);
    AdjXOperands xo;
    xo.m = m; xo.p = p; xo.kca = dims.kca; xo.kcb = dims.kcb; xo.xpad_m = dims.xpad_m; xo.xpad_p = dims.xpad_p;
    xo.grad = grad;
    xo.XU = ws;
    xo.XV = ws + align256((size_t)(dims.kcb * dims.xpad_m) * 4);
    const size_t head = adj_head_bytes(m, p);
    // the cumulative index weights follow the head
    uint64_t* cum = index_weights ? reinterpret_cast<uint64_t*>(ws + head) : nullptr;
    const size_t cum_bytes = index_weights ? align256((size_t)n * sizeof(uint64_t)) : 0;
    char* buf = ws + head + cum_bytes;
    // the pass buffers: what the workspace holds, up to what all draws need
    if (head + cum_bytes + adj_pass_layout(kAdjRows, m, p).total > ws_bytes) return hipErrorInvalidValue;
    size_t budget = ws_bytes - head - cum_bytes;
    const size_t want = adj_budget(m, p, num_levels, c, N);
    if (budget > want) budget = want;
    {
        ScopedTiming t(timer, 3);
        const int64_t total = dims.kcb * dims.xpad_m + dims.kca * dims.xpad_p;
        if (bf16)
            hipLaunchKernelGGL(adj_x_operands_kernel<true>, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, stream,
                               xo);
        else
            hipLaunchKernelGGL(adj_x_operands_kernel<false>, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0,
                               stream, xo);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (index_weights && (e = build_cumulative(index_weights, n, cum, stream)) != hipSuccess) return e;
    // digits of the column: 8 bits per sort pass
    int bits = 0;
    while (bits < 32 && ((uint64_t)(n - 1) >> bits) != 0) ++bits;
    const int digit_passes = (bits + 7) / 8;
    AdjLevelTable lt;
    lt.nlev = num_levels;
    lt.first[0] = 0;
    for (int l = 0; l < num_levels; ++l) {
        const int64_t cl = c[l], cp = l > 0 ? c[l - 1] : 0;
        const double base = (double)n / (double)cl / (double)N[l];
        const uint32_t lf = shared ? 0xFFu : (uint32_t)l;
        lt.c[l] = (uint32_t)cl;
        lt.c_prev[l] = (uint32_t)cp;
        lt.stride[l] = stride && cp > 0 ? (uint32_t)(cl / cp) : 0u;
        lt.sid_index[l] = stream_id(kTagIndex, lf, keys.problem);
        lt.sid_value[l] = stream_id(kTagValue, lf, keys.problem);
        lt.kappa_coarse[l] = (float)(base * (cp > 0 ? 1.0 - (double)cl / (double)cp : 1.0));
        lt.kappa_fine[l] = (float)base;
        lt.first[l + 1] = lt.first[l] + N[l] * cl;
    }
    const int64_t draws = lt.first[num_levels];
    const int64_t per_pass = adj_pass_draws(m, p, budget, draws);
    for (int64_t g0 = 0; g0 < draws; g0 += per_pass) {
        const int64_t E = (draws - g0) < per_pass ? (draws - g0) : per_pass;
        const AdjPassLayout L = adj_pass_layout(E, m, p);
        if (L.total > budget) return hipErrorInvalidValue;
        uint32_t* kbuf[2] = {reinterpret_cast<uint32_t*>(buf + L.keys0), reinterpret_cast<uint32_t*>(buf + L.keys1)};
        uint32_t* vbuf[2] = {reinterpret_cast<uint32_t*>(buf + L.vals0), reinterpret_cast<uint32_t*>(buf + L.vals1)};
        uint32_t* counts = reinterpret_cast<uint32_t*>(buf + L.counts);
        const int64_t nb = ceil_div(E, kSortBlock), tiles = ceil_div(E, kAdjRows);
        int cur = 0;
        {
            ScopedTiming t(timer, 1);
            AdjKeyParams kp;
            kp.lt = lt;
            kp.g0 = g0; kp.E = E; kp.n = (uint32_t)n;
            kp.key0 = keys.key0; kp.key1 = keys.key1;
            kp.cum = cum; kp.keys = kbuf[0]; kp.vals = vbuf[0];
            hipLaunchKernelGGL(adj_keys_kernel, dim3((unsigned)ceil_div(E, 256)), dim3(256), 0, stream, kp);
            for (int d = 0; d < digit_passes; ++d) {
                hipLaunchKernelGGL(adj_radix_hist_kernel, dim3((unsigned)nb), dim3(kSortThreads), 0, stream,
                                   kbuf[cur], E, 8 * d, counts, nb);
                hipLaunchKernelGGL(adj_radix_scan_kernel, dim3(1), dim3(kSortScanThreads), 0, stream, counts,
                                   (int64_t)kSortThreads * nb);
                hipLaunchKernelGGL(adj_radix_scatter_kernel, dim3((unsigned)nb), dim3(kSortThreads), 0, stream,
                                   kbuf[cur], vbuf[cur], kbuf[cur ^ 1], vbuf[cur ^ 1], E, 8 * d, counts, nb);
                cur ^= 1;
            }
            AdjGatherParams g;
            g.lt = lt;
            g.m = m; g.p = p; g.g0 = g0; g.E = E;
            g.kca = dims.kca; g.kcb = dims.kcb;
            g.n = (uint32_t)n;
            g.key0 = keys.key0; g.key1 = keys.key1;
            g.A = A; g.B = B;
            g.keys = kbuf[cur]; g.vals = vbuf[cur];
            g.iw = index_weights; g.cum = cum;
            g.VA = buf + L.VA; g.VB = buf + L.VB;
            g.info = reinterpret_cast<uint2*>(buf + L.info);
            g.kap = reinterpret_cast<float*>(buf + L.kap);
            g.value16 = value16;
            if (bf16) hipLaunchKernelGGL(adj_gather_kernel<true>, dim3((unsigned)tiles), dim3(kAdjThreads), 0, stream, g);
            else hipLaunchKernelGGL(adj_gather_kernel<false>, dim3((unsigned)tiles), dim3(kAdjThreads), 0, stream, g);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        AdjTileParams a;
        a.m = m; a.p = p; a.E = E; a.kca = dims.kca; a.kcb = dims.kcb;
        a.xpad_m = dims.xpad_m; a.xpad_p = dims.xpad_p;
        a.XU = xo.XU; a.XV = xo.XV;
        a.VA = buf + L.VA; a.VB = buf + L.VB;
        a.info = reinterpret_cast<const uint2*>(buf + L.info);
        a.key0 = keys.key0; a.key1 = keys.key1; a.value16 = value16;
        a.kap = reinterpret_cast<const float*>(buf + L.kap);
        a.keys = kbuf[cur];
        a.tiles = tiles;
        a.tiles_u = ceil_div(m, kAdjCols);
        a.tiles_v = ceil_div(p, kAdjCols);
        a.dMA = dMA; a.dSA = dSA; a.lda = A.ld;
        a.dMB = dMB; a.dSB = dSB; a.ldb = B.ld;
        a.carry = reinterpret_cast<float*>(buf + L.carry);
        {
            ScopedTiming t(timer, 0);
            const dim3 grid((unsigned)(tiles * (a.tiles_u + a.tiles_v)));
            if (bf16) hipLaunchKernelGGL(adj_tile_kernel<true>, grid, dim3(kAdjThreads), 0, stream, a);
            else hipLaunchKernelGGL(adj_tile_kernel<false>, grid, dim3(kAdjThreads), 0, stream, a);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        AdjFixParams f;
        f.m = m; f.p = p; f.E = E; f.keys = kbuf[cur];
        f.carry = reinterpret_cast<const float*>(buf + L.carry);
        f.dMA = dMA; f.dSA = dSA; f.lda = A.ld;
        f.dMB = dMB; f.dSB = dSB; f.ldb = B.ld;
        {
            ScopedTiming t(timer, 2);
            hipLaunchKernelGGL(adj_fixup_kernel, dim3((unsigned)tiles), dim3(kAdjThreads), 0, stream, f);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mlmc
