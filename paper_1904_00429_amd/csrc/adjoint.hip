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
// Per pass over a batch of realisations of one level:
//   adjoint_gather:  per realisation, A_S^T (m x K, [i][t]), B_S^T (p x K,
//                    [q][t]) for the MFMA operands, Z_S (K x m, [t][i]) and
//                    W_S (K x p, [t][q]) for the epilogue, and the indices;
//   adjoint_mfma:    U^T = B_S G^T (K x m) and V = A_S^T G (K x p) with
//                    v_mfma_f32_32x32x2_f32 on LDS-staged operand chunks;
//                    each output row t is scaled by
//                    kappa_t and added (FP32 atomics, a contiguous row of the
//                    gradient per draw) into row r_t of dM/dS.
#include "internal.hpp"

namespace mlmc {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kAdjGatherThreads = 64;
constexpr int kAdjPositions = 8;
constexpr int kAdjThreads = 256;
constexpr int kAdjKStep = 2;
constexpr int64_t kAdjBudget = 192ll << 20;

struct AdjGatherParams {
    int64_t m, p;
    uint32_t n, c, c_prev;
    int64_t kpad;                 // draws per realisation rounded up to kAdjPositions
    uint32_t key0, key1, sid_index, sid_value;
    uint32_t k_first;
    Law A, B;
    float* AT;                    // batch x m x kpad
    float* BT;                    // batch x p x kpad
    float* ZS;                    // batch x kpad x m
    float* WS;                    // batch x kpad x p
    int32_t* R;                   // batch x kpad (-1 for padding)
    // BF16 form: the values position-major instead of AT/BT, element (t, i)
    // at t mk + i (mk, pk: m and p rounded up to 8)
    __bf16* ASb;                  // batch x kpad x mk
    __bf16* BSb;                  // batch x kpad x pk
    int64_t mk, pk;
    const uint64_t* cum;          // cumulative index weights (NULL: uniform draws)
    bool value16;                 // the forward's values came from 16-bit uniforms
};

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <bool BF16>
__global__ __launch_bounds__(kAdjGatherThreads) void adjoint_gather_kernel(AdjGatherParams prm)
{
    __shared__ uint32_t cols[kAdjPositions];
    __shared__ int valid[kAdjPositions];
    const int64_t pos0 = (int64_t)blockIdx.x * kAdjPositions;
    const int64_t slot = blockIdx.y;
    const uint32_t k = prm.k_first + (uint32_t)slot;
    if (threadIdx.x < kAdjPositions) {
        const int64_t t = pos0 + threadIdx.x;
        const bool ok = t < (int64_t)prm.c;
        valid[threadIdx.x] = ok;
        uint32_t j = 0u;
        if (ok)
            j = prm.cum ? draw_index_weighted((uint32_t)t, k, prm.sid_index, prm.key0, prm.key1, prm.cum, prm.n,
                                              prm.cum[prm.n - 1])
                        : draw_index((uint32_t)t, k, prm.sid_index, prm.key0, prm.key1, prm.n);
        cols[threadIdx.x] = j;
        prm.R[slot * prm.kpad + t] = ok ? (int32_t)j : -1;
    }
    __syncthreads();
    const int64_t rows = prm.m + prm.p;
    const int64_t quads = ceil_div(rows, 4);
    float* AT = prm.AT + slot * prm.m * prm.kpad;
    float* BT = prm.BT + slot * prm.p * prm.kpad;
    float* ZS = prm.ZS + slot * prm.kpad * prm.m;
    float* WS = prm.WS + slot * prm.kpad * prm.p;
    for (int64_t q = threadIdx.x; q < quads; q += kAdjGatherThreads) {
        float val[kAdjPositions][4], nrm[kAdjPositions][4];
        for (int ip = 0; ip < kAdjPositions; ++ip) {
            if (!valid[ip]) {
                for (int r = 0; r < 4; ++r) { val[ip][r] = 0.0f; nrm[ip][r] = 0.0f; }
                continue;
            }
            const uint32_t j = cols[ip];
            float u[4], z[4];
            if (prm.value16) {
                // rows 4q .. 4q+3 are halves of words 2 (q & 1) and 2 (q & 1) + 1
                // of the call for rows 8 (q / 2) .. 8 (q / 2) + 7
                const Words4 w = philox4x32_10((uint32_t)(q >> 1), k, j, prm.sid_value, prm.key0, prm.key1);
                const uint32_t a = (q & 1) ? w.w2 : w.w0, b = (q & 1) ? w.w3 : w.w1;
                u[0] = unit16<float>(a & 0xFFFFu);
                u[1] = unit16<float>(a >> 16);
                u[2] = unit16<float>(b & 0xFFFFu);
                u[3] = unit16<float>(b >> 16);
                box_muller(u[0], u[1], z[0], z[1]);
                box_muller(u[2], u[3], z[2], z[3]);
            } else {
                const Words4 w = philox4x32_10((uint32_t)q, k, j, prm.sid_value, prm.key0, prm.key1);
                quad_values<float>(w, true, u[0], u[1], u[2], u[3], z[0], z[1], z[2], z[3]);
            }
            for (int r = 0; r < 4; ++r) {
                const int64_t e = 4 * q + r;
                float v = 0.0f;
                if (e < prm.m) v = law_value<float>(prm.A, z[r], u[r], (int64_t)j * prm.A.ld + e);
                else if (e < rows) v = law_value<float>(prm.B, z[r], u[r], (int64_t)j * prm.B.ld + (e - prm.m));
                val[ip][r] = v;
                nrm[ip][r] = z[r];
            }
        }
        const int64_t e0 = 4 * q;
        if constexpr (BF16) {
            // position-major BF16 values (round to nearest even): the quad's
            // four rows are adjacent, one 8-byte store per position when they
            // lie in A, or in B at a row that is a multiple of 4
            __bf16* AS = prm.ASb + slot * prm.kpad * prm.mk;
            __bf16* BS = prm.BSb + slot * prm.kpad * prm.pk;
            const bool qa = e0 + 3 < prm.m;
            const bool qb = e0 >= prm.m && e0 + 3 < rows && ((e0 - prm.m) & 3) == 0;
            if (qa || qb) {
                __bf16* V = qa ? AS : BS;
                const int64_t st = qa ? prm.mk : prm.pk;
                const int64_t row = qa ? e0 : e0 - prm.m;
                for (int ip = 0; ip < kAdjPositions; ++ip) {
                    bf16x4 v;
                    for (int r = 0; r < 4; ++r) v[r] = (__bf16)val[ip][r];
                    *reinterpret_cast<bf16x4*>(V + (pos0 + ip) * st + row) = v;
                }
            } else {
                for (int r = 0; r < 4; ++r) {
                    const int64_t e = e0 + r;
                    if (e >= rows) break;
                    const bool in_a = e < prm.m;
                    __bf16* V = in_a ? AS : BS;
                    const int64_t st = in_a ? prm.mk : prm.pk;
                    const int64_t row = in_a ? e : e - prm.m;
                    for (int ip = 0; ip < kAdjPositions; ++ip) V[(pos0 + ip) * st + row] = (__bf16)val[ip][r];
                }
            }
        } else {
            // K-major values: a row's eight positions are adjacent (two 16-byte
            // stores; kpad and pos0 are multiples of 8)
            for (int r = 0; r < 4; ++r) {
                const int64_t e = e0 + r;
                if (e >= rows) break;
                const bool in_a = e < prm.m;
                const int64_t row = in_a ? e : e - prm.m;
                float4* T = reinterpret_cast<float4*>((in_a ? AT + row * prm.kpad : BT + row * prm.kpad) + pos0);
                T[0] = make_float4(val[0][r], val[1][r], val[2][r], val[3][r]);
                T[1] = make_float4(val[4][r], val[5][r], val[6][r], val[7][r]);
            }
        }
        // position-major normals: the quad's four rows are adjacent (one
        // 16-byte store per position when the row count keeps them aligned)
        const bool quad_a = e0 + 3 < prm.m && (prm.m & 3) == 0;
        const bool quad_b = e0 >= prm.m && e0 + 3 < rows && (prm.m & 3) == 0 && (prm.p & 3) == 0;
        if (quad_a || quad_b) {
            float* N = quad_a ? ZS : WS;
            const int64_t R = quad_a ? prm.m : prm.p;
            const int64_t row = quad_a ? e0 : e0 - prm.m;
            for (int ip = 0; ip < kAdjPositions; ++ip)
                *reinterpret_cast<float4*>(N + (pos0 + ip) * R + row) =
                    make_float4(nrm[ip][0], nrm[ip][1], nrm[ip][2], nrm[ip][3]);
        } else {
            for (int r = 0; r < 4; ++r) {
                const int64_t e = e0 + r;
                if (e >= rows) break;
                const bool in_a = e < prm.m;
                float* N = in_a ? ZS : WS;
                const int64_t R = in_a ? prm.m : prm.p;
                const int64_t row = in_a ? e : e - prm.m;
                for (int ip = 0; ip < kAdjPositions; ++ip) N[(pos0 + ip) * R + row] = nrm[ip][r];
            }
        }
    }
}

// Draw t is one of the coarse draws of its level sample.
__device__ __forceinline__ bool coarse_draw(int t, uint32_t c_prev, uint32_t stride)
{
    return stride ? ((uint32_t)t + 1u) % stride == 0u : t < (int)c_prev;
}

struct AdjMfmaParams {
    int64_t m, p, kpad;
    uint32_t c_prev;
    uint32_t stride;                  // stride coupling M (0: prefix)
    float kappa_coarse, kappa_fine;   // (n / c_l) w_t / N_l for the two segments
    const float* GT;                  // p x m: G^T
    const float* G;                   // m x p
    const float* AT;                  // batch x m x kpad
    const float* BT;                  // batch x p x kpad
    const float* ZS;                  // batch x kpad x m
    const float* WS;                  // batch x kpad x p
    const int32_t* R;                 // batch x kpad
    int64_t tiles_t, tiles_u_cols, tiles_v_cols;
    float* dMA; float* dSA;           // n x m
    float* dMB; float* dSB;           // n x p
    const uint32_t* iw;               // index weights (NULL: uniform): factor 1 / (n xi_j) per draw
    const uint64_t* cum;
    uint32_t n;
};

// One 64 x 128 tile of U^T (rows t, columns i; K = p) or of V (rows t,
// columns q; K = m) for one realisation, then the scaled scatter-add.  Both
// operands are K-major ([k][t] and [k][x]); chunks of kAdjChunk k-values are
// staged in LDS with 16-byte loads, double-buffered so the next chunk's
// global loads are in flight during the MFMAs.  2 x 2 waves, each 32 x 64
// (two 32x32x2 f32 blocks sharing the t fragment).
constexpr int kAdjChunk = 32;
constexpr int kAdjTileT = 64, kAdjTileX = 128;

__global__ __launch_bounds__(kAdjThreads) void adjoint_mfma_kernel(AdjMfmaParams prm)
{
    constexpr int VA = kAdjChunk * kAdjTileT / 4 / kAdjThreads;   // uint4 per thread, t operand
    constexpr int VB = kAdjChunk * kAdjTileX / 4 / kAdjThreads;   // uint4 per thread, x operand
    __shared__ __align__(16) float lds_a[2][kAdjChunk * kAdjTileT];
    __shared__ __align__(16) float lds_b[2][kAdjChunk * kAdjTileX];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int64_t s = blockIdx.y;
    int64_t tile = blockIdx.x;
    const int64_t u_tiles = prm.tiles_t * prm.tiles_u_cols;
    const bool is_u = tile < u_tiles;
    if (!is_u) tile -= u_tiles;
    const int64_t cols_tiles = is_u ? prm.tiles_u_cols : prm.tiles_v_cols;
    const int tb = (int)(tile / cols_tiles) * kAdjTileT;     // first t of the tile
    const int xb = (int)(tile % cols_tiles) * kAdjTileX;     // first x of the tile
    const int wt = (wave / 2) * 32, wx = (wave % 2) * 64;    // wave tile inside the workgroup tile
    const int K = (int)(is_u ? prm.p : prm.m);               // contraction length
    const int X = (int)(is_u ? prm.m : prm.p);               // output columns
    const int kpad = (int)prm.kpad;
    // t operand [k][t] (row stride kpad): the transposed gathered operand of the other matrix
    const float* Aop = is_u ? prm.BT + s * prm.p * prm.kpad : prm.AT + s * prm.m * prm.kpad;
    // x operand [k][x] (row stride X): G^T (p x m) for U^T, G (m x p) for V
    const float* Bop = is_u ? prm.GT : prm.G;
    const bool vec_x = (X % 4) == 0;                         // 16-byte rows of the x operand

    float4 ra[VA], rb[VB];
    auto fetch = [&](int c) {
        const int k0 = c * kAdjChunk;
#pragma unroll
        for (int v = 0; v < VA; ++v) {
            const int vid = threadIdx.x + v * kAdjThreads;
            const int kk = vid / (kAdjTileT / 4), t = tb + (vid % (kAdjTileT / 4)) * 4;
            const int k = k0 + kk;
            // kpad is a multiple of 8, so a vector of 4 t values is whole or absent
            ra[v] = (k < K && t < kpad) ? *reinterpret_cast<const float4*>(Aop + (int64_t)k * kpad + t)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int v = 0; v < VB; ++v) {
            const int vid = threadIdx.x + v * kAdjThreads;
            const int kk = vid / (kAdjTileX / 4), x = xb + (vid % (kAdjTileX / 4)) * 4;
            const int k = k0 + kk;
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (k < K) {
                const float* row = Bop + (int64_t)k * X;
                if (vec_x && x < X) {
                    val = *reinterpret_cast<const float4*>(row + x);
                } else {
                    if (x < X) val.x = row[x];
                    if (x + 1 < X) val.y = row[x + 1];
                    if (x + 2 < X) val.z = row[x + 2];
                    if (x + 3 < X) val.w = row[x + 3];
                }
            }
            rb[v] = val;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int v = 0; v < VA; ++v)
            *reinterpret_cast<float4*>(&lds_a[buf][(threadIdx.x + v * kAdjThreads) * 4]) = ra[v];
#pragma unroll
        for (int v = 0; v < VB; ++v)
            *reinterpret_cast<float4*>(&lds_b[buf][(threadIdx.x + v * kAdjThreads) * 4]) = rb[v];
    };

    f32x16 acc[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[bj][r] = 0.0f;
    const int chunks = (K + kAdjChunk - 1) / kAdjChunk;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int c = 0; c < chunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < chunks) fetch(c + 1);
        const float* LA = lds_a[buf];
        const float* LB = lds_b[buf];
#pragma unroll 4
        for (int kk = 0; kk < kAdjChunk; kk += kAdjKStep) {
            const float a = LA[(kk + lane / 32) * kAdjTileT + wt + lane % 32];
            const float b0 = LB[(kk + lane / 32) * kAdjTileX + wx + lane % 32];
            const float b1 = LB[(kk + lane / 32) * kAdjTileX + wx + 32 + lane % 32];
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc[1], 0, 0, 0);
        }
        if (c + 1 < chunks) stash(buf ^ 1);
        __syncthreads();
    }
    // epilogue: lane l, register r holds row 8(r/4) + 4(l/32) + r%4, column l%32 of its block
    const int32_t* R = prm.R + s * prm.kpad;
    const float* N = is_u ? prm.ZS + s * prm.kpad * prm.m : prm.WS + s * prm.kpad * prm.p;
    float* dM = is_u ? prm.dMA : prm.dMB;
    float* dS = is_u ? prm.dSA : prm.dSB;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int x = xb + wx + bj * 32 + lane % 32;
        if (x >= X) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int t = tb + wt + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
            if (t >= kpad) continue;
            const int32_t col = R[t];
            if (col < 0) continue;
            float kappa = coarse_draw(t, prm.c_prev, prm.stride) ? prm.kappa_coarse : prm.kappa_fine;
            if (prm.iw) kappa *= (float)((double)prm.cum[prm.n - 1] / ((double)prm.n * (double)prm.iw[col]));
            const float g = kappa * acc[bj][r];
            unsafeAtomicAdd(dM + (int64_t)col * X + x, g);
            unsafeAtomicAdd(dS + (int64_t)col * X + x, g * N[(int64_t)t * X + x]);
        }
    }
}

// BF16 form of the same tiles: both operands are K-contiguous, so a lane's
// fragment (8 consecutive K of its row t or column x) is one 16-byte load
// from global memory (L2-resident: the values of one realisation and G),
// and v_mfma_f32_32x32x16_bf16 accumulates in FP32.  t operand: the
// position-major BF16 values of the other matrix ([t][K], row stride KS);
// x operand: G (for U^T, [i][q]) or G^T (for V, [q][i]) in BF16, stride KS.
// The accumulator layout is that of the FP32 kernel, so is the epilogue.
struct AdjBf16Params {
    int64_t m, p, kpad, mk, pk;
    uint32_t c_prev;
    uint32_t stride;
    float kappa_coarse, kappa_fine;
    const __bf16* Gb;                 // m x pk: G
    const __bf16* GTb;                // p x mk: G^T
    const __bf16* ASb;                // batch x kpad x mk
    const __bf16* BSb;                // batch x kpad x pk
    const float* ZS;                  // batch x kpad x m
    const float* WS;                  // batch x kpad x p
    const int32_t* R;                 // batch x kpad
    int64_t tiles_t, tiles_u_cols, tiles_v_cols;
    float* dMA; float* dSA;
    float* dMB; float* dSB;
    const uint32_t* iw;
    const uint64_t* cum;
    uint32_t n;
};

// 8 consecutive K values of one row (stride KS), zero beyond K or for an
// absent row; KS and k0 are multiples of 8, so the vector is aligned.
__device__ __forceinline__ bf16x8 adj_frag(const __bf16* base, int64_t row, bool row_ok, int k0, int K, int64_t KS)
{
    bf16x8 v;
    if (row_ok && k0 + 8 <= K) {
        v = *reinterpret_cast<const bf16x8*>(base + row * KS + k0);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (row_ok && k0 + i < K) ? base[row * KS + k0 + i] : (__bf16)0.0f;
    }
    return v;
}

__global__ __launch_bounds__(kAdjThreads) void adjoint_mfma_bf16_kernel(AdjBf16Params prm)
{
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int64_t s = blockIdx.y;
    int64_t tile = blockIdx.x;
    const int64_t u_tiles = prm.tiles_t * prm.tiles_u_cols;
    const bool is_u = tile < u_tiles;
    if (!is_u) tile -= u_tiles;
    const int64_t cols_tiles = is_u ? prm.tiles_u_cols : prm.tiles_v_cols;
    const int tb = (int)(tile / cols_tiles) * kAdjTileT;
    const int xb = (int)(tile % cols_tiles) * kAdjTileX;
    const int wt = (wave / 2) * 32, wx = (wave % 2) * 64;
    const int K = (int)(is_u ? prm.p : prm.m);
    const int X = (int)(is_u ? prm.m : prm.p);
    const int64_t KS = is_u ? prm.pk : prm.mk;
    const int kpad = (int)prm.kpad;
    const __bf16* Aop = is_u ? prm.BSb + s * prm.kpad * prm.pk : prm.ASb + s * prm.kpad * prm.mk;
    const __bf16* Bop = is_u ? prm.Gb : prm.GTb;
    const int t = tb + wt + lane % 32;
    const int x0 = xb + wx + lane % 32, x1 = x0 + 32;
    const bool t_ok = t < kpad, x0_ok = x0 < X, x1_ok = x1 < X;
    const int koff = 8 * (lane / 32);

    f32x16 acc[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[bj][r] = 0.0f;
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 16) {
        const bf16x8 a = adj_frag(Aop, t, t_ok, k0 + koff, K, KS);
        const bf16x8 b0 = adj_frag(Bop, x0, x0_ok, k0 + koff, K, KS);
        const bf16x8 b1 = adj_frag(Bop, x1, x1_ok, k0 + koff, K, KS);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc[1], 0, 0, 0);
    }
    const int32_t* R = prm.R + s * prm.kpad;
    const float* N = is_u ? prm.ZS + s * prm.kpad * prm.m : prm.WS + s * prm.kpad * prm.p;
    float* dM = is_u ? prm.dMA : prm.dMB;
    float* dS = is_u ? prm.dSA : prm.dSB;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int x = xb + wx + bj * 32 + lane % 32;
        if (x >= X) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int tt = tb + wt + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
            if (tt >= kpad) continue;
            const int32_t col = R[tt];
            if (col < 0) continue;
            float kappa = coarse_draw(tt, prm.c_prev, prm.stride) ? prm.kappa_coarse : prm.kappa_fine;
            if (prm.iw) kappa *= (float)((double)prm.cum[prm.n - 1] / ((double)prm.n * (double)prm.iw[col]));
            const float g = kappa * acc[bj][r];
            unsafeAtomicAdd(dM + (int64_t)col * X + x, g);
            unsafeAtomicAdd(dS + (int64_t)col * X + x, g * N[(int64_t)tt * X + x]);
        }
    }
}

// G and G^T in BF16 (round to nearest even), K-contiguous with padded strides
__global__ void grad_prepare_bf16_kernel(const double* grad, int64_t m, int64_t p, int64_t mk, int64_t pk,
                                         __bf16* Gb, __bf16* GTb)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * p) return;
    const int64_t i = e / p, q = e % p;
    const __bf16 v = (__bf16)(float)grad[e];
    Gb[i * pk + q] = v;
    GTb[q * mk + i] = v;
}

__global__ void grad_prepare_kernel(const double* grad, int64_t m, int64_t p, float* G, float* GT)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * p) return;
    const int64_t i = e / p, q = e % p;
    const float v = (float)grad[e];
    G[e] = v;
    GT[q * m + i] = v;
}

static int64_t round_up_adj(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Head of the workspace: G and G^T in FP32, then in BF16 (padded strides).
static size_t adj_head_bytes(int64_t m, int64_t p)
{
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t mk = round_up_adj(m, 8), pk = round_up_adj(p, 8);
    return align(2 * m * p * sizeof(float)) + align((size_t)(m * pk + p * mk) * sizeof(__bf16));
}

// Bytes per draw position of the gathered values of A (or B): FP32 K-major
// or BF16 position-major with the row padded to 8, whichever is larger.
static int64_t adj_value_bytes(int64_t rows)
{
    const int64_t f32 = 4 * rows, b16 = 2 * round_up_adj(rows, 8);
    return f32 > b16 ? f32 : b16;
}

size_t adjoint_workspace_size(int64_t m, int64_t n, int64_t p, int num_levels, const int64_t* c, bool weighted)
{
    const int64_t kpad = round_up_adj(c[num_levels - 1], kAdjPositions);
    const int64_t per_sample = kpad * (adj_value_bytes(m) + adj_value_bytes(p) + (m + p) * 4 + 4);
    int64_t budget = kAdjBudget < per_sample ? per_sample : kAdjBudget;
    // slack for the five 256-byte-aligned regions of a pass
    size_t total = (size_t)budget + 2048;
    total += adj_head_bytes(m, p);
    if (weighted) total += ((size_t)n * sizeof(uint64_t) + 255) & ~(size_t)255;
    return total;
}

hipError_t adjoint_run(int64_t m, int64_t n, int64_t p, const Law& A, const Law& B, int num_levels,
                       const int64_t* c, const int64_t* N, const StreamKeys& keys, bool shared,
                       const double* grad, float* dMA, float* dSA, float* dMB, float* dSB,
                       const uint32_t* index_weights, char* ws, size_t ws_bytes, bool bf16, bool stride,
                       bool value16, hipStream_t stream, KernelTimer* timer)
{
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t mk = round_up_adj(m, 8), pk = round_up_adj(p, 8);
    float* G = reinterpret_cast<float*>(ws);
    float* GT = G + m * p;
    __bf16* Gb = reinterpret_cast<__bf16*>(ws + align(2 * m * p * sizeof(float)));
    __bf16* GTb = Gb + m * pk;
    const size_t head = adj_head_bytes(m, p);
    // the cumulative index weights follow the head
    uint64_t* cum = index_weights ? reinterpret_cast<uint64_t*>(ws + head) : nullptr;
    const size_t cum_bytes = index_weights ? align((size_t)n * sizeof(uint64_t)) : 0;
    char* buf = ws + head + cum_bytes;
    const size_t budget = ws_bytes - head - cum_bytes;
    {
        ScopedTiming t(timer, 3);
        if (bf16)
            hipLaunchKernelGGL(grad_prepare_bf16_kernel, dim3((unsigned)ceil_div(m * p, 256)), dim3(256), 0, stream,
                               grad, m, p, mk, pk, Gb, GTb);
        else
            hipLaunchKernelGGL(grad_prepare_kernel, dim3((unsigned)ceil_div(m * p, 256)), dim3(256), 0, stream, grad,
                               m, p, G, GT);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (index_weights && (e = build_cumulative(index_weights, n, cum, stream)) != hipSuccess) return e;
    for (int l = 0; l < num_levels; ++l) {
        const int64_t cl = c[l], cp = l > 0 ? c[l - 1] : 0;
        const int64_t kpad = round_up_adj(cl, kAdjPositions);
        const size_t per_sample = (size_t)kpad * (adj_value_bytes(m) + adj_value_bytes(p) + (m + p) * 4 + 4) + 5 * 256;
        int64_t batch = (int64_t)(budget / per_sample);
        if (batch < 1) batch = 1;
        if (batch > 65535) batch = 65535;
        const double base = (double)n / (double)cl / (double)N[l];
        const float kc = (float)(base * (cp > 0 ? 1.0 - (double)cl / (double)cp : 1.0));
        const float kf = (float)base;
        for (int64_t b0 = 0; b0 < N[l]; b0 += batch) {
            const int64_t S = (N[l] - b0) < batch ? (N[l] - b0) : batch;
            size_t off = 0;
            // FP32: K-major AT, BT; BF16: position-major ASb, BSb in the same regions
            float* AT = reinterpret_cast<float*>(buf + off); off = align(off + (size_t)(S * kpad * adj_value_bytes(m)));
            float* BT = reinterpret_cast<float*>(buf + off); off = align(off + (size_t)(S * kpad * adj_value_bytes(p)));
            __bf16* ASb = reinterpret_cast<__bf16*>(AT);
            __bf16* BSb = reinterpret_cast<__bf16*>(BT);
            float* ZS = reinterpret_cast<float*>(buf + off); off = align(off + sizeof(float) * S * kpad * m);
            float* WS = reinterpret_cast<float*>(buf + off); off = align(off + sizeof(float) * S * kpad * p);
            int32_t* Rr = reinterpret_cast<int32_t*>(buf + off); off = align(off + sizeof(int32_t) * S * kpad);
            if (off > budget) return hipErrorInvalidValue;
            AdjGatherParams g;
            g.m = m; g.p = p; g.n = (uint32_t)n; g.c = (uint32_t)cl; g.c_prev = (uint32_t)cp; g.kpad = kpad;
            g.key0 = keys.key0; g.key1 = keys.key1;
            const uint32_t lf = shared ? 0xFFu : (uint32_t)l;
            g.sid_index = stream_id(kTagIndex, lf, keys.problem);
            g.sid_value = stream_id(kTagValue, lf, keys.problem);
            g.k_first = (uint32_t)b0;
            g.A = A; g.B = B;
            g.AT = AT; g.BT = BT; g.ZS = ZS; g.WS = WS; g.R = Rr;
            g.ASb = ASb; g.BSb = BSb; g.mk = mk; g.pk = pk;
            g.cum = cum;
            g.value16 = value16;
            {
                ScopedTiming t(timer, 1);
                const dim3 grid((unsigned)(kpad / kAdjPositions), (unsigned)S);
                if (bf16) hipLaunchKernelGGL(adjoint_gather_kernel<true>, grid, dim3(kAdjGatherThreads), 0, stream, g);
                else hipLaunchKernelGGL(adjoint_gather_kernel<false>, grid, dim3(kAdjGatherThreads), 0, stream, g);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if (bf16) {
                AdjBf16Params a;
                a.m = m; a.p = p; a.kpad = kpad; a.mk = mk; a.pk = pk; a.c_prev = (uint32_t)cp;
                a.stride = stride && cp > 0 ? (uint32_t)(cl / cp) : 0u;
                a.kappa_coarse = kc; a.kappa_fine = kf;
                a.Gb = Gb; a.GTb = GTb; a.ASb = ASb; a.BSb = BSb; a.ZS = ZS; a.WS = WS; a.R = Rr;
                a.tiles_t = ceil_div(kpad, kAdjTileT);
                a.tiles_u_cols = ceil_div(m, kAdjTileX);
                a.tiles_v_cols = ceil_div(p, kAdjTileX);
                a.dMA = dMA; a.dSA = dSA; a.dMB = dMB; a.dSB = dSB;
                a.iw = index_weights; a.cum = cum; a.n = (uint32_t)n;
                const int64_t tiles = a.tiles_t * (a.tiles_u_cols + a.tiles_v_cols);
                {
                    ScopedTiming t(timer, 0);
                    hipLaunchKernelGGL(adjoint_mfma_bf16_kernel, dim3((unsigned)tiles, (unsigned)S), dim3(kAdjThreads),
                                       0, stream, a);
                }
                if ((e = hipGetLastError()) != hipSuccess) return e;
                continue;
            }
            AdjMfmaParams a;
            a.m = m; a.p = p; a.kpad = kpad; a.c_prev = (uint32_t)cp;
            a.stride = stride && cp > 0 ? (uint32_t)(cl / cp) : 0u;
            a.kappa_coarse = kc; a.kappa_fine = kf;
            a.GT = GT; a.G = G; a.AT = AT; a.BT = BT; a.ZS = ZS; a.WS = WS; a.R = Rr;
            a.tiles_t = ceil_div(kpad, kAdjTileT);
            a.tiles_u_cols = ceil_div(m, kAdjTileX);
            a.tiles_v_cols = ceil_div(p, kAdjTileX);
            a.dMA = dMA; a.dSA = dSA; a.dMB = dMB; a.dSB = dSB;
            a.iw = index_weights; a.cum = cum; a.n = (uint32_t)n;
            const int64_t tiles = a.tiles_t * (a.tiles_u_cols + a.tiles_v_cols);
            {
                ScopedTiming t(timer, 0);
                hipLaunchKernelGGL(adjoint_mfma_kernel, dim3((unsigned)tiles, (unsigned)S), dim3(kAdjThreads), 0,
                                   stream, a);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace mlmc
