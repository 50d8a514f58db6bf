// Host-side interfaces between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "common.hpp"

namespace mlmc {

// One level's sample range as the launchers see it.
struct LevelRange {
    int level;             // l
    uint32_t level_field;  // l, or 0xFF in shared-sample mode
    int64_t c;             // c_l
    int64_t c_prev;        // c_{l-1}, 0 at level 0
    int64_t k_begin;       // first realisation
    int64_t count;         // number of realisations
    int64_t stride;        // stride coupling: M = c_l / c_{l-1} (the coarse draws are
                           // M - 1, 2M - 1, ...), 0: the first c_{l-1} draws
};

// Optional HIP-event timing of kernel launches, by kernel class (the
// MLMC_KERNEL_* classes of the C ABI).  Events come from a per-thread pool
// that grows on demand; elapsed times are read after the stream is synced.
class KernelTimer {
public:
    explicit KernelTimer(hipStream_t s) : stream_(s) {}
    void begin(int cls);
    void end();
    // Sums elapsed milliseconds and launch counts per class; the stream must
    // have been synchronised.
    void collect(double* ms, int64_t* launches) const;

private:
    hipStream_t stream_;
    int open_cls_ = -1;
    size_t used_ = 0;
    std::vector<int> classes_;
};

struct ScopedTiming {
    ScopedTiming(KernelTimer* t, int cls) : t_(t) { if (t_) t_->begin(cls); }
    ~ScopedTiming() { if (t_) t_->end(); }
    KernelTimer* t_;
};

// Index weights of a call (eq. (18) with a general xi): w is NULL for
// uniform draws; cum is the library's cumulative table in workspace.
struct IndexWeights {
    const uint32_t* w;
    const uint64_t* cum;
};

struct StreamKeys {
    uint32_t key0, key1;
    uint32_t problem;
};

// ---- inner product (m = p = 1) -------------------------------------------
// Device state per level: one Moments (count, mean, M2) of the level samples.
size_t inner_partials_capacity();  // Moments slots needed in workspace
struct InnerSlot;                   // a launch's parameters in device memory
size_t inner_slot_bytes();
// One launch over every level's range (pilot, extension or fixed mode), then a
// fold of the workgroup partials into the running level states.
// index_word32: four index draws per Philox call from 32-bit words (n a power
// of two, uniform draws, no experiment laws: checked by the caller).
// Where a phase's fold writes the estimate (the last phase of a fixed or
// target-mode estimate): Y, the level means (nullable) and V_l.
struct InnerTelescope {
    double* out;
    double* level_means;
    double* level_var;
};
// One phase over every level's range: its parameters stored into the slot by
// a kernel (zero_state: the level states cleared first), the level launch, and
// a one-workgroup fold of the partials into the level states (with tele, then
// the telescoping sum).
hipError_t inner_levels_run(const LevelRange* ranges, int num_levels, int64_t n, const Law& x,
                            const Law& y, const TargetFunc& f, const IndexWeights& iw, int prec,
                            bool index_word32, const StreamKeys& keys, Moments* partials, Moments* level_state,
                            InnerSlot* slot, bool zero_state, const InnerTelescope* tele, hipStream_t stream,
                            KernelTimer* timer);
// Target mode with no host synchronisation: the pilot (pilot ranges, level
// states cleared), its fold, which evaluates eq. (28) on the device from the
// level states (schedule_counts, the host's arithmetic) and writes the
// extension's partition into the slot, the extension of every level to
// max(N_l, pilot) realisations, and the last fold with the telescoping sum.
// counts (device, num_levels) receives the realisations of every level
// after it, status (device) the schedule's code and failing level (the
// extension is empty when it is not 0), status_value the offending number.
struct InnerScheduleInputs {
    double eps;
    int64_t pilot, max_total_draws;
    const int64_t* c;                    // host, num_levels
    uint32_t level_field[32], stride[32];
    int64_t* counts;
    int32_t* status;
    double* status_value;
};
hipError_t inner_target_run(const InnerScheduleInputs& s, const LevelRange* pilot, int num_levels, int64_t n,
                            const Law& x, const Law& y, const TargetFunc& f, const IndexWeights& iw, int prec,
                            bool index_word32, const StreamKeys& keys, Moments* partials, Moments* level_state,
                            InnerSlot* slot, const InnerTelescope& tele, hipStream_t stream, KernelTimer* timer);
hipError_t inner_telescope(const Moments* level_state, int num_levels, double* out,
                           double* level_means, double* level_var, hipStream_t stream);

// ---- matrix product ----------------------------------------------------------
// One product of a table; a single estimate is the one-entry table.
struct MatmulProblem {
    int64_t m, n, p;
    Law A, B;
    uint32_t problem;          // Philox stream id
    double* out;               // device m x p
    double* level_means;       // device (L+1) x m x p, or null
};

struct MatmulTuning {
    int tile;                  // workgroup output tile edge (0: default)
    int64_t target_blocks;     // sketch work items per pass (0: default)
    int64_t gather_budget;     // bytes of gathered operands per pass (0: default)
    int single_launch;         // 1: the persistent single-launch form where it is built
};

// Device-side description of one product of the table.
struct ProblemDesc {
    int64_t m, n, p;
    int64_t m_pad, p_pad;      // gathered row counts, padded to the workgroup tile
    Law A, B;
    uint32_t sid_problem;
    int64_t tiles_n, tiles, tile_first;
    int64_t rows_prefix;       // sum of (m_pad + p_pad) over earlier products
    int64_t mp_prefix;         // sum of m p over earlier products
    int64_t merge_blocks, between_prefix;
    float pre_a, pre_b;        // FP8, i.i.d. laws: the row (column) factor 2^s folded into the law's constants, else 1
    const int8_t* exp_a;       // FP8: exponent s of the factor 2^s of every row of A (m_pad) ...
    const int8_t* exp_b;       // ... and column of B (p_pad), in workspace; NULL otherwise
    double mean0;              // E[Z_0] entry for i.i.d. laws: n E[a] E[b]
    double* out;
    double* level_means;
};

// One pass of the single-launch (persistent) form of a fixed-N_l estimate: a
// batch of realisations of one level, gathered in one phase of the launch and
// sketched in the next.
struct PassDesc {
    int32_t level;
    int32_t stats;             // the sketch's statistics form: 2 shifted sums, 3 two accumulators
    uint32_t c, c_prev, stride, level_field;
    uint32_t k_first;          // realisation of the batch's first slot
    int32_t octets;            // gather position groups per unit
    int64_t kc, kpad, batch;
    int64_t gx;                // gather units along the positions
    int64_t units;             // gx * batch * nprob
    double done_before;        // realisations of the level merged by earlier passes
    double omega;              // 1 - c_l / c_{l-1}: the coarse draws' weight (1 at level 0)
};

struct MatmulPlan {
    int prec;
    int num_levels;
    int64_t c[32];
    int nprob;
    int kstep, kpack, elem, nb, tile;
    int kmem;                  // shortest padded realisation (a divisor of kstep)
    int laws;                  // law pair shared by every product (kLaws*), else kLawsAny
    TargetFunc func;           // f of E[f(AB)]; not the identity: both sketches kept (tile 64)
    const uint32_t* index_weights;   // NULL: uniform draws
    size_t off_cum;                  // the cumulative weights (n uint64) when index_weights is set
    bool iid;                  // no product has a reparameterised law
    bool value16 = false;      // values from 16-bit uniforms (eight per Philox call)
    bool whole_tiles;          // every m and p is a multiple of the workgroup tile
    int64_t min_rows;          // smallest m + p over the products
    int64_t kpad_max;
    int64_t sum_rows, sum_mp, sum_merge_blocks, total_tiles, max_mp, max_merge_blocks;
    int64_t groups_max, gather_bytes, state_doubles;
    size_t off_means, off_between, off_within, off_tile_acc, off_var, off_norm, off_desc, off_tile_owner,
        off_gather, off_part_mean, off_part_m2, total;
    std::vector<ProblemDesc> descs;
    std::vector<int32_t> tile_owner;
    // FP8: the exponents of the rows of A and columns of B, product after
    // product (m_pad then p_pad entries at rows_prefix); reparameterised
    // operands' entries are filled on the device by matmul_reset
    std::vector<int8_t> exp_host;
    bool fp8_reparam = false;
    size_t off_exp = 0, off_bound = 0;
    // the single-launch form (matmul_plan_persistent): its passes, their
    // table and step counters in workspace, and the second and third gather
    // buffers
    bool persistent = false;
    std::vector<PassDesc> passes;
    size_t off_passes = 0, off_sync = 0, off_gather2 = 0, off_gather3 = 0;
    int64_t sync_words = 0;
    // the set form of a realisation (matmul_plan_set_form): per-realisation
    // hash tables and position weights in workspace
    bool set_form = false;
    size_t off_set = 0;
    int64_t set_bytes = 0;
};

// index_weights: NULL, or (one product) the device weights whose cumulative
// table the plan keeps in workspace (off_cum)
bool matmul_plan(const MatmulProblem* probs, int nprob, int prec, int num_levels, const int64_t* c,
                 const MatmulTuning* tune, const TargetFunc& func, const uint32_t* index_weights,
                 MatmulPlan& plan);
// copies the problem table into the workspace (synchronises `stream`)
hipError_t matmul_upload(const MatmulPlan& plan, char* ws, hipStream_t stream);
// zeroes the level state; FP8 with reparameterised laws: the operand
// exponents from the current means and scales
hipError_t matmul_reset(const MatmulPlan& plan, char* ws, hipStream_t stream);
hipError_t matmul_level_run(const MatmulPlan& plan, const LevelRange& lr, int64_t done_before,
                            const StreamKeys& keys, char* ws, hipStream_t stream, KernelTimer* timer);
// The single-launch form of a fixed-N_l estimate (ranges: each level's
// realisations): every level's passes run in one persistent kernel whose
// phase p gathers pass p while it sketches pass p - 1.  Sets plan.persistent
// when the plan's form has such a kernel (FP32, BF16 or FP8 operands, i.i.d.
// normal or uniform laws, f = identity, uniform draws, products in whole
// tiles at tile 64 or of any shape at tile 128) and then lays out its
// workspace after plan.total (the pass table is copied by matmul_upload).
void matmul_plan_persistent(MatmulPlan& plan, const LevelRange* ranges, int num_levels);
// The set form of every realisation (the note after Alg. 1 in Sec. 3.1): the
// index tuple is mapped to its distinct indices with their multiplicities
// before the gather, each distinct column is generated once, at the first
// position that drew it, weighted by the sum of the weights of the draws that
// took it, and the other positions are left zero.  f = identity, uniform
// draws, FP64 / FP32 operands (checked by the caller).  Lays out the tables
// after plan.total; the passes then also bound their batch by that region.
void matmul_plan_set_form(MatmulPlan& plan);
// Runs the planned passes: one fill of the phase counters and one launch.
hipError_t matmul_persistent_run(const MatmulPlan& plan, const StreamKeys& keys, char* ws, hipStream_t stream,
                                 KernelTimer* timer);
// Non-zero when a launch of the single-launch form gave up on a phase barrier
// (its workgroups were not all resident); reads the flag (synchronises).
hipError_t matmul_persistent_status(const MatmulPlan& plan, char* ws, hipStream_t stream, bool* failed);
// V_l of every product (levels x nprob at matmul_level_var_ptr); with
// write_outputs, also the telescoping sums and level means
hipError_t matmul_finalize(const MatmulPlan& plan, const int64_t* counts, char* ws, bool write_outputs,
                           hipStream_t stream);
double* matmul_level_var_ptr(const MatmulPlan& plan, char* ws);
// ||Ybar_level||_F^2 of the first product into matmul_norm_ptr (device)
hipError_t matmul_level_norm2(const MatmulPlan& plan, char* ws, int level, hipStream_t stream);
double* matmul_norm_ptr(const MatmulPlan& plan, char* ws);

hipError_t fill_doubles(double* p, int64_t count, double v, hipStream_t stream);

// ---- adjoint of the matrix estimator (reparameterised laws) ---------------
// N: the forward's N_l (NULL: the largest size any N_l can need)
size_t adjoint_workspace_size(int64_t m, int64_t n, int64_t p, int num_levels, const int64_t* c, const int64_t* N,
                              bool weighted);
// The least workspace the adjoint runs with (passes of 64 draws).
size_t adjoint_workspace_min(int64_t m, int64_t n, int64_t p, bool weighted);
hipError_t adjoint_run(int64_t m, int64_t n, int64_t p, const Law& A, const Law& B, int num_levels,
                       const int64_t* c, const int64_t* N, const StreamKeys& keys, bool shared,
                       const double* grad, float* dMA, float* dSA, float* dMB, float* dSB,
                       const uint32_t* index_weights, char* ws, size_t ws_bytes, bool bf16, bool stride,
                       bool value16, hipStream_t stream, KernelTimer* timer);

// ---- building blocks exported for tests -----------------------------------
hipError_t philox_batch(int64_t count, const uint32_t* ctr, uint32_t key0, uint32_t key1,
                        uint32_t* out, hipStream_t stream);
hipError_t sample_indices(const StreamKeys& keys, uint32_t level_field, uint32_t k0,
                          int64_t num_samples, int64_t c, int64_t n, int32_t* out,
                          hipStream_t stream);
// cum[j] = w_0 + ... + w_j (one workgroup, exact integer sums)
hipError_t build_cumulative(const uint32_t* w, int64_t n, uint64_t* cum, hipStream_t stream);
hipError_t sample_indices_weighted(const StreamKeys& keys, uint32_t level_field, uint32_t k0,
                                   int64_t num_samples, int64_t c, int64_t n, const uint64_t* cum, int32_t* out,
                                   hipStream_t stream);
// Theorem 3.1's xi** as integer weights; scratch: n + 1 doubles
hipError_t optimal_weights(int64_t m, int64_t n, int64_t p, const Law& A, const Law& B, uint32_t* w,
                           double* scratch, hipStream_t stream);
hipError_t gather_columns_f64(int64_t m, int64_t n, int64_t p, const Law& A, const Law& B,
                              const StreamKeys& keys, uint32_t level_field, uint32_t k0,
                              int64_t num_samples, int64_t c, int prec, double* AS, double* BS,
                              hipStream_t stream);

}  // namespace mlmc
