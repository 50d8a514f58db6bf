// C ABI of the MLMC library: validation, workspace layout, and the driver of
// Alg. 2 for a fixed finest level L (fixed N_l, or pilot -> eq. (28) ->
// extension for a target RMSE).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "mlmc.h"

using namespace mlmc;

namespace {

thread_local std::string g_last_error;
thread_local std::vector<hipEvent_t> g_event_pool;

mlmc_status fail(mlmc_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

mlmc_status device_fail(hipError_t e, const char* what)
{
    return fail(MLMC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr int64_t kU32 = int64_t(1) << 32;

mlmc_status check_levels(const mlmc_levels* lv, bool inner)
{
    if (!lv) return fail(MLMC_EINVAL, "levels is NULL");
    if (lv->num_levels < 1 || lv->num_levels > MLMC_MAX_LEVELS)
        return fail(MLMC_EINVAL, "num_levels must be in [1, %d]", MLMC_MAX_LEVELS);
    if (!lv->c) return fail(MLMC_EINVAL, "ladder c is NULL");
    if (lv->c[0] < 1) return fail(MLMC_EINVAL, "c[0] must be >= 1");
    for (int l = 1; l < lv->num_levels; ++l) {
        if (lv->c[l] < 2 * lv->c[l - 1] || lv->c[l] % lv->c[l - 1] != 0)
            return fail(MLMC_EINVAL, "c[%d] = %lld is not an integer multiple >= 2 of c[%d] = %lld", l,
                        (long long)lv->c[l], l - 1, (long long)lv->c[l - 1]);
    }
    // below 2^31, every 32-bit count of draws, pairs, quads and padded K
    // positions the kernels form from c stays in range
    if (lv->c[lv->num_levels - 1] >= ((int64_t)1 << 31)) return fail(MLMC_EINVAL, "c_L must be < 2^31");
    // matrix products: the gather grid has 8 lanes per padded K position in
    // one 32-bit launch dimension, and a pass's padded positions are counted
    // in 32 bits; c_L < 2^28 keeps both in range
    if (!inner && lv->c[lv->num_levels - 1] >= ((int64_t)1 << 28))
        return fail(MLMC_EINVAL, "matrix products need c_L < 2^28");
    if (lv->prec < MLMC_PREC_FP64 || lv->prec > (inner ? MLMC_PREC_FP32 : MLMC_PREC_FP8))
        return fail(MLMC_EINVAL, "unsupported precision %d", lv->prec);
    if (lv->problem >= (1u << 20)) return fail(MLMC_EINVAL, "problem id must be < 2^20");
    if (lv->rmse_target > 0.0) {
        if (lv->n_samples) return fail(MLMC_EINVAL, "give either n_samples or rmse_target, not both");
        if (lv->pilot_samples < 2 || lv->pilot_samples >= kU32)
            return fail(MLMC_EINVAL, "target mode needs 2 <= pilot_samples < 2^32");
        if (!isfinite(lv->rmse_target)) return fail(MLMC_EINVAL, "rmse_target must be finite");
    } else {
        if (!lv->n_samples) return fail(MLMC_EINVAL, "fixed mode needs n_samples (or rmse_target > 0)");
        for (int l = 0; l < lv->num_levels; ++l)
            if (lv->n_samples[l] < 1 || lv->n_samples[l] >= kU32)
                return fail(MLMC_EINVAL, "n_samples[%d] must be in [1, 2^32)", l);
    }
    if (lv->max_total_draws < 0) return fail(MLMC_EINVAL, "max_total_draws must be >= 0");
    if (lv->index_weights && lv->prec == MLMC_PREC_FP8)
        return fail(MLMC_EINVAL, "weighted index draws are not offered with FP8 operands");
    if ((lv->flags & MLMC_FLAG_VALUE16) && inner)
        return fail(MLMC_EINVAL, "16-bit value uniforms are offered for matrix products");
    if ((lv->flags & MLMC_FLAG_INDEX_WORD32) && (!inner || lv->index_weights))
        return fail(MLMC_EINVAL, "32-bit index words are offered for uniform draws of the inner product");
    if ((lv->flags & MLMC_FLAG_ADAPTIVE_LEVELS) && !(lv->rmse_target > 0.0))
        return fail(MLMC_EINVAL, "the adaptive number of levels needs target mode (rmse_target > 0)");
    if (lv->func < MLMC_FUNC_IDENTITY || lv->func > MLMC_FUNC_INV_ABS_STEP)
        return fail(MLMC_EINVAL, "unknown target function %d", lv->func);
    if (lv->func != MLMC_FUNC_IDENTITY && (!isfinite(lv->func_param[0]) || !isfinite(lv->func_param[1])))
        return fail(MLMC_EINVAL, "target function parameters must be finite");
    if (lv->func == MLMC_FUNC_INV_ABS_STEP && !(lv->func_param[1] > 0.0))
        return fail(MLMC_EINVAL, "1 / (|x| H(x + theta0) + theta1) needs theta1 > 0");
    if (lv->flags & MLMC_FLAG_SET_FORM) {
        if (inner) return fail(MLMC_EINVAL, "the set form is offered for matrix products");
        if (lv->prec != MLMC_PREC_FP64 && lv->prec != MLMC_PREC_FP32)
            return fail(MLMC_EINVAL, "the set form takes FP64 or FP32 operands");
        if (lv->func != MLMC_FUNC_IDENTITY) return fail(MLMC_EINVAL, "the set form takes f = identity");
        if (lv->index_weights) return fail(MLMC_EINVAL, "the set form takes uniform index draws");
    }
    return MLMC_OK;
}

mlmc_status check_dist(const mlmc_dist* d, const char* name, int64_t min_ld, bool inner)
{
    if (!d) return fail(MLMC_EINVAL, "%s is NULL", name);
    if (d->law < MLMC_LAW_NORMAL || d->law > MLMC_LAW_COS_POISSON_STEP)
        return fail(MLMC_EINVAL, "%s: unknown law", name);
    if (d->law == MLMC_LAW_COS_POISSON_EXP || d->law == MLMC_LAW_COS_POISSON_STEP) {
        // exp(-loc) stays a normal FP64 number and the CDF walk ends well
        // inside its 1000 terms
        if (!(d->loc > 0.0 && d->loc <= 500.0)) return fail(MLMC_EINVAL, "%s: Poisson rate must be in (0, 500]", name);
        if (!(d->scale >= 0.0 && d->scale <= 1.0))
            return fail(MLMC_EINVAL, "%s: Bernoulli rate must be in [0, 1]", name);
    } else if (d->law == MLMC_LAW_REPARAM) {
        if (!d->mean || !d->stdev) return fail(MLMC_EINVAL, "%s: reparam law needs mean and stdev", name);
        if (!inner && d->ld < min_ld) return fail(MLMC_EINVAL, "%s: ld must be >= %lld", name, (long long)min_ld);
    } else if (!isfinite(d->loc) || !isfinite(d->scale)) {
        return fail(MLMC_EINVAL, "%s: loc and scale must be finite", name);
    }
    return MLMC_OK;
}

// The laws of Sec. 4 pair only with each other (their gather is a kernel of
// its own) and are not offered with FP8 operands.
mlmc_status check_pair(const mlmc_dist* a, const mlmc_dist* b, int32_t prec, uint32_t flags = 0)
{
    const bool ea = a->law >= MLMC_LAW_RAMP_NORMAL, eb = b->law >= MLMC_LAW_RAMP_NORMAL;
    if (ea != eb) return fail(MLMC_EINVAL, "the laws of the experiments pair only with each other");
    if (ea && prec == MLMC_PREC_FP8) return fail(MLMC_EINVAL, "the laws of the experiments are not offered with FP8");
    if (ea && (flags & MLMC_FLAG_VALUE16))
        return fail(MLMC_EINVAL, "the laws of the experiments have their own stream (no 16-bit values)");
    return MLMC_OK;
}

Law to_law(const mlmc_dist& d)
{
    Law l;
    l.kind = d.law;
    l.loc = d.loc;
    l.scale = d.scale;
    l.mean = d.mean;
    l.stdev = d.stdev;
    l.ld = d.ld;
    // first term of the Poisson CDF walk, exp(-lambda), on the host
    l.aux = (d.law == MLMC_LAW_COS_POISSON_EXP || d.law == MLMC_LAW_COS_POISSON_STEP) ? exp(-d.loc) : 0.0;
    return l;
}

TargetFunc func_of(const mlmc_levels* lv)
{
    return TargetFunc{lv->func, lv->func_param[0], lv->func_param[1]};
}

StreamKeys keys_of(const mlmc_levels* lv)
{
    StreamKeys k;
    k.key0 = (uint32_t)lv->seed;
    k.key1 = (uint32_t)(lv->seed >> 32);
    k.problem = lv->problem;
    return k;
}

// The status of eq. (28)'s schedule_counts as a C ABI status.
mlmc_status schedule_status(const mlmc_levels* lv, int code, int bad_level, double bad_value)
{
    if (code == 1)
        return fail(MLMC_EBUDGET, "scheduled N_%d = %g exceeds the realisation counter range", bad_level, bad_value);
    if (code == 2)
        return fail(MLMC_EBUDGET, "scheduled draws %.6g exceed max_total_draws %lld", bad_value,
                    (long long)lv->max_total_draws);
    return MLMC_OK;
}

// eq. (28) over levels 0 .. nlev - 1 on the host
mlmc_status schedule(const mlmc_levels* lv, const double* var, int nlev, int64_t* n_out)
{
    int bad_level = 0;
    double bad_value = 0.0;
    const int code = schedule_counts(lv->rmse_target, lv->c, var, nlev, lv->pilot_samples, lv->max_total_draws,
                                     n_out, &bad_level, &bad_value);
    return schedule_status(lv, code, bad_level, bad_value);
}

// The bias test of the adaptive loop on the finest level mean so far (its
// Frobenius norm, or absolute value for the inner product).
bool bias_test(const mlmc_levels* lv, int L, double norm, bool inner)
{
    const double M = (double)lv->c[L] / (double)lv->c[L - 1];
    return norm < (sqrt(M) + (inner ? -1.0 : 1.0)) * lv->rmse_target / sqrt(2.0);
}

void fill_report(const mlmc_levels* lv, const int64_t* counts, const double* var, const KernelTimer* timer,
                 mlmc_report* rep, int levels_used, bool passed)
{
    for (int i = 0; i < MLMC_KERNEL_CLASSES; ++i) {
        rep->kernel_ms[i] = 0.0;
        rep->kernel_launches[i] = 0;
    }
    if (timer) timer->collect(rep->kernel_ms, rep->kernel_launches);
    double s = 0.0;
    int64_t draws = 0;
    for (int l = 0; l < MLMC_MAX_LEVELS; ++l) {
        rep->n_used[l] = l < lv->num_levels ? counts[l] : 0;
        rep->level_var[l] = l < lv->num_levels ? var[l] : 0.0;
    }
    for (int l = 0; l < lv->num_levels; ++l) {
        if (counts[l] > 0) s += var[l] / (double)counts[l];
        draws += counts[l] * lv->c[l];
    }
    rep->rmse_est = sqrt(s);
    rep->total_draws = draws;
    rep->levels_used = levels_used;
    rep->bias_test_passed = passed ? 1 : 0;
}

LevelRange range_of(const mlmc_levels* lv, int l, int64_t k_begin, int64_t count)
{
    LevelRange r;
    r.level = l;
    r.level_field = (lv->flags & MLMC_FLAG_SHARED_SAMPLES) ? 0xFFu : (uint32_t)l;
    r.c = lv->c[l];
    r.c_prev = l > 0 ? lv->c[l - 1] : 0;
    r.k_begin = k_begin;
    r.count = count;
    r.stride = (lv->flags & MLMC_FLAG_STRIDE_COUPLING) && l > 0 ? lv->c[l] / lv->c[l - 1] : 0;
    return r;
}

// Inner-product workspace: per-level Moments, workgroup partials, V_l, and
// the cumulative index weights when the draws are weighted.
struct InnerLayout {
    size_t off_state, off_partials, off_var, off_cum, off_slot, off_counts, off_status, total;
};

InnerLayout inner_layout(int num_levels, int64_t n, bool weighted)
{
    InnerLayout L;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    L.off_state = 0;
    L.off_partials = align(sizeof(Moments) * num_levels);
    // V_l, then the scheduled counts and the schedule's status: one readback
    L.off_var = align(L.off_partials + sizeof(Moments) * inner_partials_capacity());
    L.off_counts = L.off_var + sizeof(double) * num_levels;
    L.off_status = L.off_counts + sizeof(int64_t) * num_levels;
    L.off_cum = align(L.off_status + 2 * sizeof(int32_t) + sizeof(double));
    L.off_slot = align(L.off_cum + (weighted ? sizeof(uint64_t) * n : 0));
    L.total = align(L.off_slot + inner_slot_bytes());
    return L;
}

}  // namespace

namespace mlmc {

void KernelTimer::begin(int cls)
{
    open_cls_ = -1;
    while (g_event_pool.size() < 2 * (used_ + 1)) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return;
        g_event_pool.push_back(ev);
    }
    if (hipEventRecord(g_event_pool[2 * used_], stream_) != hipSuccess) return;
    open_cls_ = cls;
}

void KernelTimer::end()
{
    if (open_cls_ < 0) return;
    if (hipEventRecord(g_event_pool[2 * used_ + 1], stream_) == hipSuccess) {
        classes_.push_back(open_cls_);
        ++used_;
    }
    open_cls_ = -1;
}

void KernelTimer::collect(double* ms, int64_t* launches) const
{
    for (size_t i = 0; i < used_; ++i) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, g_event_pool[2 * i], g_event_pool[2 * i + 1]) != hipSuccess) continue;
        ms[classes_[i]] += (double)t;
        launches[classes_[i]] += 1;
    }
}

}  // namespace mlmc

namespace {

// Arguments of an inner-product estimate, checked before any device call.
mlmc_status check_inner(int64_t n, const mlmc_dist* x, const mlmc_dist* y, const mlmc_levels* lv,
                        const double* out, const void* workspace, size_t workspace_bytes)
{
    if (n < 1 || n >= kU32) return fail(MLMC_EINVAL, "n must be in [1, 2^32)");
    mlmc_status st = check_levels(lv, true);
    if (st != MLMC_OK) return st;
    if ((st = check_dist(x, "x", 1, true)) != MLMC_OK) return st;
    if ((st = check_dist(y, "y", 1, true)) != MLMC_OK) return st;
    if ((st = check_pair(x, y, lv->prec)) != MLMC_OK) return st;
    if ((lv->flags & MLMC_FLAG_INDEX_WORD32) && ((n & (n - 1)) != 0 || x->law >= MLMC_LAW_RAMP_NORMAL))
        return fail(MLMC_EINVAL, "32-bit index words need a power-of-two n and laws 0-2");
    if (!out) return fail(MLMC_EINVAL, "out is NULL");
    const InnerLayout L = inner_layout(lv->num_levels, n, lv->index_weights != nullptr);
    if (!workspace || workspace_bytes < L.total) return fail(MLMC_EWORKSPACE, "workspace needs %zu bytes", L.total);
    return MLMC_OK;
}

// The device work of a non-adaptive inner-product estimate: fixed N_l, or
// target mode (the pilot, eq. (28) on the device, the extension).  Launches
// only, no synchronisation: a stream capture records all of it.
hipError_t inner_enqueue(int64_t n, const mlmc_dist* x, const mlmc_dist* y, const mlmc_levels* lv, double* out,
                         double* level_means, char* ws, hipStream_t stream, KernelTimer* timer)
{
    const InnerLayout L = inner_layout(lv->num_levels, n, lv->index_weights != nullptr);
    Moments* state = reinterpret_cast<Moments*>(ws + L.off_state);
    Moments* partials = reinterpret_cast<Moments*>(ws + L.off_partials);
    double* var_dev = reinterpret_cast<double*>(ws + L.off_var);
    InnerSlot* slot = reinterpret_cast<InnerSlot*>(ws + L.off_slot);
    const IndexWeights iw{lv->index_weights,
                          lv->index_weights ? reinterpret_cast<const uint64_t*>(ws + L.off_cum) : nullptr};
    hipError_t e = hipSuccess;
    if (iw.w) {
        ScopedTiming t(timer, MLMC_KERNEL_FINAL);
        if ((e = build_cumulative(iw.w, n, reinterpret_cast<uint64_t*>(ws + L.off_cum), stream)) != hipSuccess)
            return e;
    }
    const Law lx = to_law(*x), ly = to_law(*y);
    const StreamKeys keys = keys_of(lv);
    const int L1 = lv->num_levels;
    const bool word32 = (lv->flags & MLMC_FLAG_INDEX_WORD32) != 0;
    const InnerTelescope tele{out, level_means, var_dev};
    if (lv->rmse_target > 0.0) {
        InnerScheduleInputs sch;
        sch.eps = lv->rmse_target;
        sch.pilot = lv->pilot_samples;
        sch.max_total_draws = lv->max_total_draws;
        sch.c = lv->c;
        LevelRange pilot[MLMC_MAX_LEVELS];
        for (int l = 0; l < L1; ++l) {
            pilot[l] = range_of(lv, l, 0, lv->pilot_samples);
            sch.level_field[l] = pilot[l].level_field;
            sch.stride[l] = (uint32_t)pilot[l].stride;
        }
        sch.counts = reinterpret_cast<int64_t*>(ws + L.off_counts);
        sch.status = reinterpret_cast<int32_t*>(ws + L.off_status);
        sch.status_value = reinterpret_cast<double*>(ws + L.off_status + 2 * sizeof(int32_t));
        return inner_target_run(sch, pilot, L1, n, lx, ly, func_of(lv), iw, lv->prec, word32, keys, partials, state,
                                slot, tele, stream, timer);
    }
    LevelRange ranges[MLMC_MAX_LEVELS];
    for (int l = 0; l < L1; ++l) ranges[l] = range_of(lv, l, 0, lv->n_samples[l]);
    return inner_levels_run(ranges, L1, n, lx, ly, func_of(lv), iw, lv->prec, word32, keys, partials, state, slot,
                            true, &tele, stream, timer);
}

// V_l and N_l of a non-adaptive estimate that has been enqueued on `stream`
// (synchronises it), and in target mode the schedule's status: one readback
// of V_l, N_l and the status, which lie in that order in the workspace.
mlmc_status inner_collect(int64_t n, const mlmc_levels* lv, const char* ws, hipStream_t stream, double* var,
                          int64_t* counts)
{
    const InnerLayout L = inner_layout(lv->num_levels, n, lv->index_weights != nullptr);
    const int L1 = lv->num_levels;
    hipError_t e = hipSuccess;
    if (lv->rmse_target <= 0.0) {
        if ((e = hipMemcpyAsync(var, ws + L.off_var, sizeof(double) * L1, hipMemcpyDeviceToHost, stream)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return device_fail(e, "level variance readback");
        for (int l = 0; l < L1; ++l) counts[l] = lv->n_samples[l];
        return MLMC_OK;
    }
    std::vector<char> back(sizeof(double) * L1 + sizeof(int64_t) * L1 + 2 * sizeof(int32_t) + sizeof(double));
    if ((e = hipMemcpyAsync(back.data(), ws + L.off_var, back.size(), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return device_fail(e, "schedule readback");
    memcpy(var, back.data(), sizeof(double) * L1);
    memcpy(counts, back.data() + sizeof(double) * L1, sizeof(int64_t) * L1);
    int32_t code[2];
    double value;
    memcpy(code, back.data() + 16 * L1, sizeof(code));
    memcpy(&value, back.data() + 16 * L1 + sizeof(code), sizeof(value));
    return schedule_status(lv, code[0], code[1], value);
}

}  // namespace

extern "C" {

const char* mlmc_status_string(mlmc_status st)
{
    switch (st) {
    case MLMC_OK: return "MLMC_OK";
    case MLMC_EINVAL: return "MLMC_EINVAL";
    case MLMC_EDEVICE: return "MLMC_EDEVICE";
    case MLMC_EBUDGET: return "MLMC_EBUDGET";
    case MLMC_EWORKSPACE: return "MLMC_EWORKSPACE";
    }
    return "unknown mlmc_status";
}

const char* mlmc_last_error(void) { return g_last_error.c_str(); }

size_t mlmc_inner_product_workspace_size(int64_t n, const mlmc_levels* levels)
{
    (void)n;
    if (!levels || levels->num_levels < 1 || levels->num_levels > MLMC_MAX_LEVELS) return 0;
    return inner_layout(levels->num_levels, n, levels->index_weights != nullptr).total;
}

size_t mlmc_matmul_workspace_size(int64_t m, int64_t n, int64_t p, const mlmc_levels* levels)
{
    if (check_levels(levels, false) != MLMC_OK || m < 1 || p < 1 || n < 1) return 0;
    MatmulProblem pr{m, n, p, Law{}, Law{}, levels->problem, nullptr, nullptr};
    MatmulPlan plan;
    if (!matmul_plan(&pr, 1, levels->prec, levels->num_levels, levels->c, nullptr, func_of(levels),
                     levels->index_weights, plan))
        return 0;
    if (levels->flags & MLMC_FLAG_SET_FORM) matmul_plan_set_form(plan);
    return plan.total;
}

mlmc_status mlmc_inner_product_estimate(int64_t n, const mlmc_dist* x, const mlmc_dist* y,
                                        const mlmc_levels* lv, double* out, double* level_means,
                                        void* workspace, size_t workspace_bytes, mlmc_report* report,
                                        void* stream_ptr)
{
    g_last_error.clear();
    mlmc_status st = check_inner(n, x, y, lv, out, workspace, workspace_bytes);
    if (st != MLMC_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    char* ws = static_cast<char*>(workspace);
    const int L1 = lv->num_levels;
    std::vector<int64_t> counts(L1, 0);
    std::vector<double> var(L1, 0.0);
    KernelTimer timer_obj(stream);
    KernelTimer* timer = (lv->flags & MLMC_FLAG_TIMING) ? &timer_obj : nullptr;
    hipError_t e = hipSuccess;
    if (!(lv->flags & MLMC_FLAG_ADAPTIVE_LEVELS)) {
        // fixed N_l, or target mode with eq. (28) on the device: one
        // synchronisation at the end (target mode reads V_l, N_l and the
        // schedule's status; fixed N_l only when a report is asked for)
        if ((e = inner_enqueue(n, x, y, lv, out, level_means, ws, stream, timer)) != hipSuccess)
            return device_fail(e, lv->rmse_target > 0.0 ? "target-mode launch" : "level launch");
        if (lv->rmse_target <= 0.0 && !report) return MLMC_OK;
        if ((st = inner_collect(n, lv, ws, stream, var.data(), counts.data())) != MLMC_OK) return st;
        if (report) fill_report(lv, counts.data(), var.data(), timer, report, L1, true);
        return MLMC_OK;
    }
    const InnerLayout L = inner_layout(L1, n, lv->index_weights != nullptr);
    Moments* state = reinterpret_cast<Moments*>(ws + L.off_state);
    Moments* partials = reinterpret_cast<Moments*>(ws + L.off_partials);
    double* var_dev = reinterpret_cast<double*>(ws + L.off_var);
    InnerSlot* slot = reinterpret_cast<InnerSlot*>(ws + L.off_slot);
    const IndexWeights iw{lv->index_weights,
                          lv->index_weights ? reinterpret_cast<const uint64_t*>(ws + L.off_cum) : nullptr};
    const Law lx = to_law(*x), ly = to_law(*y);
    const StreamKeys keys = keys_of(lv);
    if (iw.w) {
        ScopedTiming t(timer, MLMC_KERNEL_FINAL);
        e = build_cumulative(iw.w, n, reinterpret_cast<uint64_t*>(ws + L.off_cum), stream);
    }
    if (e != hipSuccess) return device_fail(e, "cumulative weights");
    const bool word32 = (lv->flags & MLMC_FLAG_INDEX_WORD32) != 0;

    // every level of a phase goes into one launch; the first phase of an
    // estimate clears the level states
    auto run_all = [&](const int64_t* k0, const int64_t* cnt, bool first) -> hipError_t {
        LevelRange ranges[MLMC_MAX_LEVELS];
        for (int l = 0; l < L1; ++l) ranges[l] = range_of(lv, l, k0[l], cnt[l]);
        return inner_levels_run(ranges, L1, n, lx, ly, func_of(lv), iw, lv->prec, word32, keys, partials, state,
                                slot, first, nullptr, stream, timer);
    };
    // Alg. 2's loop over L: pilot of the new level, eq. (28) over the levels
    // so far, extension of every level, then the bias test
    std::vector<int64_t> amount(L1, 0), target(L1);
    int used = 0;
    bool passed = false;
    for (int L = 0; L < L1 && !passed; ++L) {
        std::fill(amount.begin(), amount.end(), 0);
        amount[L] = lv->pilot_samples;
        if ((e = run_all(counts.data(), amount.data(), L == 0)) != hipSuccess) return device_fail(e, "pilot launch");
        counts[L] = lv->pilot_samples;
        used = L + 1;
        {
            ScopedTiming t(timer, MLMC_KERNEL_FINAL);
            e = inner_telescope(state, L1, out, nullptr, var_dev, stream);
        }
        if (e != hipSuccess) return device_fail(e, "level statistics");
        if ((e = hipMemcpyAsync(var.data(), var_dev, sizeof(double) * L1, hipMemcpyDeviceToHost, stream)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return device_fail(e, "level statistics readback");
        if ((st = schedule(lv, var.data(), used, target.data())) != MLMC_OK) return st;
        for (int l = 0; l < L1; ++l) amount[l] = l < used && target[l] > counts[l] ? target[l] - counts[l] : 0;
        if ((e = run_all(counts.data(), amount.data(), false)) != hipSuccess)
            return device_fail(e, "extension launch");
        for (int l = 0; l < L1; ++l) counts[l] += amount[l];
        if (used >= 3) {
            Moments fin;
            if ((e = hipMemcpyAsync(&fin, state + L, sizeof(Moments), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
                (e = hipStreamSynchronize(stream)) != hipSuccess)
                return device_fail(e, "level mean readback");
            passed = bias_test(lv, L, fabs(fin.mean), true);
        }
    }
    {
        ScopedTiming t(timer, MLMC_KERNEL_FINAL);
        e = inner_telescope(state, L1, out, level_means, var_dev, stream);
        if (e != hipSuccess) return device_fail(e, "telescope");
    }
    if (report) {
        if ((e = hipMemcpyAsync(var.data(), var_dev, sizeof(double) * L1, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return device_fail(e, "report readback");
        fill_report(lv, counts.data(), var.data(), timer, report, used, passed);
    }
    return MLMC_OK;
}

mlmc_status mlmc_matmul_estimate(int64_t m, int64_t n, int64_t p, const mlmc_dist* A, const mlmc_dist* B,
                                 const mlmc_levels* lv, double* out, double* level_means, void* workspace,
                                 size_t workspace_bytes, mlmc_report* report, void* stream_ptr)
{
    g_last_error.clear();
    if (m < 1 || p < 1 || n < 1) return fail(MLMC_EINVAL, "m, n, p must be >= 1");
    if (n >= kU32) return fail(MLMC_EINVAL, "n must be < 2^32");
    mlmc_status st = check_levels(lv, false);
    if (st != MLMC_OK) return st;
    if ((st = check_dist(A, "A", m, false)) != MLMC_OK) return st;
    if ((st = check_dist(B, "B", p, false)) != MLMC_OK) return st;
    if ((st = check_pair(A, B, lv->prec, lv->flags)) != MLMC_OK) return st;
    if (!out) return fail(MLMC_EINVAL, "out is NULL");
    MatmulProblem pr{m, n, p, to_law(*A), to_law(*B), lv->problem, out, level_means};
    MatmulPlan plan;
    if (!matmul_plan(&pr, 1, lv->prec, lv->num_levels, lv->c, nullptr, func_of(lv), lv->index_weights, plan))
        return fail(MLMC_EINVAL, "no launch plan for this shape and precision");
    plan.value16 = (lv->flags & MLMC_FLAG_VALUE16) != 0;
    if (lv->flags & MLMC_FLAG_SET_FORM) matmul_plan_set_form(plan);
    if (!workspace || workspace_bytes < plan.total)
        return fail(MLMC_EWORKSPACE, "workspace needs %zu bytes", plan.total);
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    char* ws = static_cast<char*>(workspace);
    const StreamKeys keys = keys_of(lv);
    const int L1 = lv->num_levels;
    std::vector<int64_t> counts(L1, 0);
    std::vector<double> var(L1, 0.0);
    double* var_dev = matmul_level_var_ptr(plan, ws);
    KernelTimer timer_obj(stream);
    KernelTimer* timer = (lv->flags & MLMC_FLAG_TIMING) ? &timer_obj : nullptr;
    hipError_t e = matmul_upload(plan, ws, stream);
    if (e != hipSuccess) return device_fail(e, "problem table upload");
    {
        ScopedTiming t(timer, MLMC_KERNEL_FINAL);
        e = matmul_reset(plan, ws, stream);
        if (e == hipSuccess && lv->index_weights)
            e = build_cumulative(lv->index_weights, n, reinterpret_cast<uint64_t*>(ws + plan.off_cum), stream);
    }
    if (e != hipSuccess) return device_fail(e, "state reset");

    auto run = [&](int l, int64_t k0, int64_t cnt, int64_t before) -> hipError_t {
        return matmul_level_run(plan, range_of(lv, l, k0, cnt), before, keys, ws, stream, timer);
    };
    int used = L1;
    bool passed = true;
    if (lv->flags & MLMC_FLAG_ADAPTIVE_LEVELS) {
        // Alg. 2's loop over L: pilot of the new level, eq. (28) over the
        // levels so far, extension of every level, then the bias test
        used = 0;
        passed = false;
        std::vector<int64_t> target(L1);
        for (int L = 0; L < L1 && !passed; ++L) {
            if ((e = run(L, 0, lv->pilot_samples, 0)) != hipSuccess) return device_fail(e, "pilot launch");
            counts[L] = lv->pilot_samples;
            used = L + 1;
            {
                ScopedTiming t(timer, MLMC_KERNEL_FINAL);
                e = matmul_finalize(plan, counts.data(), ws, false, stream);
            }
            if (e != hipSuccess) return device_fail(e, "level statistics");
            if ((e = hipMemcpyAsync(var.data(), var_dev, sizeof(double) * L1, hipMemcpyDeviceToHost, stream)) !=
                    hipSuccess ||
                (e = hipStreamSynchronize(stream)) != hipSuccess)
                return device_fail(e, "level statistics readback");
            if ((st = schedule(lv, var.data(), used, target.data())) != MLMC_OK) return st;
            for (int l = 0; l < used; ++l) {
                if (target[l] <= counts[l]) continue;
                if ((e = run(l, counts[l], target[l] - counts[l], counts[l])) != hipSuccess)
                    return device_fail(e, "extension launch");
                counts[l] = target[l];
            }
            if (used >= 3) {
                double norm2 = 0.0;
                if ((e = matmul_level_norm2(plan, ws, L, stream)) != hipSuccess ||
                    (e = hipMemcpyAsync(&norm2, matmul_norm_ptr(plan, ws), sizeof(double), hipMemcpyDeviceToHost,
                                        stream)) != hipSuccess ||
                    (e = hipStreamSynchronize(stream)) != hipSuccess)
                    return device_fail(e, "level mean norm");
                passed = bias_test(lv, L, sqrt(norm2), false);
            }
        }
    } else if (lv->rmse_target > 0.0) {
        for (int l = 0; l < L1; ++l) {
            if ((e = run(l, 0, lv->pilot_samples, 0)) != hipSuccess) return device_fail(e, "pilot launch");
            counts[l] = lv->pilot_samples;
        }
        {
            ScopedTiming t(timer, MLMC_KERNEL_FINAL);
            e = matmul_finalize(plan, counts.data(), ws, false, stream);
        }
        if (e != hipSuccess) return device_fail(e, "pilot statistics");
        if ((e = hipMemcpyAsync(var.data(), var_dev, sizeof(double) * L1, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return device_fail(e, "pilot readback");
        std::vector<int64_t> target(L1);
        if ((st = schedule(lv, var.data(), L1, target.data())) != MLMC_OK) return st;
        for (int l = 0; l < L1; ++l) {
            if ((e = run(l, counts[l], target[l] - counts[l], counts[l])) != hipSuccess)
                return device_fail(e, "extension launch");
            counts[l] = target[l];
        }
    } else {
        for (int l = 0; l < L1; ++l) {
            if ((e = run(l, 0, lv->n_samples[l], 0)) != hipSuccess) return device_fail(e, "level launch");
            counts[l] = lv->n_samples[l];
        }
    }
    {
        ScopedTiming t(timer, MLMC_KERNEL_FINAL);
        e = matmul_finalize(plan, counts.data(), ws, true, stream);
    }
    if (e != hipSuccess) return device_fail(e, "finalize");
    if (report) {
        if ((e = hipMemcpyAsync(var.data(), var_dev, sizeof(double) * L1, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return device_fail(e, "report readback");
        fill_report(lv, counts.data(), var.data(), timer, report, used, passed);
    }
    return MLMC_OK;
}

}  // extern "C"

// ---- allocation-free inner product ----------------------------------------
// The inner-product estimator's device workspace (level states, workgroup
// partials, V_l, cumulative index weights) as one fixed array per GPU, for
// callers that cannot allocate.  In host code the name `scratch` is a
// host-side stand-in, not a device address: only the address that
// hipGetSymbolAddress returns, taken once per device with that device
// current, is handed to kernels.
static __device__ __align__(256) unsigned char scratch[MLMC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on the device of `stream` (the current
// device for the null stream).
mlmc_status scratch_for_stream(hipStream_t stream, void** out)
{
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    int dev = cur;
    if (stream && (e = hipStreamGetDevice(stream, &dev)) != hipSuccess) return device_fail(e, "hipStreamGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MLMC_EDEVICE, "device %d is beyond the library's table of %d", dev,
                                                   kMaxDevices);
    std::lock_guard<std::mutex> guard(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return device_fail(e, "hipSetDevice");
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (dev != cur) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess && r != hipSuccess) return device_fail(r, "hipSetDevice (restore)");
        }
        if (e != hipSuccess) return device_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(MLMC_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MLMC_OK;
}

}  // namespace

extern "C" {

size_t mlmc_inner_product_noalloc_limit(void) { return MLMC_NOALLOC_SCRATCH_BYTES; }

mlmc_status mlmc_inner_product_estimate_noalloc(int64_t n, const mlmc_dist* x, const mlmc_dist* y,
                                                const mlmc_levels* lv, double* out, double* level_means,
                                                mlmc_report* report, void* stream_ptr)
{
    g_last_error.clear();
    if (!lv || lv->num_levels < 1 || lv->num_levels > MLMC_MAX_LEVELS)
        return fail(MLMC_EINVAL, "num_levels must be in [1, %d]", MLMC_MAX_LEVELS);
    if (n < 1 || n >= kU32) return fail(MLMC_EINVAL, "n must be in [1, 2^32)");
    const size_t need = inner_layout(lv->num_levels, n, lv->index_weights != nullptr).total;
    if (need > MLMC_NOALLOC_SCRATCH_BYTES)
        return fail(MLMC_EINVAL,
                    "the estimate needs %zu bytes of scratch, beyond the allocation-free limit of %zu "
                    "(weighted draws need 8 n bytes: n too large)",
                    need, (size_t)MLMC_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    const mlmc_status st = scratch_for_stream(static_cast<hipStream_t>(stream_ptr), &ws);
    if (st != MLMC_OK) return st;
    // the estimator clears its level states itself and writes every partial
    // before it reads it, so the previous call's contents do not matter
    return mlmc_inner_product_estimate(n, x, y, lv, out, level_means, ws, MLMC_NOALLOC_SCRATCH_BYTES, report,
                                       stream_ptr);
}

}  // extern "C"

namespace {

mlmc_status check_batch(int32_t nprob, const mlmc_problem* probs, const mlmc_levels* lv, const mlmc_tuning* tune,
                        std::vector<MatmulProblem>& out, MatmulTuning& tuning)
{
    mlmc_status st = check_levels(lv, false);
    if (st != MLMC_OK) return st;
    if (nprob < 1 || !probs) return fail(MLMC_EINVAL, "nprob must be >= 1 with a problem table");
    if (lv->rmse_target > 0.0 || !lv->n_samples) return fail(MLMC_EINVAL, "batched estimates take fixed N_l");
    if (lv->index_weights) return fail(MLMC_EINVAL, "batched estimates draw indices uniformly");
    std::vector<uint32_t> ids;
    out.clear();
    for (int32_t i = 0; i < nprob; ++i) {
        const mlmc_problem& pr = probs[i];
        if (pr.m < 1 || pr.p < 1 || pr.n < 1 || pr.n >= kU32)
            return fail(MLMC_EINVAL, "problem %d: m, p >= 1 and 1 <= n < 2^32 required", i);
        if ((st = check_dist(&pr.A, "A", pr.m, false)) != MLMC_OK) return st;
        if ((st = check_dist(&pr.B, "B", pr.p, false)) != MLMC_OK) return st;
        if ((st = check_pair(&pr.A, &pr.B, lv->prec, lv->flags)) != MLMC_OK) return st;
        if ((pr.A.law >= MLMC_LAW_RAMP_NORMAL) != (probs[0].A.law >= MLMC_LAW_RAMP_NORMAL))
            return fail(MLMC_EINVAL, "problem %d: the laws of the experiments are used by every product or none", i);
        if (!pr.out) return fail(MLMC_EINVAL, "problem %d: out is NULL", i);
        if (pr.problem >= (1u << 20)) return fail(MLMC_EINVAL, "problem %d: stream id must be < 2^20", i);
        ids.push_back(pr.problem);
        out.push_back(MatmulProblem{pr.m, pr.n, pr.p, to_law(pr.A), to_law(pr.B), pr.problem, pr.out, pr.level_means});
    }
    std::sort(ids.begin(), ids.end());
    for (size_t i = 1; i < ids.size(); ++i)
        if (ids[i] == ids[i - 1]) return fail(MLMC_EINVAL, "duplicate stream id %u", ids[i]);
    tuning = MatmulTuning{0, 0, 0, 0};
    if (tune) {
        if (tune->tile != 0 && tune->tile != 64 && tune->tile != 128)
            return fail(MLMC_EINVAL, "tuning.tile must be 0, 64 or 128");
        if (tune->target_blocks < 0 || tune->gather_budget < 0) return fail(MLMC_EINVAL, "negative tuning value");
        if (tune->single_launch != 0 && tune->single_launch != 1)
            return fail(MLMC_EINVAL, "tuning.single_launch must be 0 or 1");
        tuning = MatmulTuning{tune->tile, tune->target_blocks, tune->gather_budget, tune->single_launch};
    }
    return MLMC_OK;
}

// The launch plan of a batched estimate: the table checked, the shapes
// planned, and the single-launch form chosen where it is built.
mlmc_status plan_batch(int32_t nprob, const mlmc_problem* probs, const mlmc_levels* lv, const mlmc_tuning* tuning,
                       MatmulPlan& plan)
{
    std::vector<MatmulProblem> pr;
    MatmulTuning tune;
    mlmc_status st = check_batch(nprob, probs, lv, tuning, pr, tune);
    if (st != MLMC_OK) return st;
    if (!matmul_plan(pr.data(), nprob, lv->prec, lv->num_levels, lv->c, &tune, func_of(lv), nullptr, plan))
        return fail(MLMC_EINVAL, "no launch plan for this table");
    plan.value16 = (lv->flags & MLMC_FLAG_VALUE16) != 0;
    if (lv->flags & MLMC_FLAG_SET_FORM) matmul_plan_set_form(plan);
    if (tune.single_launch) {
        std::vector<LevelRange> ranges;
        for (int l = 0; l < lv->num_levels; ++l) ranges.push_back(range_of(lv, l, 0, lv->n_samples[l]));
        matmul_plan_persistent(plan, ranges.data(), lv->num_levels);
    }
    return MLMC_OK;
}

// Enqueues a whole fixed-N batched estimate (no host synchronisation): the
// reset, then one persistent launch for every pass of every level (or a
// gather, a sketch and a merge launch per pass), then the finalisation.
hipError_t enqueue_batched(const MatmulPlan& plan, const mlmc_levels* lv, char* ws, hipStream_t stream,
                           KernelTimer* timer)
{
    hipError_t e;
    {
        ScopedTiming t(timer, MLMC_KERNEL_FINAL);
        e = matmul_reset(plan, ws, stream);
    }
    if (e != hipSuccess) return e;
    const StreamKeys keys = keys_of(lv);
    if (plan.persistent) {
        if ((e = matmul_persistent_run(plan, keys, ws, stream, timer)) != hipSuccess) return e;
    } else {
        for (int l = 0; l < lv->num_levels; ++l)
            if ((e = matmul_level_run(plan, range_of(lv, l, 0, lv->n_samples[l]), 0, keys, ws, stream, timer)) !=
                hipSuccess)
                return e;
    }
    ScopedTiming t(timer, MLMC_KERNEL_FINAL);
    return matmul_finalize(plan, lv->n_samples, ws, true, stream);
}

}  // namespace

struct mlmc_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

size_t mlmc_matmul_batched_workspace_size(int32_t nprob, const mlmc_problem* probs, const mlmc_levels* levels,
                                          const mlmc_tuning* tuning)
{
    MatmulPlan plan;
    if (plan_batch(nprob, probs, levels, tuning, plan) != MLMC_OK) return 0;
    return plan.total;
}

mlmc_status mlmc_matmul_estimate_batched(int32_t nprob, const mlmc_problem* probs, const mlmc_levels* lv,
                                         const mlmc_tuning* tuning, void* workspace, size_t workspace_bytes,
                                         double* level_var, void* stream_ptr)
{
    g_last_error.clear();
    MatmulPlan plan;
    mlmc_status st = plan_batch(nprob, probs, lv, tuning, plan);
    if (st != MLMC_OK) return st;
    if (!workspace || workspace_bytes < plan.total)
        return fail(MLMC_EWORKSPACE, "workspace needs %zu bytes", plan.total);
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    char* ws = static_cast<char*>(workspace);
    hipError_t e = matmul_upload(plan, ws, stream);
    if (e != hipSuccess) return device_fail(e, "problem table upload");
    if ((e = enqueue_batched(plan, lv, ws, stream, nullptr)) != hipSuccess) return device_fail(e, "batched launch");
    if (level_var) {
        if ((e = hipMemcpyAsync(level_var, matmul_level_var_ptr(plan, ws), sizeof(double) * lv->num_levels * nprob,
                                hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return device_fail(e, "level variance readback");
        bool failed = false;
        if ((e = matmul_persistent_status(plan, ws, stream, &failed)) != hipSuccess)
            return device_fail(e, "status readback");
        if (failed) return fail(MLMC_EDEVICE, "the single-launch estimate gave up at a phase barrier");
    }
    return MLMC_OK;
}

mlmc_status mlmc_matmul_batched_graph_create(int32_t nprob, const mlmc_problem* probs, const mlmc_levels* lv,
                                             const mlmc_tuning* tuning, void* workspace, size_t workspace_bytes,
                                             void* stream_ptr, mlmc_graph* graph)
{
    g_last_error.clear();
    if (!graph) return fail(MLMC_EINVAL, "graph is NULL");
    *graph = nullptr;
    if (!stream_ptr) return fail(MLMC_EINVAL, "graph capture needs a non-null stream");
    MatmulPlan plan;
    mlmc_status st = plan_batch(nprob, probs, lv, tuning, plan);
    if (st != MLMC_OK) return st;
    if (!workspace || workspace_bytes < plan.total)
        return fail(MLMC_EWORKSPACE, "workspace needs %zu bytes", plan.total);
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    char* ws = static_cast<char*>(workspace);
    hipError_t e = matmul_upload(plan, ws, stream);
    if (e != hipSuccess) return device_fail(e, "problem table upload");
    mlmc_graph g = new mlmc_graph_s();
    if ((e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        delete g;
        return device_fail(e, "begin capture");
    }
    hipError_t launch = enqueue_batched(plan, lv, ws, stream, nullptr);
    e = hipStreamEndCapture(stream, &g->graph);
    if (launch != hipSuccess || e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return device_fail(launch != hipSuccess ? launch : e, "capture");
    }
    if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        return device_fail(e, "instantiate");
    }
    *graph = g;
    return MLMC_OK;
}

mlmc_status mlmc_graph_launch(mlmc_graph graph, void* stream)
{
    g_last_error.clear();
    if (!graph || !graph->exec) return fail(MLMC_EINVAL, "graph is NULL");
    hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? MLMC_OK : device_fail(e, "graph launch");
}

mlmc_status mlmc_graph_destroy(mlmc_graph graph)
{
    g_last_error.clear();
    if (!graph) return MLMC_OK;
    hipError_t e1 = graph->exec ? hipGraphExecDestroy(graph->exec) : hipSuccess;
    hipError_t e2 = graph->graph ? hipGraphDestroy(graph->graph) : hipSuccess;
    delete graph;
    if (e1 != hipSuccess) return device_fail(e1, "graph exec destroy");
    if (e2 != hipSuccess) return device_fail(e2, "graph destroy");
    return MLMC_OK;
}

mlmc_status mlmc_inner_product_graph_create(int64_t n, const mlmc_dist* x, const mlmc_dist* y,
                                            const mlmc_levels* lv, double* out, double* level_means,
                                            void* workspace, size_t workspace_bytes, void* stream_ptr,
                                            mlmc_graph* graph)
{
    g_last_error.clear();
    if (!graph) return fail(MLMC_EINVAL, "graph is NULL");
    *graph = nullptr;
    if (!stream_ptr) return fail(MLMC_EINVAL, "graph capture needs a non-null stream");
    mlmc_status st = check_inner(n, x, y, lv, out, workspace, workspace_bytes);
    if (st != MLMC_OK) return st;
    if (lv->flags & MLMC_FLAG_ADAPTIVE_LEVELS)
        return fail(MLMC_EINVAL, "the adaptive loop over L reads its bias test on the host: no graph form");
    if (lv->flags & MLMC_FLAG_TIMING) return fail(MLMC_EINVAL, "kernel timing is not available in a graph");
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    mlmc_graph g = new mlmc_graph_s();
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete g;
        return device_fail(e, "begin capture");
    }
    const hipError_t launch = inner_enqueue(n, x, y, lv, out, level_means, static_cast<char*>(workspace), stream,
                                            nullptr);
    e = hipStreamEndCapture(stream, &g->graph);
    if (launch != hipSuccess || e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return device_fail(launch != hipSuccess ? launch : e, "capture");
    }
    if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        return device_fail(e, "instantiate");
    }
    *graph = g;
    return MLMC_OK;
}

mlmc_status mlmc_inner_product_graph_report(int64_t n, const mlmc_levels* lv, const void* workspace,
                                            size_t workspace_bytes, mlmc_report* report, void* stream_ptr)
{
    g_last_error.clear();
    if (n < 1 || n >= kU32) return fail(MLMC_EINVAL, "n must be in [1, 2^32)");
    mlmc_status st = check_levels(lv, true);
    if (st != MLMC_OK) return st;
    if (lv->flags & MLMC_FLAG_ADAPTIVE_LEVELS) return fail(MLMC_EINVAL, "adaptive estimates have no graph form");
    const size_t need = inner_layout(lv->num_levels, n, lv->index_weights != nullptr).total;
    if (!workspace || workspace_bytes < need) return fail(MLMC_EWORKSPACE, "workspace needs %zu bytes", need);
    std::vector<int64_t> counts(lv->num_levels, 0);
    std::vector<double> var(lv->num_levels, 0.0);
    if ((st = inner_collect(n, lv, static_cast<const char*>(workspace), static_cast<hipStream_t>(stream_ptr),
                            var.data(), counts.data())) != MLMC_OK)
        return st;
    if (report) fill_report(lv, counts.data(), var.data(), nullptr, report, lv->num_levels, true);
    return MLMC_OK;
}

size_t mlmc_matmul_adjoint_workspace_size(int64_t m, int64_t n, int64_t p, const mlmc_levels* levels)
{
    if (check_levels(levels, false) != MLMC_OK || m < 1 || p < 1 || n < 1) return 0;
    return adjoint_workspace_size(m, n, p, levels->num_levels, levels->c, levels->n_samples,
                                  levels->index_weights != nullptr);
}

mlmc_status mlmc_matmul_adjoint_reparam(int64_t m, int64_t n, int64_t p, const mlmc_dist* A, const mlmc_dist* B,
                                        const mlmc_levels* lv, const double* grad_out, float* dMA, float* dSA,
                                        float* dMB, float* dSB, void* workspace, size_t workspace_bytes,
                                        void* stream_ptr)
{
    g_last_error.clear();
    if (m < 1 || p < 1 || n < 1) return fail(MLMC_EINVAL, "m, n, p must be >= 1");
    if (n >= kU32) return fail(MLMC_EINVAL, "n must be < 2^32");
    mlmc_status st = check_levels(lv, false);
    if (st != MLMC_OK) return st;
    if (lv->rmse_target > 0.0 || !lv->n_samples)
        return fail(MLMC_EINVAL, "the adjoint needs the forward's N_l (fixed mode)");
    if (lv->func != MLMC_FUNC_IDENTITY) return fail(MLMC_EINVAL, "the adjoint is defined for f = identity");
    if (lv->prec != MLMC_PREC_FP32 && lv->prec != MLMC_PREC_BF16)
        return fail(MLMC_EINVAL, "the adjoint runs in FP32 or with BF16 operands");
    if ((st = check_dist(A, "A", m, false)) != MLMC_OK) return st;
    if ((st = check_dist(B, "B", p, false)) != MLMC_OK) return st;
    if (A->law != MLMC_LAW_REPARAM || B->law != MLMC_LAW_REPARAM)
        return fail(MLMC_EINVAL, "the adjoint is defined for reparameterised laws");
    if (!grad_out || !dMA || !dSA || !dMB || !dSB) return fail(MLMC_EINVAL, "null gradient pointer");
    // any workspace from the least one up works (a smaller one takes more passes)
    const size_t need = adjoint_workspace_min(m, n, p, lv->index_weights != nullptr);
    if (!workspace || workspace_bytes < need)
        return fail(MLMC_EWORKSPACE, "workspace needs at least %zu bytes (%zu for the fewest passes)", need,
                    adjoint_workspace_size(m, n, p, lv->num_levels, lv->c, lv->n_samples,
                                           lv->index_weights != nullptr));
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    KernelTimer timer_obj(stream);
    KernelTimer* timer = (lv->flags & MLMC_FLAG_TIMING) ? &timer_obj : nullptr;
    hipError_t e = adjoint_run(m, n, p, to_law(*A), to_law(*B), lv->num_levels, lv->c, lv->n_samples, keys_of(lv),
                               (lv->flags & MLMC_FLAG_SHARED_SAMPLES) != 0, grad_out, dMA, dSA, dMB, dSB,
                               lv->index_weights, static_cast<char*>(workspace), workspace_bytes,
                               lv->prec == MLMC_PREC_BF16, (lv->flags & MLMC_FLAG_STRIDE_COUPLING) != 0,
                               (lv->flags & MLMC_FLAG_VALUE16) != 0, stream, timer);
    return e == hipSuccess ? MLMC_OK : device_fail(e, "adjoint launch");
}

mlmc_status mlmc_philox4x32_10(int64_t count, const uint32_t* ctr, uint64_t seed, uint32_t* out, void* stream)
{
    g_last_error.clear();
    if (count < 0 || (count > 0 && (!ctr || !out))) return fail(MLMC_EINVAL, "bad philox arguments");
    hipError_t e = philox_batch(count, ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out,
                                static_cast<hipStream_t>(stream));
    return e == hipSuccess ? MLMC_OK : device_fail(e, "philox launch");
}

mlmc_status mlmc_sample_indices(uint64_t seed, uint32_t problem, uint32_t level_field, uint32_t k0,
                                int64_t num_samples, int64_t c, int64_t n, int32_t* out, void* stream)
{
    g_last_error.clear();
    if (num_samples < 0 || c < 1 || c >= kU32 || n < 1 || n >= kU32 || (num_samples > 0 && !out) ||
        problem >= (1u << 20) || level_field > 0xFFu || (int64_t)k0 + num_samples > kU32)
        return fail(MLMC_EINVAL, "bad sample_indices arguments");
    StreamKeys keys{(uint32_t)seed, (uint32_t)(seed >> 32), problem};
    hipError_t e = sample_indices(keys, level_field, k0, num_samples, c, n, out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? MLMC_OK : device_fail(e, "sample_indices launch");
}

mlmc_status mlmc_sample_indices_weighted(uint64_t seed, uint32_t problem, uint32_t level_field, uint32_t k0,
                                         int64_t num_samples, int64_t c, int64_t n, const uint32_t* weights,
                                         uint64_t* cum, int32_t* out, void* stream)
{
    g_last_error.clear();
    if (num_samples < 0 || c < 1 || c >= kU32 || n < 1 || n >= kU32 || (num_samples > 0 && !out) || !weights ||
        !cum || problem >= (1u << 20) || level_field > 0xFFu || (int64_t)k0 + num_samples > kU32)
        return fail(MLMC_EINVAL, "bad sample_indices_weighted arguments");
    StreamKeys keys{(uint32_t)seed, (uint32_t)(seed >> 32), problem};
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = build_cumulative(weights, n, cum, st);
    if (e == hipSuccess) e = sample_indices_weighted(keys, level_field, k0, num_samples, c, n, cum, out, st);
    return e == hipSuccess ? MLMC_OK : device_fail(e, "sample_indices_weighted launch");
}

mlmc_status mlmc_optimal_index_weights(int64_t m, int64_t n, int64_t p, const mlmc_dist* A, const mlmc_dist* B,
                                       uint32_t* weights, double* scratch, void* stream)
{
    g_last_error.clear();
    if (m < 1 || p < 1 || n < 1 || n >= kU32) return fail(MLMC_EINVAL, "m, p >= 1 and 1 <= n < 2^32 required");
    if (!weights) return fail(MLMC_EINVAL, "weights is NULL");
    mlmc_status st;
    if ((st = check_dist(A, "A", m, false)) != MLMC_OK) return st;
    if ((st = check_dist(B, "B", p, false)) != MLMC_OK) return st;
    if (A->law >= MLMC_LAW_RAMP_NORMAL || B->law >= MLMC_LAW_RAMP_NORMAL)
        return fail(MLMC_EINVAL, "xi** is computed for reparameterised or i.i.d. laws");
    const bool reparam = A->law == MLMC_LAW_REPARAM;
    if (reparam != (B->law == MLMC_LAW_REPARAM))
        return fail(MLMC_EINVAL, "A and B must both be reparameterised, or both i.i.d.");
    if (reparam && !scratch) return fail(MLMC_EINVAL, "scratch is NULL");
    hipError_t e = optimal_weights(m, n, p, to_law(*A), to_law(*B), weights, scratch, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? MLMC_OK : device_fail(e, "optimal weights launch");
}

mlmc_status mlmc_gather_columns(int64_t m, int64_t n, int64_t p, const mlmc_dist* A, const mlmc_dist* B,
                                uint64_t seed, uint32_t problem, uint32_t level_field, uint32_t k0,
                                int64_t num_samples, int64_t c, int32_t prec, double* AS, double* BS,
                                void* stream)
{
    g_last_error.clear();
    if (m < 1 || p < 1 || n < 1 || n >= kU32 || c < 1 || c >= kU32 || num_samples < 0 || !AS || !BS ||
        prec < MLMC_PREC_FP64 || prec > MLMC_PREC_BF16 || problem >= (1u << 20) || level_field > 0xFFu)
        return fail(MLMC_EINVAL, "bad gather_columns arguments");
    mlmc_status st;
    if ((st = check_dist(A, "A", m, false)) != MLMC_OK) return st;
    if ((st = check_dist(B, "B", p, false)) != MLMC_OK) return st;
    if ((st = check_pair(A, B, prec)) != MLMC_OK) return st;
    StreamKeys keys{(uint32_t)seed, (uint32_t)(seed >> 32), problem};
    hipError_t e = gather_columns_f64(m, n, p, to_law(*A), to_law(*B), keys, level_field, k0, num_samples, c, prec,
                                      AS, BS, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? MLMC_OK : device_fail(e, "gather_columns launch");
}

}  // extern "C"
