// H.v launch plans and the autotuner: time every valid plan on the device and
// keep the fastest.  All plans sum each output in the same order, so the
// choice changes speed only, never results.
#include <cfloat>
#include <vector>

#include "pdz_internal.h"

using namespace pdz;

namespace {

pdz_status check_dt(pdz_problem p, pdz_dtype dt) {
    if (!p) return fail(PDZ_EINVAL, "problem is NULL");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be PDZ_F64 or PDZ_F32");
    if (p->ks || p->par) return fail(PDZ_EINVAL, "a symmetry-sector problem has one H.v kernel and no launch plans");
    return ok();
}

}  // namespace

extern "C" {

pdz_status pdz_hv_get_plan(pdz_problem p, pdz_dtype dt, pdz_hv_plan* out) {
    pdz_status st = check_dt(p, dt);
    if (st != PDZ_OK) return st;
    if (!out) return fail(PDZ_EINVAL, "out is NULL");
    const std::vector<HvPlan> c = hv_candidates(p, dt);
    HvPlan pl = p->plan[dt];
    if (pl.down == 0) pl.down = c[0].down;
    if (pl.up_cw == 0) pl.up_cw = c[0].up_cw;
    if (pl.up == 0) pl.up = c[0].up;
    if (pl.map == 0) pl.map = c[0].map;
    out->down = pl.down;
    out->up_cw = pl.up_cw;
    out->up = pl.up;
    out->map = pl.map;
    return ok();
}

pdz_status pdz_hv_set_plan(pdz_problem p, pdz_dtype dt, const pdz_hv_plan* plan) {
    pdz_status st = check_dt(p, dt);
    if (st != PDZ_OK) return st;
    if (!plan) return fail(PDZ_EINVAL, "plan is NULL");
    HvPlan pl;
    pl.down = plan->down;
    pl.up_cw = plan->up_cw;
    pl.up = plan->up;
    pl.map = plan->map;
    if (!hv_plan_valid(p, dt, pl)) return fail(PDZ_EINVAL, "plan not available for this problem and precision");
    p->plan[dt] = pl;
    return ok();
}

pdz_status pdz_hv_tune(pdz_problem p, pdz_dtype dt, const void* x, void* y, int32_t reps, pdz_hv_trial* trials,
                       int32_t max_trials, int32_t* n_trials, pdz_hv_plan* best, void* stream) {
    pdz_status st = check_dt(p, dt);
    if (st != PDZ_OK) return st;
    if (!x || !y) return fail(PDZ_EINVAL, "NULL vector");
    if (reps < 1) return fail(PDZ_EINVAL, "reps must be >= 1");
    if (max_trials > 0 && !trials) return fail(PDZ_EINVAL, "trials is NULL");
    hipStream_t s = (hipStream_t)stream;
    const HvPlan saved = p->plan[dt];
    const std::vector<HvPlan> cands = hv_candidates(p, dt);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PDZ_HIP(hipEventCreate(&e0));
    PDZ_HIP(hipEventCreate(&e1));
    double best_ms = DBL_MAX;
    HvPlan best_plan = cands[0];
    int n = 0;
    st = ok();
    for (const HvPlan& c : cands) {
        p->plan[dt] = c;
        st = pdz_hv(p, dt, x, y, stream);   // warm-up
        if (st != PDZ_OK) break;
        hipError_t e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == PDZ_OK && e == hipSuccess; ++r) st = pdz_hv(p, dt, x, y, stream);
        if (st != PDZ_OK) break;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = hip_fail(e, "autotune timing");
            break;
        }
        const double avg = (double)ms / reps;
        if (n < max_trials) {
            trials[n].plan.down = c.down;
            trials[n].plan.up_cw = c.up_cw;
            trials[n].plan.up = c.up;
            trials[n].plan.map = c.map;
            trials[n].ms = avg;
        }
        ++n;
        if (avg < best_ms) {
            best_ms = avg;
            best_plan = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PDZ_OK) {
        p->plan[dt] = saved;
        return st;
    }
    p->plan[dt] = best_plan;
    if (n_trials) *n_trials = n < max_trials ? n : max_trials;
    if (best) {
        best->down = best_plan.down;
        best->up_cw = best_plan.up_cw;
        best->up = best_plan.up;
        best->map = best_plan.map;
    }
    return ok();
}

pdz_status pdz_hv_kernel_times(pdz_problem p, pdz_dtype dt, const void* x, void* y, int32_t reps, double* ms,
                               void* stream) {
    pdz_status st = check_dt(p, dt);
    if (st != PDZ_OK) return st;
    if (!x || !y || !ms) return fail(PDZ_EINVAL, "NULL argument");
    if (reps < 1 || reps > 1000) return fail(PDZ_EINVAL, "reps must be in [1, 1000]");
    hipStream_t s = (hipStream_t)stream;
    ms[0] = ms[1] = ms[2] = 0.0;
    // ev[3r], ev[3r+1], ev[3r+2] bracket the down and the up launch of H.v number r
    std::vector<hipEvent_t> ev(3 * (size_t)reps + 2, nullptr);
    for (auto& e : ev) {
        hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) {
            st = hip_fail(he, "hipEventCreate");
            break;
        }
    }
    const bool two = p->hv_path == 0;
    if (st == PDZ_OK) st = launch_hv(p, dt, x, y, s);   // warm-up
    for (int r = 0; r < reps && st == PDZ_OK; ++r) {
        hipError_t he = hipEventRecord(ev[3 * r], s);
        if (two) {
            if (he == hipSuccess) st = launch_hv(p, dt, x, y, s, nullptr, kPassDown);
            if (st == PDZ_OK && he == hipSuccess) he = hipEventRecord(ev[3 * r + 1], s);
            if (st == PDZ_OK && he == hipSuccess) st = launch_hv(p, dt, x, y, s, nullptr, kPassUp);
        } else {
            if (he == hipSuccess) st = launch_hv(p, dt, x, y, s);
            if (st == PDZ_OK && he == hipSuccess) he = hipEventRecord(ev[3 * r + 1], s);
        }
        if (st == PDZ_OK && he == hipSuccess) he = hipEventRecord(ev[3 * r + 2], s);
        if (he != hipSuccess && st == PDZ_OK) st = hip_fail(he, "hipEventRecord");
    }
    // whole H.v, back to back
    const size_t w0 = 3 * (size_t)reps, w1 = w0 + 1;
    if (st == PDZ_OK) {
        hipError_t he = hipEventRecord(ev[w0], s);
        for (int r = 0; r < reps && st == PDZ_OK && he == hipSuccess; ++r) st = launch_hv(p, dt, x, y, s);
        if (st == PDZ_OK && he == hipSuccess) he = hipEventRecord(ev[w1], s);
        if (he == hipSuccess) he = hipEventSynchronize(ev[w1]);
        if (he != hipSuccess && st == PDZ_OK) st = hip_fail(he, "kernel timing");
    }
    if (st == PDZ_OK) {
        double sd = 0.0, su = 0.0;
        float t = 0.f;
        for (int r = 0; r < reps && st == PDZ_OK; ++r) {
            hipError_t he = hipEventElapsedTime(&t, ev[3 * r], ev[3 * r + 1]);
            sd += t;
            if (he == hipSuccess) he = hipEventElapsedTime(&t, ev[3 * r + 1], ev[3 * r + 2]);
            su += t;
            if (he != hipSuccess) st = hip_fail(he, "hipEventElapsedTime");
        }
        if (st == PDZ_OK) {
            hipError_t he = hipEventElapsedTime(&t, ev[w0], ev[w1]);
            if (he != hipSuccess) st = hip_fail(he, "hipEventElapsedTime");
        }
        if (st == PDZ_OK) {
            ms[0] = sd / reps;
            ms[1] = two ? su / reps : 0.0;
            ms[2] = (double)t / reps;
        }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

}  // extern "C"
