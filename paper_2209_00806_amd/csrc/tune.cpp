// Autotuner of the Chebyshev pass launch shape: times every candidate
// (workgroup chunks x XCD remap x non-temporal streaming x elements per
// thread x states per thread; LDS-staged and two-order fused shapes) on three
// time steps of scratch states, times the three fastest again on eight steps
// (shapes within a few percent of each other swap places between short runs)
// and keeps the fastest of those in the handle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tbpm_engine.h"

namespace tbpm {

tbpm_status autotune_impl(Engine &eng, const std::vector<double> &rescale, int32_t n_states, bool fp32,
                          tbpm_launch_config *best, double *best_ms, hipStream_t stream) {
    const int32_t ni = eng.n_inst();
    const int32_t n_steps = 4;   // three timed Chebyshev steps per candidate
    const int32_t n_steps2 = 9;  // eight for the finalists
    int64_t max_rows = 0;
    for (int32_t i = 0; i < ni; ++i) max_rows = std::max(max_rows, eng.inst_row0[i + 1] - eng.inst_row0[i]);
    std::vector<double> h_psi(2 * (size_t)max_rows * n_states);
    for (int64_t r = 0; r < max_rows * n_states; ++r) {
        h_psi[2 * r] = std::cos(0.37 * (double)r) / std::sqrt((double)max_rows);
        h_psi[2 * r + 1] = std::sin(0.37 * (double)r) / std::sqrt((double)max_rows);
    }
    DevBuf psi, corr;
    hipError_t e = psi.ensure(sizeof(double) * h_psi.size());
    if (e != hipSuccess) return hip_fail(e, "autotune alloc");
    e = corr.ensure(sizeof(double) * 2 * (size_t)ni * n_steps2 * n_states);
    if (e != hipSuccess) {
        psi.release();
        return hip_fail(e, "autotune alloc");
    }
    e = hipMemcpy(psi.ptr, h_psi.data(), sizeof(double) * h_psi.size(), hipMemcpyHostToDevice);
    std::vector<const double *> p0(ni, (const double *)psi.ptr);
    std::vector<double *> c0(ni);
    for (int32_t i = 0; i < ni; ++i) c0[i] = (double *)corr.ptr + 2 * (size_t)i * n_steps2 * n_states;
    std::vector<double> dt(ni);
    for (int32_t i = 0; i < ni; ++i) dt[i] = M_PI / rescale[i];
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    tbpm_status st = TBPM_OK;
    tbpm_launch_config keep = eng.cfgs[fp32 ? 1 : 0], win = keep;
    double win_ms = 1e300;
    if (e != hipSuccess) st = hip_fail(e, "autotune setup");
    // plain shapes: chunks x unroll x vec x (remap 0/1, non-temporal); staged shapes, tier outer: LDS tier 1 x vec x
    // (remap, non-temporal), and for wide rows tiers 2-4 x vec x remap (remap 0-6 for wide rows); fused shapes
    // (sparse rows): LDS tier x vec x remap 1-6, non-temporal streams.  Staged and fused tile tables depend on the row bytes and the tier only,
    // so the vec variants of a tier share them when they are tried one after the other.
    std::vector<tbpm_launch_config> cands;
    int32_t s_pad = 1;
    while (s_pad < n_states) s_pad <<= 1;
    const int chunk_list[] = {1, 2, 4, 8, 16};
    const bool wide_rows = eng.mat.n_rows > 0 && (double)eng.mat.ell_size > 8.0 * (double)eng.mat.n_rows;
    auto vec_ok = [&](int vec) { return !(fp32 && vec == 1 && s_pad > 1); };  // 8-byte units never beat 16
    for (int vec = 1; vec <= 4 && vec <= s_pad; vec *= 2) {
        if (!vec_ok(vec)) continue;
        for (int ch : chunk_list)
            for (int un = 1; un <= 2; ++un)
                for (int remap = 0; remap <= 1; ++remap)
                    for (int nt = 0; nt <= 1; ++nt)
                        if (un <= ch) cands.push_back(tbpm_launch_config{ch, remap, nt, un, 0, vec, 0});
    }
    // the staged shape; for wide rows also the smaller LDS tiers, where the
    // halo sets the trade between tile size and resident workgroups, and the
    // tile orders that give each XCD runs of consecutive tiles
    for (int tier = 1; tier <= (wide_rows ? 4 : 1); ++tier)
        for (int vec = 1; vec <= 4 && vec <= s_pad; vec *= 2) {
            if (!vec_ok(vec)) continue;
            for (int remap = 0; remap <= (wide_rows ? 6 : 1); ++remap)
                for (int nt = 0; nt <= (tier == 1 ? 1 : 0); ++nt)
                    cands.push_back(tbpm_launch_config{2, remap, nt, 1, tier, vec, 0});
        }
    // fused shapes, tier outer; the two-hop halo grows with the square of
    // the row width, so fusing pays off only for sparse rows
    if (!wide_rows)
        for (int tier = 1; tier <= kFusedTiers; ++tier)
            for (int vec = 1; vec <= 4 && vec <= s_pad; vec *= 2)
                if (!(fp32 && vec == 1 && s_pad > 1))
                    for (int remap = 1; remap <= 6; ++remap)
                        cands.push_back(tbpm_launch_config{2, remap, 1, 1, 0, vec, tier});
    // time one shape on `steps` time steps (after a warm-up run that builds
    // its tiles and graphs); ms per step, or a negative value on failure
    auto time_cfg = [&](const tbpm_launch_config &cand, int32_t steps) -> double {
        eng.cfgs[fp32 ? 1 : 0] = cand;
        Engine::RunArgs a{};
        a.psi0 = p0.data();
        a.s_user = n_states;
        a.n_steps = steps;
        a.dt = dt.data();
        a.rescale = rescale.data();
        a.tol = 1e-12;
        a.fp32 = fp32;
        a.corr = c0.data();
        a.norm2 = nullptr;
        a.flags = TBPM_FLAG_ASYNC;
        a.stream = stream;
        st = eng.run(a);
        if (st != TBPM_OK) return -1.0;
        e = hipEventRecord(t0, stream);
        if (e == hipSuccess) st = eng.run(a);
        if (e == hipSuccess && st == TBPM_OK) e = hipEventRecord(t1, stream);
        if (e == hipSuccess && st == TBPM_OK) e = hipEventSynchronize(t1);
        float ms = 0;
        if (e == hipSuccess && st == TBPM_OK) e = hipEventElapsedTime(&ms, t0, t1);
        if (e != hipSuccess && st == TBPM_OK) st = hip_fail(e, "autotune timing");
        if (st != TBPM_OK) return -1.0;
        return ms / (steps - 1);
    };
    std::vector<std::pair<double, size_t>> timed;
    for (size_t c = 0; c < cands.size() && st == TBPM_OK; ++c) {
        const double per_step = time_cfg(cands[c], n_steps);
        if (per_step >= 0.0) timed.push_back({per_step, c});
    }
    if (st == TBPM_OK) {
        std::sort(timed.begin(), timed.end());
        for (size_t k = 0; k < timed.size() && k < 3 && st == TBPM_OK; ++k) {
            const double per_step = time_cfg(cands[timed[k].second], n_steps2);
            if (per_step >= 0.0 && per_step < win_ms) {
                win_ms = per_step;
                win = cands[timed[k].second];
            }
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipStreamSynchronize(stream);
    psi.release();
    corr.release();
    if (st != TBPM_OK) {
        eng.cfgs[fp32 ? 1 : 0] = keep;
        return st;
    }
    eng.cfgs[fp32 ? 1 : 0] = win;
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return TBPM_OK;
}

}  // namespace tbpm
