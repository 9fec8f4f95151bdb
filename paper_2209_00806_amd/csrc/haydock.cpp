// Host driver of the Haydock recursion (paper, Sec. "Local density of
// states", the recursion method): the Lanczos chains of all states advance
// together, two iterations per replay of a captured HIP graph (the two
// Lanczos buffers swap roles every iteration).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tbpm_engine.h"

namespace tbpm {

#define TRY_HIP(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

tbpm_status Engine::haydock(const double *psi0, int32_t s_user, int32_t n_iter, double thr, double *a_out,
                            double *b_out, uint32_t flags, hipStream_t st) {
    int32_t s_pad = 1, log2s = 0;
    while (s_pad < s_user) {
        s_pad <<= 1;
        ++log2s;
    }
    const int64_t n = mat.n_rows;
    // tiles and tile order of the FP64 launch configuration (the kernels take
    // one state per thread whatever its states per thread)
    const tbpm_launch_config &lc = cfgs[0];
    tbpm_status s0 = build_tiles(s_pad, lc.wg_chunks, 1);
    if (s0 != TBPM_OK) return s0;
    const int32_t n_tiles = (int32_t)h_tiles.size();
    const size_t vec = sizeof(double) * 2 * (size_t)n * s_pad;
    TRY_HIP(hay_u.ensure(2 * vec), "alloc Lanczos vectors");
    TRY_HIP(hay_y.ensure(vec), "alloc Lanczos product");
    TRY_HIP(hay_s.ensure(sizeof(double) * 4 * (size_t)s_pad), "alloc Lanczos scalars");
    const size_t n_part = 3 * (size_t)n_tiles * s_pad;
    TRY_HIP(partials.ensure(sizeof(double) * (n_part + (size_t)hay_fold_count(n_tiles) * s_pad)), "alloc partials");
    TRY_HIP(counter.ensure(sizeof(int32_t)), "alloc counter");
    double *u[2] = {(double *)hay_u.ptr, (double *)((char *)hay_u.ptr + vec)};
    double *y = (double *)hay_y.ptr;
    double *hs = (double *)hay_s.ptr;
    double *part = (double *)partials.ptr;
    double *fold = part + n_part;
    int32_t *cnt = (int32_t *)counter.ptr;
    const TileDesc *td = (const TileDesc *)tiles.ptr;
    const void *val = mat.val64;  // double or complex128 per stored element

    // u_0 = psi0 (internal order, padded states zero), u_{-1} = 0, 1/b_0 = 1/||psi0||
    TRY_HIP(launch_expand_states(psi0, mat.perm, s_user, u[0], log2s, n, st), "load start vectors");
    TRY_HIP(launch_fill_zero(u[1], 2 * n * s_pad, st), "clear Lanczos vector");
    TRY_HIP(launch_hay_axpy(td, n_tiles, lc.xcd_remap, 0, log2s, u[0], nullptr, nullptr, hs, part, st), "start norm");
    TRY_HIP(launch_hay_reduce(part, n_tiles, s_pad, s_user, 2, thr, hs, cnt, n_iter, a_out, b_out, fold, st),
            "start norm reduce");

    auto iteration = [&](int par, hipStream_t s) -> hipError_t {
        double *cur = u[par], *prev = u[1 - par];
        hipError_t e = launch_hay_spmv(mat.is_complex, td, n_tiles, lc.xcd_remap, log2s, mat.col, val,
                                       mat.slice_off, mat.uniform_w, mat.onsite64, cur, prev, y, hs, cnt, part, s);
        if (e == hipSuccess)
            e = launch_hay_reduce(part, n_tiles, s_pad, s_user, 0, thr, hs, cnt, n_iter, a_out, b_out, fold, s);
        if (e == hipSuccess) e = launch_hay_axpy(td, n_tiles, lc.xcd_remap, 1, log2s, y, cur, prev, hs, part, s);
        if (e == hipSuccess)
            e = launch_hay_reduce(part, n_tiles, s_pad, s_user, 1, thr, hs, cnt, n_iter, a_out, b_out, fold, s);
        return e;
    };

    const int32_t pairs = n_iter / 2;
    if ((flags & TBPM_FLAG_NO_GRAPH) || pairs < 2) {
        for (int32_t i = 0; i < n_iter; ++i) TRY_HIP(iteration(i & 1, st), "launch Lanczos iteration");
    } else {
        TRY_HIP(hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        hipError_t ce = iteration(0, capture_stream);
        if (ce == hipSuccess) ce = iteration(1, capture_stream);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(capture_stream, &g);
        if (ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(ce, "capture Lanczos iterations");
        }
        if (ee != hipSuccess) return hip_fail(ee, "end capture");
        hipGraphExec_t ge = nullptr;
        hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
        hipError_t le = hipSuccess;
        for (int32_t p = 0; p < pairs && le == hipSuccess; ++p) le = hipGraphLaunch(ge, st);
        if (le == hipSuccess && (n_iter & 1)) le = iteration(0, st);
        // the executable graph is destroyed once its replays have finished
        hipError_t se = hipStreamSynchronize(st);
        (void)hipGraphExecDestroy(ge);
        if (le != hipSuccess) return hip_fail(le, "launch Lanczos iterations");
        if (se != hipSuccess) return hip_fail(se, "stream synchronize");
    }
    TRY_HIP(hipStreamSynchronize(st), "stream synchronize");
    TRY_HIP(hipGetLastError(), "kernel execution");
    return TBPM_OK;
}

}  // namespace tbpm
