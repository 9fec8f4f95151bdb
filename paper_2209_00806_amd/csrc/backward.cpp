// Driver of tbpm_backward: exact discrete adjoint of the Clenshaw propagation.
//
// Segments of K steps are replayed forward from their checkpoints (psi_0 =
// phi0, psi_{mK} from tbpm_propagate), keeping every step's Clenshaw vectors
// b_1 .. b_{M-2} (b_{M-1} = c_{M-1} psi_l is recomputed on the fly); the
// adjoint then runs backwards through the segment, one fused kernel per
// Chebyshev order j (see backward.hip).  Device memory: (K+1) + K (M-2)
// state vectors for the segment plus four adjoint vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <cstring>
#include <vector>

#include "tbpm_engine.h"

namespace tbpm {

using cd = std::complex<double>;

#define TRY_HIP(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

tbpm_status backward_impl(tbpm_hamiltonian *H, const double *psi0, int32_t s_user, int32_t N, double dt, double f,
                          double tol, const double *gcorr, int32_t K, const double *ckpt, double *grad_val,
                          double *grad_onsite, hipStream_t st) {
    Engine &eng = H->eng;
    int dev = 0;
    TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != eng.device) return fail(TBPM_E_ARG, "handle was created on another device");
    const bool cplx = eng.mat.is_complex;
    const int64_t n_rows = eng.mat.n_rows;
    const int64_t nnz = H->csr.nnz();
    int32_t s_pad = 1, log2s = 0;
    while (s_pad < s_user) {
        s_pad <<= 1;
        ++log2s;
    }
    std::vector<cd> c;
    const int32_t M = cheb_coeffs(f * dt, tol, c);
    if (M < 3) return fail(TBPM_E_ARG, "Bessel series does not converge");
    const std::vector<PassPlan> plan = plan_step({c}, {f}, M);
    const int n_passes = (int)plan.size();

    eng.cfg = eng.cfgs[0];
    eng.cfg.staged = 0;  // the replay and the adjoint use single-state units
    eng.cfg.vec = 1;
    eng.cfg.fused = 0;
    // With the fused shape in the FP64 launch configuration the replay takes
    // two Clenshaw orders per launch (when the two-hop tile tables fit): every
    // order's output has a slot of its own in the segment store, so a pair's
    // outputs never alias what its tiles read.  The adjoint passes run on the
    // same tiles (any tiling of the rows serves them).
    // Those launches take the configuration's states per thread (vs) and
    // non-temporal streaming; the single-order adjoint keeps one state per
    // thread.  The two-hop tables depend on the bytes of a row only, so one
    // set serves every unit width (the LDS size in units follows the width).
    bool pairs = eng.cfgs[0].fused > 0 && M - 2 >= 2;
    int32_t pvs = 1, log2pvs = 0;
    while (pvs < eng.cfgs[0].vec && pvs < s_pad && pvs < 4) {
        pvs <<= 1;
        ++log2pvs;
    }
    const bool pnt = eng.cfgs[0].nontemporal != 0;
    if (pairs && eng.build_fused_tiles(s_pad, log2s - log2pvs, 16 * pvs, eng.cfgs[0].fused) != TBPM_OK)
        pairs = false;
    tbpm_status s = pairs ? TBPM_OK : eng.build_tiles(s_pad, eng.cfg.wg_chunks, 1);
    if (s != TBPM_OK) return s;
    const int32_t n_tiles = (int32_t)eng.h_tiles.size();
    const int64_t n_el = n_rows * s_pad;
    if (n_el >= (int64_t)INT32_MAX) return fail(TBPM_E_ARG, "n_orb * n_states (padded to a power of two) must be < 2^31");
    const size_t vb = sizeof(double) * 2 * (size_t)n_el;

    if (N < 2) {
        TRY_HIP(launch_fill_zero(grad_val, 2 * nnz, st), "zero grad");
        TRY_HIP(launch_fill_zero(grad_onsite, n_rows, st), "zero grad");
        TRY_HIP(hipStreamSynchronize(st), "stream synchronize");
        return TBPM_OK;
    }
    const int32_t seg_len = std::min<int32_t>(K, N - 1);
    const int32_t n_b = M - 2;  // stored b_1 .. b_{M-2} per step
    const size_t n_store = (size_t)(seg_len + 1) + (size_t)seg_len * n_b;
    TRY_HIP(eng.bwd_store.ensure(vb * n_store), "alloc segment store (reduce ckpt_every)");
    TRY_HIP(eng.bwd_adj.ensure(vb * (pairs ? 5 : 4)), "alloc adjoint vectors");
    TRY_HIP(eng.phi0.ensure(vb), "alloc phi0");
    TRY_HIP(eng.bwd_gacc.ensure((cplx ? 16 : 8) * (size_t)std::max<int64_t>(eng.mat.ell_size, 1)), "alloc gradient");
    TRY_HIP(eng.bwd_gdiag.ensure(8 * (size_t)n_rows), "alloc gradient");
    TRY_HIP(eng.bwd_coef.ensure(sizeof(PassCoef) * n_passes), "alloc coefficients");
    if (!eng.partner_ready) {
        const std::vector<int32_t> part = ell_partner_slots(n_rows, eng.h_slice_off, eng.h_col);
        if (part.empty()) return fail(TBPM_E_NOT_HERMITIAN, "a stored element has no transposed partner");
        TRY_HIP(hipStreamSynchronize(st), "stream synchronize");
        TRY_HIP(eng.bwd_partner.ensure(sizeof(int32_t) * std::max<size_t>(part.size(), 1)), "alloc partner slots");
        TRY_HIP(hipMemcpy(eng.bwd_partner.ptr, part.data(), sizeof(int32_t) * part.size(), hipMemcpyHostToDevice),
                "upload partner slots");
        eng.partner_ready = true;
    }
    TRY_HIP(eng.partials.ensure(sizeof(double) * 3 * (size_t)n_tiles * s_pad), "alloc partials");
    TRY_HIP(eng.counter.ensure(sizeof(int32_t) * 64), "alloc counter");
    std::vector<PassCoef> hc(n_passes);
    for (int p = 0; p < n_passes; ++p) hc[p] = plan[p].coef[0];
    TRY_HIP(hipStreamSynchronize(st), "stream synchronize");
    TRY_HIP(hipMemcpy(eng.bwd_coef.ptr, hc.data(), sizeof(PassCoef) * n_passes, hipMemcpyHostToDevice),
            "upload coefficients");

    // the replay needs psi_{l+1} but not its correlation: the last pass runs
    // as the same combination without the correlation stream
    auto replay_kind = [](int kind) {
        return kind == kPassLast ? (int)kPassMid : (kind == kPassLastNoB2 ? (int)kPassNoB2 : kind);
    };
    double *store = (double *)eng.bwd_store.ptr;
    auto psi_slot = [&](int t) { return store + (size_t)t * 2 * n_el; };
    auto b_slot = [&](int t, int j) {  // b_j, j = 1 .. M-2, of local step t
        return store + ((size_t)(seg_len + 1) + (size_t)t * n_b + (size_t)(j - 1)) * 2 * n_el;
    };
    double *adj = (double *)eng.bwd_adj.ptr;
    double *lam = adj, *acc = adj + 2 * n_el;
    double *rot[3] = {lam, adj + 4 * n_el, adj + 6 * n_el};
    double *rot4 = pairs ? adj + 8 * n_el : nullptr;  // the fourth alpha buffer of the paired sweep
    double *phi0p = (double *)eng.phi0.ptr;

    TRY_HIP(launch_expand_states(psi0, eng.mat.perm, s_user, phi0p, log2s, n_rows, st), "expand psi0");
    TRY_HIP(launch_lam_init(lam, phi0p, gcorr + 2 * (size_t)(N - 1) * s_user, s_user, log2s, n_rows, st),
            "adjoint init");
    TRY_HIP(launch_fill_zero((double *)eng.bwd_gacc.ptr, (cplx ? 2 : 1) * eng.mat.ell_size, st), "zero gradient");
    TRY_HIP(launch_fill_zero((double *)eng.bwd_gdiag.ptr, n_rows, st), "zero gradient");

    // Clenshaw pass j of each plan entry (FIRST, NOB2, MID..., LAST)
    std::vector<int> pass_j(n_passes);
    if (M == 3) {
        pass_j = {1, 0};
    } else {
        pass_j[0] = M - 2;
        pass_j[1] = M - 3;
        for (int p = 2; p < n_passes - 1; ++p) pass_j[p] = M - 2 - p;
        pass_j[n_passes - 1] = 0;
    }

    PassParams pp{};
    pp.tiles = (const TileDesc *)eng.tiles.ptr;
    pp.n_tiles = n_tiles;
    pp.xcd_remap = eng.cfg.xcd_remap;
    pp.log2s = log2s;
    pp.bump_counter = 0;
    pp.col = eng.mat.col;
    pp.val = eng.mat.val64;
    pp.slice_off = eng.mat.slice_off;
    pp.onsite = eng.mat.onsite64;
    pp.counter = (int32_t *)eng.counter.ptr;
    pp.phi0 = phi0p;
    pp.phi0_ld = s_pad;
    pp.partials = (double *)eng.partials.ptr;
    pp.ckpt = nullptr;
    pp.ckpt_slot = nullptr;
    pp.s_user = s_user;
    pp.uniform_w = eng.mat.uniform_w;

    AdjParams ap{};
    ap.tiles = (const TileDesc *)eng.tiles.ptr;
    ap.n_tiles = n_tiles;
    ap.xcd_remap = eng.cfg.xcd_remap;
    ap.log2s = log2s;
    ap.s_user = s_user;
    ap.col = eng.mat.col;
    ap.val = eng.mat.val64;
    ap.slice_off = eng.mat.slice_off;
    ap.onsite = eng.mat.onsite64;
    ap.inv_f = 1.0 / f;
    ap.gacc = eng.bwd_gacc.ptr;
    ap.gdiag = (double *)eng.bwd_gdiag.ptr;
    ap.phi0 = phi0p;
    ap.partner = (const int32_t *)eng.bwd_partner.ptr;
    ap.uniform_w = eng.mat.uniform_w;

    // one step of the replay in the fused shape: orders (M-2, M-3) from psi,
    // then (j, j-1) pairs, a leftover order alone, and the last pass alone
    FusedParams fp{};
    fp.tiles = (const TileDesc *)eng.tiles.ptr;
    fp.n_tiles = n_tiles;
    fp.xcd_remap = eng.cfg.xcd_remap;
    fp.log2s = log2s;
    fp.bump_counter = 0;
    fp.col = eng.mat.col;
    fp.val = eng.mat.val64;
    fp.slice_off = eng.mat.slice_off;
    fp.onsite = eng.mat.onsite64;
    fp.counter = (int32_t *)eng.counter.ptr;
    fp.uoff = (const int32_t *)eng.st_uoff.ptr;
    fp.n1 = (const int32_t *)eng.fu_n1.ptr;
    fp.ucol = (const int32_t *)eng.st_ucol.ptr;
    fp.lidx = (const uint16_t *)eng.st_lidx.ptr;
    fp.hoff = (const int32_t *)eng.fu_hoff.ptr;
    fp.hw = (const int32_t *)eng.fu_hw.ptr;
    fp.hidx = (const uint16_t *)eng.fu_hidx.ptr;
    fp.lds_units = (int32_t)(eng.fu_max_rows << (log2s - log2pvs));
    fp.uniform_w = eng.mat.uniform_w;
    const PassCoef *coefs = (const PassCoef *)eng.bwd_coef.ptr;
    // consecutive launches walk the tiles in opposite directions, so that a
    // launch starts on the tiles whose rows the one before left in the caches
    int32_t walk = 0;
    auto replay_step_pairs = [&](int32_t t) -> hipError_t {
        // plan entry p evaluates order pass_j[p]: 0 FIRST (M-2), 1 NOB2 (M-3),
        // 2 .. n_passes-2 MID (M-4 .. 1), n_passes-1 LAST (0)
        fp.v = psi_slot(t);
        fp.x = psi_slot(t);
        fp.b2 = nullptr;
        fp.out1 = b_slot(t, M - 2);
        fp.out2 = b_slot(t, M - 3);
        fp.coef1 = coefs;
        fp.coef2 = coefs + 1;
        fp.reverse = walk;
        walk ^= 1;
        hipError_t e = launch_pair(kPairFirst, false, cplx, pnt, pvs, fp, st);
        int p = 2;
        for (; e == hipSuccess && p + 1 < n_passes - 1; p += 2) {
            const int j = pass_j[p];
            fp.x = b_slot(t, j + 1);
            fp.b2 = b_slot(t, j + 2);
            fp.out1 = b_slot(t, j);
            fp.out2 = b_slot(t, j - 1);
            fp.coef1 = coefs + p;
            fp.coef2 = coefs + p + 1;
            fp.reverse = walk;
            walk ^= 1;
            e = launch_pair(kPairMid, false, cplx, pnt, pvs, fp, st);
        }
        for (; e == hipSuccess && p < n_passes; ++p) {  // a leftover MID, then LAST
            const int j = pass_j[p];
            pp.v = psi_slot(t);
            pp.x = b_slot(t, j + 1);
            pp.b2 = b_slot(t, j + 2);
            pp.out = (j == 0) ? psi_slot(t + 1) : b_slot(t, j);
            pp.coef = coefs + p;
            pp.reverse = walk;
            walk ^= 1;
            e = launch_pass(replay_kind(plan[p].kind), false, cplx, pnt, eng.cfg.unroll, pvs, pp, st);
        }
        return e;
    };

    // one step of the adjoint with two orders per launch: (0, 1), then
    // (j, j+1) while j + 2 <= M - 2, the remaining orders with the single-order
    // kernel (the last one, j = M - 2, with b_{M-1} = c_{M-1} psi_l).  The
    // alpha vectors rotate over four buffers: a pair reads alpha_j on other
    // tiles' rows and alpha_{j-1} on its 1-hop rows, so its outputs go to the
    // two buffers it does not read.  lambda_l ends in 'acc'.
    AdjPairParams qp{};
    qp.tiles = (const TileDesc *)eng.tiles.ptr;
    qp.n_tiles = n_tiles;
    qp.xcd_remap = eng.cfg.xcd_remap;
    qp.log2s = log2s;
    qp.col = eng.mat.col;
    qp.val = eng.mat.val64;
    qp.slice_off = eng.mat.slice_off;
    qp.onsite = eng.mat.onsite64;
    qp.inv_f = 1.0 / f;
    qp.gacc = eng.bwd_gacc.ptr;
    qp.gdiag = (double *)eng.bwd_gdiag.ptr;
    qp.partner = (const int32_t *)eng.bwd_partner.ptr;
    qp.uoff = (const int32_t *)eng.st_uoff.ptr;
    qp.n1 = (const int32_t *)eng.fu_n1.ptr;
    qp.ucol = (const int32_t *)eng.st_ucol.ptr;
    qp.lidx = (const uint16_t *)eng.st_lidx.ptr;
    qp.hoff = (const int32_t *)eng.fu_hoff.ptr;
    qp.hw = (const int32_t *)eng.fu_hw.ptr;
    qp.hidx = (const uint16_t *)eng.fu_hidx.ptr;
    qp.lds_units = (int32_t)(eng.fu_max_rows << (log2s - log2pvs));
    qp.uniform_w = eng.mat.uniform_w;
    qp.cc0_re = c[0].real();
    qp.cc0_im = -c[0].imag();
    auto adjoint_step_pairs = [&](int32_t t, int32_t l) -> hipError_t {
        double *X = rot[0];  // alpha_0 = lambda_{l+1}
        double *P = nullptr;
        double *fr[2] = {rot[1], rot[2]};  // buffers no launch of this order reads
        double *spare = rot4;
        int j = 0;
        hipError_t e = hipSuccess;
        for (; e == hipSuccess && j + 2 <= M - 2; j += 2) {
            qp.x = X;
            qp.a_prev = P;
            qp.out1 = fr[0];
            qp.out2 = fr[1];
            qp.lam_acc = acc;
            qp.bq1 = b_slot(t, j + 1);
            qp.bq2 = b_slot(t, j + 2);
            qp.w1 = j == 0 ? 1.0 : 2.0;
            qp.w2 = 2.0;
            qp.cc1_re = c[j + 1].real();
            qp.cc1_im = -c[j + 1].imag();
            qp.cc2_re = c[j + 2].real();
            qp.cc2_im = -c[j + 2].imag();
            qp.reverse = walk;
            walk ^= 1;
            e = launch_adjoint_pair(j == 0 ? kAdjPairFirst : kAdjPairMid, cplx, pvs, qp, st);
            // alpha_{j+2} is the next x, alpha_{j+1} the next prev; the old x and
            // prev (or the spare buffer after the first pair) take the outputs
            double *nx = fr[1], *np = fr[0];
            fr[0] = X;
            fr[1] = P ? P : spare;
            X = nx;
            P = np;
        }
        for (; e == hipSuccess && j <= M - 2; ++j) {
            const int kind = (j == M - 2) ? kAdjFinal : kAdjMid;
            ap.a_cur = X;
            ap.a_prev = P;
            ap.a_next = fr[0];
            ap.lam_acc = acc;
            if (j + 1 <= M - 2) {
                ap.bq = b_slot(t, j + 1);
                ap.bs_re = 1.0;
                ap.bs_im = 0.0;
            } else {  // b_{M-1} = c_{M-1} psi_l
                ap.bq = psi_slot(t);
                ap.bs_re = c[M - 1].real();
                ap.bs_im = c[M - 1].imag();
            }
            ap.gw = 2.0;
            ap.cc0_re = c[0].real();
            ap.cc0_im = -c[0].imag();
            ap.ccn_re = c[j + 1].real();
            ap.ccn_im = -c[j + 1].imag();
            ap.gcorr_l = gcorr + 2 * (size_t)l * s_user;
            ap.reverse = walk;
            walk ^= 1;
            e = launch_adjoint_pass(kind, cplx, ap, st);
            double *nx = fr[0];
            fr[0] = P;
            P = X;
            X = nx;
        }
        // lambda_l is in acc: it becomes alpha_0 of the next step
        std::swap(rot[0], acc);
        return e;
    };

    const int32_t n_seg = (N - 1 + K - 1) / K;
    for (int32_t seg = n_seg - 1; seg >= 0; --seg) {
        const int32_t l0 = seg * K;
        const int32_t len = std::min(l0 + K, N - 1) - l0;
        if (seg == 0)
            TRY_HIP(hipMemcpyAsync(psi_slot(0), phi0p, vb, hipMemcpyDeviceToDevice, st), "segment start");
        else
            TRY_HIP(launch_expand_states(ckpt + 2 * (size_t)(seg - 1) * n_rows * s_user, eng.mat.perm, s_user,
                                         psi_slot(0), log2s, n_rows, st),
                    "segment start");
        // forward replay, keeping b_1 .. b_{M-2} of every step
        for (int32_t t = 0; t < len; ++t) {
            if (pairs) {
                TRY_HIP(replay_step_pairs(t), "replay pair");
                continue;
            }
            for (int p = 0; p < n_passes; ++p) {
                const int j = pass_j[p];
                const PassPlan &pl = plan[p];
                pp.v = psi_slot(t);
                if (pl.kind == kPassFirst)
                    pp.x = psi_slot(t);
                else
                    pp.x = b_slot(t, j + 1);
                pp.b2 = (pl.kind == kPassMid || pl.kind == kPassLast) ? b_slot(t, j + 2) : nullptr;
                pp.out = (j == 0) ? psi_slot(t + 1) : b_slot(t, j);
                pp.coef = (const PassCoef *)eng.bwd_coef.ptr + p;
                pp.reverse = walk;
                walk ^= 1;
                TRY_HIP(launch_pass(replay_kind(pl.kind), false, cplx, false, eng.cfg.unroll, 1, pp, st), "replay pass");
            }
        }
        // adjoint sweep through the segment
        for (int32_t t = len - 1; t >= 0; --t) {
            const int32_t l = l0 + t;
            if (pairs) {
                TRY_HIP(adjoint_step_pairs(t, l), "adjoint pair");
                continue;
            }
            for (int j = 0; j <= M - 2; ++j) {
                const int kind = (j == 0) ? kAdjFirst : (j == M - 2 ? kAdjFinal : kAdjMid);
                ap.a_cur = rot[j % 3];
                ap.a_prev = j > 0 ? rot[(j + 2) % 3] : nullptr;
                ap.a_next = rot[(j + 1) % 3];
                ap.lam_acc = acc;
                if (j + 1 <= M - 2) {
                    ap.bq = b_slot(t, j + 1);
                    ap.bs_re = 1.0;
                    ap.bs_im = 0.0;
                } else {  // b_{M-1} = c_{M-1} psi_l
                    ap.bq = psi_slot(t);
                    ap.bs_re = c[M - 1].real();
                    ap.bs_im = c[M - 1].imag();
                }
                ap.gw = (j == 0) ? 1.0 : 2.0;
                ap.cc0_re = c[0].real();
                ap.cc0_im = -c[0].imag();
                ap.ccn_re = c[j + 1].real();
                ap.ccn_im = -c[j + 1].imag();
                ap.gcorr_l = gcorr + 2 * (size_t)l * s_user;
                // the first pass (j = 0) writes alpha_1 = H~ lambda; the final pass
                // (j = M-2) leaves the new lambda in 'acc'
                ap.reverse = walk;
                walk ^= 1;
                TRY_HIP(launch_adjoint_pass(kind, cplx, ap, st), "adjoint pass");
            }
            // lambda_l is in acc; the old lambda buffer becomes the accumulator
            std::swap(rot[0], acc);
        }
    }
    TRY_HIP(launch_grad_scatter(eng.bwd_gacc.ptr, (const double *)eng.bwd_gdiag.ptr, eng.mat.ell_csr,
                                eng.mat.ell_size, cplx, 1.0 / f, grad_val, grad_onsite, eng.mat.perm, n_rows, st),
            "gradient scatter");
    TRY_HIP(hipStreamSynchronize(st), "stream synchronize");
    TRY_HIP(hipGetLastError(), "kernel execution");
    return TBPM_OK;
}

}  // namespace tbpm
