// Host driver of the kernel-polynomial moments of the Kubo-Bastin formula
// (paper, Sec. "Tight-binding propagation method", the DC conductivity
// tensor):
//     mu_mn = (1/S) sum_s <r_s| v_a T_m(H~) v_b T_n(H~) |r_s>,   m, n < M.
// With L_m = T_m(H~) v_a r and R_n = v_b T_n(H~) r (H~ and v Hermitian),
// mu_mn = <L_m|R_n>: the moments are one complex matrix product L^H R with
// an inner dimension of rows x states.  All M vectors L_m are kept in HBM
// (the Chebyshev recursion writes them in place); R is produced in blocks of
// moments, and each block's product runs on the FP64 matrix cores
// (k_kpm_product), split into chunks of the long inner dimension whose
// results are summed in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "tbpm_engine.h"

namespace tbpm {

#define TRY_HIP(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

tbpm_status Engine::kpm_moments(const double *ja, const double *jb, const double *psi0, int32_t s_user, int32_t n_mom,
                                double f, double *mu, hipStream_t st, KpmTiming *timing) {
    int32_t s_pad = 1, log2s = 0;
    while (s_pad < s_user) {
        s_pad <<= 1;
        ++log2s;
    }
    const int64_t n = mat.n_rows;
    const int64_t K = n * s_pad;  // inner dimension of the moment product
    const int32_t nb = std::min<int32_t>(n_mom, 128);
    const size_t vec = sizeof(double) * 2 * (size_t)K;
    // vectors of the L store and the R block lie vstride bytes apart: a pad
    // of 768 bytes keeps the rows the product reads at once off the same
    // offset of a large power-of-two stride (measured: their loads run 12%
    // faster than at the bare stride)
    const size_t vstride = vec + 768;
    // product split: the inner dimension (ld = 2K doubles) in chunks of a
    // multiple of 32 doubles, enough of them that the product's workgroups
    // (tiles of one chunk) fill the chip about 16 times over (two per CU)
    const int64_t ld = 2 * K;
    const KpmProductShape sh = kpm_product_shape(kpm_shape);
    const int64_t tiles_m = (n_mom + sh.wm * sh.tm * 16 - 1) / (sh.wm * sh.tm * 16);
    const int64_t tiles_n = (nb + (4 / sh.wm) * sh.tn * 16 - 1) / ((4 / sh.wm) * sh.tn * 16);
    const int64_t want = std::max<int64_t>(1, 4096 / (tiles_m * tiles_n));
    const int64_t kchunk = std::max<int64_t>(512, ((ld + want - 1) / want + 31) & ~(int64_t)31);
    const int64_t n_parts = (ld + kchunk - 1) / kchunk;
    const size_t part_bytes = sizeof(double) * 2 * (size_t)n_mom * nb;
    const size_t need = vstride * ((size_t)n_mom + nb) + vec * 5 + part_bytes * (size_t)n_parts;
    size_t free_b = 0, total_b = 0;
    TRY_HIP(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    const size_t have = kp_store.bytes + kp_rblk.bytes + kp_vec.bytes + kp_parts.bytes;
    if (need > free_b + have)
        return fail(TBPM_E_OOM, "the moment vectors need " + std::to_string(need >> 20) + " MiB of device memory");

    // With the fused shape configured, the Chebyshev orders run two per launch
    // (the Clenshaw pair with alpha = 0 is the three-term recursion: the second
    // order subtracts the first's input): L_m straight into the store, T_n
    // over four rotating blocks.
    bool pairs = cfgs[0].fused > 0 && n_mom >= 4;
    int32_t pvs = 1, log2pvs = 0;
    while (pvs < cfgs[0].vec && pvs < s_pad && pvs < 4) {
        pvs <<= 1;
        ++log2pvs;
    }
    const bool pnt = cfgs[0].nontemporal != 0;
    if (pairs && build_fused_tiles(s_pad, log2s - log2pvs, 16 * pvs, cfgs[0].fused) != TBPM_OK) pairs = false;
    if (!pairs) {
        tbpm_status s0 = build_tiles(s_pad, cfg.wg_chunks, 1);
        if (s0 != TBPM_OK) return s0;
    }
    TRY_HIP(kp_store.ensure(vstride * (size_t)n_mom), "alloc moment vectors L");
    TRY_HIP(kp_rblk.ensure(vstride * (size_t)nb), "alloc moment vectors R");
    TRY_HIP(kp_vec.ensure(5 * vec), "alloc Chebyshev vectors");
    TRY_HIP(kp_parts.ensure(part_bytes * (size_t)n_parts), "alloc product parts");
    TRY_HIP(counter.ensure(sizeof(int32_t)), "alloc counter");
    TRY_HIP(ac_zero.ensure(sizeof(double) * (size_t)std::max<int64_t>(n, 1)), "alloc zero on-site");
    TRY_HIP(launch_fill_zero((double *)ac_zero.ptr, n, st), "clear zero on-site");

    // pass coefficients: out = 0 v + beta (op x) - b2 with op = J (beta 1), H~ (1/f) or 2 H~ (2/f)
    TRY_HIP(coef.ensure(3 * sizeof(PassCoef)), "alloc coefficients");
    TRY_HIP(hipEventSynchronize(staging_done), "wait for staging");
    TRY_HIP(staging.ensure(3 * sizeof(PassCoef)), "alloc staging");
    PassCoef *hc = (PassCoef *)staging.ptr;
    hc[0] = PassCoef{0.0, 0.0, 1.0, 0.0};
    hc[1] = PassCoef{0.0, 0.0, 1.0 / f, 0.0};
    hc[2] = PassCoef{0.0, 0.0, 2.0 / f, 0.0};
    TRY_HIP(hipMemcpyAsync(coef.ptr, hc, 3 * sizeof(PassCoef), hipMemcpyHostToDevice, st), "upload coefficients");
    TRY_HIP(hipEventRecord(staging_done, st), "record staging");
    const PassCoef *c_j = (const PassCoef *)coef.ptr, *c_1 = c_j + 1, *c_2 = c_j + 2;

    // consecutive launches walk the tiles in opposite directions
    int32_t walk = 0;
    auto pass = [&](int kind, bool jop, const double *jval, const void *x, const void *b2, void *out,
                    const PassCoef *c) -> hipError_t {
        PassParams pp{};
        pp.reverse = walk;
        walk ^= 1;
        pp.tiles = (const TileDesc *)tiles.ptr;
        pp.n_tiles = (int32_t)h_tiles.size();
        pp.xcd_remap = cfg.xcd_remap;
        pp.log2s = log2s;
        pp.col = mat.col;
        pp.val = jop ? (const void *)jval : mat.val64;
        pp.slice_off = mat.slice_off;
        pp.onsite = jop ? ac_zero.ptr : (const void *)mat.onsite64;
        pp.x = x;
        pp.v = x;
        pp.b2 = b2;
        pp.out = out;
        pp.coef = c;
        pp.counter = (int32_t *)counter.ptr;
        pp.s_user = s_pad;
        return launch_pass(kind, false, jop ? true : mat.is_complex, pairs && pnt, 1, pairs ? pvs : 1, pp, st);
    };

    FusedParams fp{};
    fp.tiles = (const TileDesc *)tiles.ptr;
    fp.n_tiles = (int32_t)h_tiles.size();
    fp.xcd_remap = cfg.xcd_remap;
    fp.log2s = log2s;
    fp.col = mat.col;
    fp.val = mat.val64;
    fp.slice_off = mat.slice_off;
    fp.onsite = mat.onsite64;
    fp.counter = (int32_t *)counter.ptr;
    fp.uoff = (const int32_t *)st_uoff.ptr;
    fp.n1 = (const int32_t *)fu_n1.ptr;
    fp.ucol = (const int32_t *)st_ucol.ptr;
    fp.lidx = (const uint16_t *)st_lidx.ptr;
    fp.hoff = (const int32_t *)fu_hoff.ptr;
    fp.hw = (const int32_t *)fu_hw.ptr;
    fp.hidx = (const uint16_t *)fu_hidx.ptr;
    fp.lds_units = (int32_t)(fu_max_rows << (log2s - log2pvs));
    fp.uniform_w = mat.uniform_w;
    fp.coef1 = fp.coef2 = c_2;
    // T_{k+1}, T_{k+2} = 2 H~ T_k - T_{k-1}, 2 H~ T_{k+1} - T_k
    auto pair = [&](const void *tk, const void *tkm1, void *o1, void *o2) -> hipError_t {
        fp.x = tk;
        fp.v = tk;
        fp.b2 = tkm1;
        fp.out1 = o1;
        fp.out2 = o2;
        fp.reverse = walk;
        walk ^= 1;
        return launch_pair(kPairMid, false, mat.is_complex, pnt, pvs, fp, st);
    };

    char *Ls = (char *)kp_store.ptr;
    char *Rb = (char *)kp_rblk.ptr;
    char *vb = (char *)kp_vec.ptr;
    void *r = vb, *t0 = vb + vec, *t1 = vb + 2 * vec;
    TRY_HIP(launch_expand_states(psi0, mat.perm, s_user, (double *)r, log2s, n, st), "load random vectors");
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (timing)
        for (auto &e : ev) TRY_HIP(hipEventCreate(&e), "hipEventCreate");
    if (timing) TRY_HIP(hipEventRecord(ev[0], st), "record");

    // L_0 = v_a r, L_1 = H~ L_0, L_{m+1} = 2 H~ L_m - L_{m-1}, in place in the store
    TRY_HIP(pass(kPassFirst, true, ja, r, nullptr, Ls, c_j), "launch current operator");
    int32_t m_done = 1;  // orders written so far
    if (pairs) {
        TRY_HIP(pass(kPassFirst, false, nullptr, Ls, nullptr, Ls + vstride, c_1), "launch Chebyshev pass");
        m_done = 2;
        for (; m_done + 1 < n_mom; m_done += 2)
            TRY_HIP(pair(Ls + vstride * (size_t)(m_done - 1), Ls + vstride * (size_t)(m_done - 2), Ls + vstride * (size_t)m_done,
                         Ls + vstride * (size_t)(m_done + 1)),
                    "launch Chebyshev pair");
    }
    for (int32_t m = m_done; m < n_mom; ++m) {
        void *out = Ls + vstride * (size_t)m;
        const void *x = Ls + vstride * (size_t)(m - 1);
        if (m == 1)
            TRY_HIP(pass(kPassFirst, false, nullptr, x, nullptr, out, c_1), "launch Chebyshev pass");
        else
            TRY_HIP(pass(kPassMid, false, nullptr, x, Ls + vstride * (size_t)(m - 2), out, c_2), "launch Chebyshev pass");
    }
    if (timing) TRY_HIP(hipEventRecord(ev[1], st), "record");

    // R_n = v_b T_n(H~) r in blocks of nb moments; T_n in (t0, t1), the
    // interior order written over T_{n-1}
    const void *tc = r;  // T_n
    void *tn[2] = {t0, t1};
    // paired T recursion: T_n (n >= 1) lives in tq[n & 3]; orders are produced
    // when first needed, two per launch while the series allows (a pair writes
    // over T_{n-4} and T_{n-3}, whose current-operator passes are done)
    void *tq[4] = {vb + 3 * vec, t0, t1, vb + 4 * vec};
    int32_t produced = 0;  // T_0 = r
    float gemm_ms = 0.0f;
    for (int32_t n0 = 0; n0 < n_mom; n0 += nb) {
        const int32_t cnt = std::min(nb, n_mom - n0);
        for (int32_t j = 0; pairs && j < cnt; ++j) {
            const int32_t nn = n0 + j;
            while (produced < nn) {
                const int32_t k = produced + 1;
                if (k == 1) {
                    TRY_HIP(pass(kPassFirst, false, nullptr, r, nullptr, tq[1], c_1), "launch Chebyshev pass");
                    produced = 1;
                } else if (k == 2) {
                    TRY_HIP(pass(kPassMid, false, nullptr, tq[1], r, tq[2], c_2), "launch Chebyshev pass");
                    produced = 2;
                } else if (k + 1 < n_mom) {
                    TRY_HIP(pair(tq[(k - 1) & 3], tq[(k - 2) & 3], tq[k & 3], tq[(k + 1) & 3]), "launch Chebyshev pair");
                    produced = k + 1;
                } else {
                    TRY_HIP(pass(kPassMid, false, nullptr, tq[(k - 1) & 3], tq[(k - 2) & 3], tq[k & 3], c_2),
                            "launch Chebyshev pass");
                    produced = k;
                }
            }
            const void *tcur = nn == 0 ? r : tq[nn & 3];
            TRY_HIP(pass(kPassFirst, true, jb, tcur, nullptr, Rb + vstride * (size_t)j, c_j), "launch current operator");
        }
        for (int32_t j = 0; !pairs && j < cnt; ++j) {
            const int32_t nn = n0 + j;
            if (nn == 1) {
                TRY_HIP(pass(kPassFirst, false, nullptr, r, nullptr, t0, c_1), "launch Chebyshev pass");
                tc = t0;
            } else if (nn == 2) {
                TRY_HIP(pass(kPassMid, false, nullptr, t0, r, t1, c_2), "launch Chebyshev pass");
                tc = t1;
            } else if (nn > 2) {
                // T_k lives in tn[(k - 1) & 1]: T_nn = 2 H~ T_{nn-1} - T_{nn-2} is
                // written over T_{nn-2}
                void *prev = tn[(nn - 1) & 1];
                TRY_HIP(pass(kPassMid, false, nullptr, tn[nn & 1], prev, prev, c_2), "launch Chebyshev pass");
                tc = prev;
            }
            TRY_HIP(pass(kPassFirst, true, jb, tc, nullptr, Rb + vstride * (size_t)j, c_j), "launch current operator");
        }
        hipEvent_t g0 = nullptr, g1 = nullptr;
        if (timing) {
            TRY_HIP(hipEventCreate(&g0), "hipEventCreate");
            TRY_HIP(hipEventCreate(&g1), "hipEventCreate");
            TRY_HIP(hipEventRecord(g0, st), "record");
        }
        // parts[p][n][m] = sum over chunk p of conj(L_m) R_{n0+n}, then
        // mu[:, n0 : n0 + cnt] = (1/S) sum_p parts[p] in order
        double *P = (double *)kp_parts.ptr;
        const int64_t pstride = (int64_t)n_mom * cnt;
        TRY_HIP(launch_kpm_product(kpm_shape, (const double *)Ls, (const double *)Rb, (int64_t)(vstride / 8), ld,
                                   n_mom, cnt, kchunk, (int32_t)n_parts, P, st),
                "launch moment product");
        TRY_HIP(launch_kpm_sum_parts(P, pstride, (int32_t)n_parts, pstride, 1.0 / s_user,
                                     mu + 2 * (size_t)n0 * n_mom, st),
                "sum moment parts");
        if (timing) {
            TRY_HIP(hipEventRecord(g1, st), "record");
            TRY_HIP(hipEventSynchronize(g1), "sync");
            float ms = 0.0f;
            TRY_HIP(hipEventElapsedTime(&ms, g0, g1), "elapsed");
            gemm_ms += ms;
            (void)hipEventDestroy(g0);
            (void)hipEventDestroy(g1);
        }
    }
    if (timing) {
        TRY_HIP(hipEventRecord(ev[2], st), "record");
        TRY_HIP(hipEventSynchronize(ev[2]), "sync");
        float a = 0.0f, b = 0.0f;
        TRY_HIP(hipEventElapsedTime(&a, ev[0], ev[1]), "elapsed");
        TRY_HIP(hipEventElapsedTime(&b, ev[1], ev[2]), "elapsed");
        timing->l_ms = a;
        timing->r_ms = b - gemm_ms;
        timing->gemm_ms = gemm_ms;
        timing->n_parts = (int32_t)n_parts;
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
    TRY_HIP(hipStreamSynchronize(st), "stream synchronize");
    TRY_HIP(hipGetLastError(), "kernel execution");
    return TBPM_OK;
}

}  // namespace tbpm
