// HIP kernels of the TBPM adjoint (gradient) path for gfx950.
//
// For one time step psi_{l+1} = P psi_l, P = sum_{m<M} c_m T_m(H~), evaluated
// by Clenshaw (b_j = c_j psi_l + 2 H~ b_{j+1} - b_{j+2}, psi_{l+1} = c_0 psi_l
// + H~ b_1 - b_2), reverse-mode differentiation with respect to H~ gives,
// for the incoming adjoint lambda_{l+1} =: alpha_0,
//     alpha_1 = H~ alpha_0,   alpha_{j+1} = 2 H~ alpha_j - alpha_{j-1}
//     lambda_l = sum_{j<M} conj(c_j) alpha_j + (dL/dC_l) phi0
//     dL/dH~ = alpha_0 b_1^+ + 2 sum_{j=1}^{M-2} alpha_j b_{j+1}^+
// (the alpha_j = T_j(H~) lambda_{l+1} run the Chebyshev recurrence forward,
// the transpose of Clenshaw's backward sweep).  One kernel launch per j
// gathers alpha_j and b_{j+1} at each row's columns, writes alpha_{j+1},
// accumulates lambda, and adds alpha_j[p] conj(b_{j+1}[q]) summed over the
// states to the gradient slot of every stored entry (p, q) and to the
// diagonal.  Each slot belongs to one row, so the accumulation needs no
// atomics and is deterministic.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_util.h"
#include "tbpm_internal.h"

namespace tbpm {
namespace {

// sum over the S consecutive lanes that hold the states of one row
__device__ __forceinline__ double row_sum(double x, int log2s) {
    for (int off = 1; off < (1 << log2s); off <<= 1) x += __shfl_xor(x, off);
    return x;
}

template <bool CH, int KIND>
__global__ __launch_bounds__(kWG) void k_adj_pass(const AdjParams p) {
    using HV = std::conditional_t<CH, d2, double>;
    using GV = std::conditional_t<CH, d2, double>;
    constexpr int KG = 4;
    const int tile = tile_of_block(blockIdx.x, p.n_tiles, p.xcd_remap);
    const TileDesc td = p.tiles[tile];
    const int log2s = p.log2s;
    const uint32_t smask = (1u << log2s) - 1u;
    const uint32_t n_el = (uint32_t)td.rows << log2s;
    const uint32_t row0 = (uint32_t)td.row0;
    const uint32_t e0 = row0 << log2s;
    const d2 *__restrict__ acur = (const d2 *)p.a_cur;
    const d2 *__restrict__ bq = (const d2 *)p.bq;
    const int32_t *__restrict__ col = p.col;
    const HV *__restrict__ val = (const HV *)p.val;
    const uint32_t *__restrict__ soff = p.slice_off;
    GV *gacc = (GV *)p.gacc;
    d2 bs, ccn, cc0;
    bs.x = p.bs_re;
    bs.y = p.bs_im;
    ccn.x = p.ccn_re;
    ccn.y = p.ccn_im;
    cc0.x = p.cc0_re;
    cc0.y = p.cc0_im;
    const double gw = p.gw, inv_f = p.inv_f;

    // n_el is a multiple of S and every row's S elements sit in consecutive
    // lanes of one wave, so all lanes of a row take the same trip counts.
    for (uint32_t e = threadIdx.x; e < n_el; e += kWG) {
        const uint32_t row = row0 + (e >> log2s);
        const uint32_t s = e & smask;
        const uint32_t g = e0 + e;
        const uint32_t sl = row / kSliceRows;
        const uint32_t off = soff[sl];
        const int w = (int)((soff[sl + 1] - off) / kSliceRows);
        const uint32_t base = off + row % kSliceRows;
        // every load that does not depend on a column index first
        const d2 a = acur[g];  // alpha_j at this row
        const d2 bown = bq[g];
        const double on = p.onsite[row];
        d2 aprev, lacc, ph;
        if constexpr (KIND != kAdjFirst) {
            aprev = ((const d2 *)p.a_prev)[g];
            lacc = ((const d2 *)p.lam_acc)[g];
        }
        if constexpr (KIND == kAdjFinal) ph = ((const d2 *)p.phi0)[g];
        const double gd_old = p.gdiag[row];
        const d2 ga = a * gw;
        d2 acc;
        acc.x = on * a.x;
        acc.y = on * a.y;
        {
            // diagonal gradient: Re(alpha_j[p] conj(b[p])) summed over states
            const d2 b = cmul(bs, bown);
            const double dg = row_sum(ga.x * b.x + ga.y * b.y, log2s);
            if (s == 0) p.gdiag[row] = gd_old + dg;
        }
        for (int k = 0; k < w; k += KG) {
            uint32_t slot[KG], gc[KG];
            HV h[KG];
            bool valid[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                valid[i] = k + i < w;
                slot[i] = valid[i] ? base + (uint32_t)(k + i) * kSliceRows : 0u;
                const int32_t c = col[slot[i]];
                const HV hv = val[slot[i]];
                gc[i] = ((valid[i] ? (uint32_t)c : row) << log2s) + s;
                h[i] = valid[i] ? hv : HV{};
            }
            d2 xa[KG], xb[KG];
            GV gold[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                xa[i] = acur[gc[i]];
                xb[i] = bq[gc[i]];
                gold[i] = gacc[slot[i]];
            }
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                acc = hmad(h[i], xa[i], acc);
                const d2 b = cmul(bs, xb[i]);
                // alpha_j[p] * conj(b[q]) summed over the states of the row
                const double gr = row_sum(ga.x * b.x + ga.y * b.y, log2s);
                if constexpr (CH) {
                    const double gi = row_sum(ga.y * b.x - ga.x * b.y, log2s);
                    if (s == 0 && valid[i]) {
                        d2 nv = gold[i];
                        nv.x += gr;
                        nv.y += gi;
                        gacc[slot[i]] = nv;
                    }
                } else {
                    if (s == 0 && valid[i]) gacc[slot[i]] = gold[i] + gr;
                }
            }
        }
        acc *= inv_f;  // (H~ alpha_j)[row]
        d2 an;
        if constexpr (KIND == kAdjFirst)
            an = acc;
        else
            an = 2.0 * acc - aprev;
        d2 lam;
        if constexpr (KIND == kAdjFirst)
            lam = cmul(cc0, a) + cmul(ccn, an);
        else
            lam = lacc + cmul(ccn, an);
        if constexpr (KIND == kAdjFinal) {
            if ((int)s < p.s_user) {
                const d2 gl = ((const d2 *)p.gcorr_l)[s];
                lam += cmul(gl, ph);
            }
        } else {
            ((d2 *)p.a_next)[g] = an;
        }
        ((d2 *)p.lam_acc)[g] = lam;
    }
}

__global__ __launch_bounds__(kWG) void k_expand(const d2 *__restrict__ src, const int32_t *__restrict__ perm,
                                                int s_user, d2 *__restrict__ dst, int log2s, int64_t n_el) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < n_el; e += stride) {
        const int64_t row = perm ? (int64_t)perm[e >> log2s] : (e >> log2s);
        const int s = (int)(e & ((1 << log2s) - 1));
        d2 a;
        a.x = 0.0;
        a.y = 0.0;
        if (s < s_user) a = src[row * s_user + s];
        dst[e] = a;
    }
}

__global__ __launch_bounds__(kWG) void k_lam_init(d2 *__restrict__ lam, const d2 *__restrict__ phi0,
                                                  const d2 *__restrict__ g, int s_user, int log2s, int64_t n_el) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < n_el; e += stride) {
        const int s = (int)(e & ((1 << log2s) - 1));
        d2 a;
        a.x = 0.0;
        a.y = 0.0;
        if (s < s_user) a = cmul(g[s], phi0[e]);
        lam[e] = a;
    }
}

__global__ __launch_bounds__(kWG) void k_fill_zero(double *__restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

template <bool CH>
__global__ __launch_bounds__(kWG) void k_grad_scatter(const void *__restrict__ gacc, const double *__restrict__ gdiag,
                                                      const int64_t *__restrict__ ell_csr, int64_t ell_size,
                                                      double inv_f, d2 *__restrict__ grad_val,
                                                      double *__restrict__ grad_onsite,
                                                      const int32_t *__restrict__ perm, int64_t n_rows) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t q = (int64_t)blockIdx.x * kWG + threadIdx.x; q < ell_size; q += stride) {
        const int64_t pos = ell_csr[q];
        if (pos < 0) continue;
        d2 v;
        if constexpr (CH) {
            v = ((const d2 *)gacc)[q] * inv_f;
        } else {
            v.x = ((const double *)gacc)[q] * inv_f;
            v.y = 0.0;
        }
        grad_val[pos] = v;
    }
    for (int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x; r < n_rows; r += stride)
        grad_onsite[perm ? perm[r] : r] = gdiag[r] * inv_f;
}

int64_t grid_for(int64_t n) {
    int64_t b = (n + kWG - 1) / kWG;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : b;
}

}  // namespace

hipError_t launch_adjoint_pass(int kind, bool cplx, const AdjParams &p, hipStream_t st) {
    if (p.n_tiles <= 0) return hipSuccess;
    const dim3 grid(p.n_tiles), block(kWG);
#define TBPM_ADJ(CHV, K) hipLaunchKernelGGL((k_adj_pass<CHV, K>), grid, block, 0, st, p)
    if (cplx) {
        if (kind == kAdjFirst)
            TBPM_ADJ(true, kAdjFirst);
        else if (kind == kAdjMid)
            TBPM_ADJ(true, kAdjMid);
        else
            TBPM_ADJ(true, kAdjFinal);
    } else {
        if (kind == kAdjFirst)
            TBPM_ADJ(false, kAdjFirst);
        else if (kind == kAdjMid)
            TBPM_ADJ(false, kAdjMid);
        else
            TBPM_ADJ(false, kAdjFinal);
    }
#undef TBPM_ADJ
    return hipGetLastError();
}

hipError_t launch_expand_states(const double *src, const int32_t *perm, int32_t s_user, double *dst, int32_t log2s,
                                int64_t n_rows, hipStream_t st) {
    const int64_t n_el = n_rows << log2s;
    hipLaunchKernelGGL(k_expand, dim3((unsigned)grid_for(n_el)), dim3(kWG), 0, st, (const d2 *)src, perm, s_user,
                       (d2 *)dst, log2s, n_el);
    return hipGetLastError();
}

hipError_t launch_lam_init(double *lam, const double *phi0, const double *gcorr_last, int32_t s_user,
                           int32_t log2s, int64_t n_rows, hipStream_t st) {
    const int64_t n_el = n_rows << log2s;
    hipLaunchKernelGGL(k_lam_init, dim3((unsigned)grid_for(n_el)), dim3(kWG), 0, st, (d2 *)lam, (const d2 *)phi0,
                       (const d2 *)gcorr_last, s_user, log2s, n_el);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)grid_for(n)), dim3(kWG), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_grad_scatter(const void *gacc, const double *gdiag, const int64_t *ell_csr, int64_t ell_size,
                               bool cplx, double inv_f, double *grad_val, double *grad_onsite, const int32_t *perm,
                               int64_t n_rows, hipStream_t st) {
    const int64_t work = ell_size > n_rows ? ell_size : n_rows;
    if (cplx)
        hipLaunchKernelGGL(k_grad_scatter<true>, dim3((unsigned)grid_for(work)), dim3(kWG), 0, st, gacc, gdiag, ell_csr,
                           ell_size, inv_f, (d2 *)grad_val, grad_onsite, perm, n_rows);
    else
        hipLaunchKernelGGL(k_grad_scatter<false>, dim3((unsigned)grid_for(work)), dim3(kWG), 0, st, gacc, gdiag,
                           ell_csr, ell_size, inv_f, (d2 *)grad_val, grad_onsite, perm, n_rows);
    return hipGetLastError();
}

}  // namespace tbpm
