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
    const int tile = tile_of_block(blockIdx.x, p.n_tiles, p.xcd_remap, p.reverse);
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
        uint32_t base;
        int w;
        if (p.uniform_w > 0) {
            w = p.uniform_w;
            base = sl * (uint32_t)(p.uniform_w * kSliceRows) + row % kSliceRows;
        } else {
            const uint32_t off = soff[sl];
            w = (int)((soff[sl + 1] - off) / kSliceRows);
            base = off + row % kSliceRows;
        }
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
        // gw b at this row: the gradient of an element (p, q) is
        // gw Re/Im sum_s alpha_j[p] conj(b[q]); this row q forms it for its
        // transposed elements (q, p) from alpha_j at p (gathered anyway for
        // the product) and writes it to the slot of (p, q) (one writer per slot)
        const d2 bw = cmul(bs, bown) * gw;
        d2 acc;
        acc.x = on * a.x;
        acc.y = on * a.y;
        {
            // diagonal gradient: Re(alpha_j[p] conj(b[p])) summed over states
            const double dg = row_sum(a.x * bw.x + a.y * bw.y, log2s);
            if (s == 0) p.gdiag[row] = gd_old + dg;
        }
        for (int k = 0; k < w; k += KG) {
            uint32_t gc[KG];
            int32_t pt[KG];
            HV h[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                const bool valid = k + i < w;
                const uint32_t slot = valid ? base + (uint32_t)(k + i) * kSliceRows : 0u;
                const int32_t c = col[slot];
                const HV hv = val[slot];
                const int32_t ps = p.partner[slot];
                gc[i] = ((valid ? (uint32_t)c : row) << log2s) + s;
                h[i] = valid ? hv : HV{};
                pt[i] = valid ? ps : -1;  // -1: beyond the row or a padding slot
            }
            d2 xa[KG];
            GV gold[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                xa[i] = acur[gc[i]];
                gold[i] = pt[i] >= 0 ? gacc[pt[i]] : GV{};
            }
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                acc = hmad(h[i], xa[i], acc);
                // alpha_j[p] * conj(gw b[q]) summed over the states of the row
                const double gr = row_sum(xa[i].x * bw.x + xa[i].y * bw.y, log2s);
                if constexpr (CH) {
                    const double gi = row_sum(xa[i].y * bw.x - xa[i].x * bw.y, log2s);
                    if (s == 0 && pt[i] >= 0) {
                        d2 nv = gold[i];
                        nv.x += gr;
                        nv.y += gi;
                        gacc[pt[i]] = nv;
                    }
                } else {
                    if (s == 0 && pt[i] >= 0) gacc[pt[i]] = gold[i] + gr;
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

// Two adjoint orders per launch.  With alpha_j staged on the tile's own,
// 1-hop and 2-hop rows (xs), alpha_{j+1} = 2 H~ alpha_j - alpha_{j-1} (H~
// alpha_0 for the first pair) is evaluated on own and 1-hop rows (ys), then
// alpha_{j+2} = 2 H~ alpha_{j+1} - alpha_j on own rows.  On own rows the
// gradient slots take w1 alpha_j[p] conj(b_{j+1}[q]) + w2 alpha_{j+1}[p]
// conj(b_{j+2}[q]) summed over states in one read-modify-write, and lambda
// gains conj(c_{j+1}) alpha_{j+1} + conj(c_{j+2}) alpha_{j+2}.  A thread
// handles units of VS states; the staged-row indexing is that of k_pair.

// sum over the U consecutive lanes that hold the units of one row
__device__ __forceinline__ double unit_row_sum(double x, int log2u) {
    for (int off = 1; off < (1 << log2u); off <<= 1) x += __shfl_xor(x, off);
    return x;
}

// sum over the VS states of a unit of Re(a_i conj(b_i)) (im = false) or
// Im(a_i conj(b_i)) (im = true)
template <int VS>
__device__ __forceinline__ double unit_dot(const VecT<double, VS> &a, const VecT<double, VS> &b, bool im) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < VS; ++i)
        r += im ? (a[2 * i + 1] * b[2 * i] - a[2 * i] * b[2 * i + 1]) : (a[2 * i] * b[2 * i] + a[2 * i + 1] * b[2 * i + 1]);
    return r;
}

// acc += c * x for a complex scalar c and the VS components of x
template <int VS>
__device__ __forceinline__ void unit_cmad(d2 c, const VecT<double, VS> &x, VecT<double, VS> &acc) {
#pragma unroll
    for (int i = 0; i < VS; ++i) {
        acc[2 * i] = fma(c.x, x[2 * i], fma(-c.y, x[2 * i + 1], acc[2 * i]));
        acc[2 * i + 1] = fma(c.x, x[2 * i + 1], fma(c.y, x[2 * i], acc[2 * i + 1]));
    }
}

template <bool CH, int KIND, int VS>
__global__ __launch_bounds__(kWG) void k_adj_pair(const AdjPairParams p) {
    extern __shared__ __align__(16) unsigned char adj_mem[];
    using V = VecT<double, VS>;
    using HV = std::conditional_t<CH, d2, double>;
    using GV = std::conditional_t<CH, d2, double>;
    constexpr int KG = 4;
    constexpr bool FIRST = (KIND == kAdjPairFirst);
    constexpr int LOG2VS = VS == 4 ? 2 : (VS == 2 ? 1 : 0);
    const int tile = tile_of_block(blockIdx.x, p.n_tiles, p.xcd_remap, p.reverse);
    const TileDesc td = p.tiles[tile];
    const int log2u = p.log2s - LOG2VS;
    const uint32_t umask = (1u << log2u) - 1u;
    const uint32_t usub = threadIdx.x & umask;
    const uint32_t n_own = (uint32_t)td.rows;
    const uint32_t row0 = (uint32_t)td.row0;
    const int32_t e_beg = p.uoff[tile], e_end = p.uoff[tile + 1];
    const uint32_t n1 = (uint32_t)p.n1[tile];
    const uint32_t n_x = (n_own + (uint32_t)(e_end - e_beg)) << log2u;
    const uint32_t n_y = (n_own + n1) << log2u;
    const int32_t hoff = p.hoff[tile], hw = p.hw[tile];
    V *xs = reinterpret_cast<V *>(adj_mem);
    V *ys = xs + n_x;
    const V *__restrict__ x = (const V *)p.x;
    const V *__restrict__ bq1 = (const V *)p.bq1;
    const V *__restrict__ bq2 = (const V *)p.bq2;
    const HV *__restrict__ val = (const HV *)p.val;
    const uint32_t *__restrict__ soff = p.slice_off;
    const int32_t *__restrict__ ucol = p.ucol + e_beg;
    GV *gacc = (GV *)p.gacc;
    const double inv_f = p.inv_f;
    auto grow_of = [&](uint32_t lr) -> uint32_t { return lr < n_own ? row0 + lr : (uint32_t)ucol[lr - n_own]; };
    const int32_t uw = p.uniform_w;  // > 0: every slice has this width (no slice-offset load)
    auto slots_of = [&](uint32_t grow, uint32_t &base, int &w) {
        const uint32_t sl = grow / kSliceRows;
        if (uw > 0) {
            w = uw;
            base = sl * (uint32_t)(uw * kSliceRows) + grow % kSliceRows;
        } else {
            const uint32_t off = soff[sl];
            w = (int)((soff[sl + 1] - off) / kSliceRows);
            base = off + grow % kSliceRows;
        }
    };

    // stage alpha_j: four loads in flight per thread
    for (uint32_t i0 = threadIdx.x; i0 < n_x; i0 += 4 * kWG) {
        V t[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t i = i0 + (uint32_t)q * kWG;
            if (i < n_x) t[q] = x[(grow_of(i >> log2u) << log2u) + (i & umask)];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t i = i0 + (uint32_t)q * kWG;
            if (i < n_x) xs[i] = t[q];
        }
    }
    __syncthreads();

    // alpha_{j+1} on own + 1-hop rows
    for (uint32_t u = threadIdx.x; u < n_y; u += kWG) {
        const uint32_t lr = u >> log2u;
        const uint32_t grow = grow_of(lr);
        const uint32_t gu = (grow << log2u) + usub;
        uint32_t base;
        int w;
        slots_of(grow, base, w);
        V ap;
        if constexpr (!FIRST) ap = ((const V *)p.a_prev)[gu];
        V acc = p.onsite[grow] * xs[u];
        const bool own = lr < n_own;
        const uint16_t *hrow = p.hidx + hoff + (int64_t)(own ? 0 : (lr - n_own)) * hw;
        for (int k = 0; k < w; k += KG) {
            uint32_t li[KG];
            HV h[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                const bool valid = k + i < w;
                const uint32_t slot = valid ? base + (uint32_t)(k + i) * kSliceRows : 0u;
                const uint32_t l = valid ? (own ? (uint32_t)p.lidx[slot] : (uint32_t)hrow[k + i]) : lr;
                const HV hv = val[slot];
                li[i] = (l << log2u) + usub;
                h[i] = valid ? hv : HV{};
            }
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                if constexpr (CH)
                    unit_mad_cplx<double, VS>(h[i], xs[li[i]], acc);
                else
                    unit_mad_real<double, VS>(h[i], xs[li[i]], acc);
            }
        }
        V an;
        if constexpr (FIRST)
            an = acc * inv_f;
        else
            an = (2.0 * inv_f) * acc - ap;
        ys[u] = an;
        if (own) ((V *)p.out1)[gu] = an;
    }
    __syncthreads();

    // alpha_{j+2}, lambda and the gradient on own rows
    d2 cc0, cc1, cc2;
    cc0.x = p.cc0_re;
    cc0.y = p.cc0_im;
    cc1.x = p.cc1_re;
    cc1.y = p.cc1_im;
    cc2.x = p.cc2_re;
    cc2.y = p.cc2_im;
    const double w1 = p.w1, w2 = p.w2;
    const uint32_t n_u = n_own << log2u;
    // n_u is a multiple of the units per row and the units of a row are
    // consecutive lanes of one wave, so the lanes of a row take the same trip
    // counts
    for (uint32_t u = threadIdx.x; u < n_u; u += kWG) {
        const uint32_t lr = u >> log2u;
        const uint32_t row = row0 + lr;
        const uint32_t gu = (row << log2u) + usub;
        uint32_t base;
        int w;
        slots_of(row, base, w);
        const V aj = xs[u], aj1 = ys[u];
        V lam;
        if constexpr (!FIRST) lam = ((const V *)p.lam_acc)[gu];
        // b_{j+1}, b_{j+2} on this row, weighted: the gradient of an element
        // (p, q) is w1 Re/Im sum_s alpha_j[p] conj(b_{j+1}[q]) + w2 (alpha_{j+1},
        // b_{j+2}), so this row q forms it for its transposed elements (q, p)
        // from alpha at p (staged, own or 1-hop) and writes it to the slot of
        // (p, q); every slot has one transposed partner, so one writer
        const V b1w = bq1[gu] * w1, b2w = bq2[gu] * w2;
        {
            const double dg = unit_row_sum(unit_dot<VS>(aj, b1w, false) + unit_dot<VS>(aj1, b2w, false), log2u);
            if (usub == 0) p.gdiag[row] += dg;
        }
        V acc = p.onsite[row] * aj1;
        for (int k = 0; k < w; k += KG) {
            uint32_t li[KG];
            int32_t pt[KG];
            HV h[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                const bool valid = k + i < w;
                const uint32_t slot = valid ? base + (uint32_t)(k + i) * kSliceRows : 0u;
                const uint32_t l = valid ? (uint32_t)p.lidx[slot] : lr;
                const HV hv = val[slot];
                const int32_t ps = p.partner[slot];
                li[i] = (l << log2u) + usub;
                h[i] = valid ? hv : HV{};
                pt[i] = valid ? ps : -1;  // -1: beyond the row or a padding slot
            }
            GV gold[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) gold[i] = pt[i] >= 0 ? gacc[pt[i]] : GV{};
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                const V xp = xs[li[i]], yp = ys[li[i]];
                if constexpr (CH)
                    unit_mad_cplx<double, VS>(h[i], yp, acc);
                else
                    unit_mad_real<double, VS>(h[i], yp, acc);
                const double gr = unit_row_sum(unit_dot<VS>(xp, b1w, false) + unit_dot<VS>(yp, b2w, false), log2u);
                if constexpr (CH) {
                    const double gi =
                        unit_row_sum(unit_dot<VS>(xp, b1w, true) + unit_dot<VS>(yp, b2w, true), log2u);
                    if (usub == 0 && pt[i] >= 0) {
                        d2 nv = gold[i];
                        nv.x += gr;
                        nv.y += gi;
                        gacc[pt[i]] = nv;
                    }
                } else {
                    if (usub == 0 && pt[i] >= 0) gacc[pt[i]] = gold[i] + gr;
                }
            }
        }
        const V an2 = (2.0 * inv_f) * acc - aj;
        ((V *)p.out2)[gu] = an2;
        if constexpr (FIRST) {
            lam = V{};
            unit_cmad<VS>(cc0, aj, lam);
        }
        unit_cmad<VS>(cc1, aj1, lam);
        unit_cmad<VS>(cc2, an2, lam);
        ((V *)p.lam_acc)[gu] = lam;
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

template <bool CH, int VS>
hipError_t launch_adj_pair_t(int kind, const AdjPairParams &p, hipStream_t st) {
    const dim3 grid(p.n_tiles), block(kWG);
    const size_t lds = (size_t)p.lds_units * sizeof(VecT<double, VS>);
    if (kind == kAdjPairFirst)
        hipLaunchKernelGGL((k_adj_pair<CH, kAdjPairFirst, VS>), grid, block, lds, st, p);
    else
        hipLaunchKernelGGL((k_adj_pair<CH, kAdjPairMid, VS>), grid, block, lds, st, p);
    return hipGetLastError();
}

hipError_t launch_adjoint_pair(int kind, bool cplx, int vs, const AdjPairParams &p, hipStream_t st) {
    if (p.n_tiles <= 0) return hipSuccess;
    if (kind != kAdjPairFirst && kind != kAdjPairMid) return hipErrorInvalidValue;
    if (cplx) {
        if (vs == 4) return launch_adj_pair_t<true, 4>(kind, p, st);
        if (vs == 2) return launch_adj_pair_t<true, 2>(kind, p, st);
        return launch_adj_pair_t<true, 1>(kind, p, st);
    }
    if (vs == 4) return launch_adj_pair_t<false, 4>(kind, p, st);
    if (vs == 2) return launch_adj_pair_t<false, 2>(kind, p, st);
    return launch_adj_pair_t<false, 1>(kind, p, st);
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
