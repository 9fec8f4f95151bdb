// Two Clenshaw orders per launch (temporal blocking of depth 2) for gfx950.
//
// A pair of passes
//     b_j     = alpha1 v + beta1 H b_{j+1} - b_{j+2}
//     b_{j-1} = alpha2 v + beta2 H b_j     - b_{j+1}
// needs b_j on the tile's own rows and on their neighbours ("1-hop" rows).
// The workgroup of a tile therefore stages b_{j+1} for its own rows, the
// 1-hop rows and the neighbours of those (2-hop rows) in LDS, evaluates b_j
// on own + 1-hop rows into a second LDS array (writing the own rows to
// global memory as well), then evaluates b_{j-1} on its own rows from LDS.
// The 1-hop evaluation is redundant work shared with the neighbouring tiles;
// in exchange a pair streams psi, b_{j+2} and b_{j+1} once and writes two
// vectors, instead of reading six and writing two.  Outputs go to buffers
// that no tile of the launch reads.  The first pair of a step (x = psi, no
// b_{j+2}, b_{M-1} folded into alpha2) is the same kernel with KIND
// kPairFirst.  The last pair (KIND kPairLast) takes b_1 and the new state
//     psi' = c_0 psi + H~ b_1 - b_2
// (Eq. (eq:psi_t) by Clenshaw's recurrence): b_1 stays in LDS, and psi' is
// written to a buffer other than psi (other tiles still read psi on their
// 1-hop rows) with <phi0|psi'> and ||psi'||^2 accumulated as in the last
// single pass (Eq. (eq:corr_dos)).  When the first order of a step runs
// alone, the second pair (KIND kPairSecond) is a middle pair whose first
// order has no b_{j+2} term.  Per element the arithmetic is that of
// k_pass, so every result, the tile partials of the correlation included,
// is the one the single passes give on the same tiles.
//
// Latency: a workgroup's phases are chains of dependent loads.  When every
// slice has the same width (uniform_w > 0, e.g. graphene) a row's slots are
// computed without loading the slice offsets, and a thread whose first unit
// of order j is an own row keeps that row's first batch of matrix entries in
// registers for order j-1, which takes the same unit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "tbpm_internal.h"

namespace tbpm {
namespace {

template <typename R, bool CH, int KIND, bool NT, int VS>
__global__ __launch_bounds__(kWG) void k_pair(const FusedParams p) {
    extern __shared__ __align__(16) unsigned char pair_mem[];
    using V = VecT<R, VS>;
    using HV = typename HValT<R, CH>::T;
    constexpr int KG = 4;
    constexpr bool FIRST = (KIND == kPairFirst);
    constexpr bool LAST = (KIND == kPairLast);
    constexpr bool B2_1 = !FIRST && KIND != kPairSecond;  // order j subtracts b_{j+2}
    constexpr int LOG2VS = VS == 4 ? 2 : (VS == 2 ? 1 : 0);

    const int tile = tile_of_block(blockIdx.x, p.n_tiles, p.xcd_remap, p.reverse);
    const TileDesc td = p.tiles[tile];
    const PassCoef c1 = p.coef1[td.inst], c2 = p.coef2[td.inst];
    const int log2u = p.log2s - LOG2VS;
    const uint32_t umask = (1u << log2u) - 1u;
    const uint32_t usub = threadIdx.x & umask;
    const uint32_t n_own = (uint32_t)td.rows;
    const uint32_t row0 = (uint32_t)td.row0;
    const int32_t e_beg = p.uoff[tile], e_end = p.uoff[tile + 1];
    const uint32_t n1 = (uint32_t)p.n1[tile];
    const uint32_t n_x = (n_own + (uint32_t)(e_end - e_beg)) << log2u;  // staged b_{j+1}
    const uint32_t n_y = (n_own + n1) << log2u;                        // b_j rows
    const int32_t hoff = p.hoff[tile], hw = p.hw[tile];
    V *xs = reinterpret_cast<V *>(pair_mem);
    V *ys = xs + n_x;

    if (p.bump_counter && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(p.counter, 1);

    const V *__restrict__ x = (const V *)p.x;
    const V *__restrict__ v = (const V *)p.v;
    const V *__restrict__ b2 = (const V *)p.b2;
    V *__restrict__ out1 = (V *)p.out1;
    V *__restrict__ out2 = (V *)p.out2;
    const R *__restrict__ ons = (const R *)p.onsite;
    const HV *__restrict__ val = (const HV *)p.val;
    const uint32_t *__restrict__ soff = p.slice_off;
    const int32_t *__restrict__ ucol = p.ucol + e_beg;

    // global row of local staged row lr (own, then 1-hop, then 2-hop)
    auto grow_of = [&](uint32_t lr) -> uint32_t { return lr < n_own ? row0 + lr : (uint32_t)ucol[lr - n_own]; };

    // psi on the thread's first two own units, kept for the second order
    V vk0{}, vk1{};
    // the first batch of matrix entries of the thread's first unit when it is
    // an own row (the same unit in both orders), kept for the second order
    uint32_t kli[KG];
    HV kh[KG];
    const int32_t uw = p.uniform_w;
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

    // stage b_{j+1}: four independent loads in flight per thread
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

    // order j on own + 1-hop rows
    {
        const R ar = (R)c1.ar, ai = (R)c1.ai, br = (R)c1.br, bi = (R)c1.bi;
        int it = 0;
        for (uint32_t u = threadIdx.x; u < n_y; u += kWG, ++it) {
            const uint32_t lr = u >> log2u;
            const uint32_t grow = grow_of(lr);
            const uint32_t gu = (grow << log2u) + usub;
            uint32_t base;
            int w;
            slots_of(grow, base, w);
            V vv, bq;
            if constexpr (!FIRST) {
                vv = v[gu];
                if constexpr (B2_1) bq = (lr < n_own) ? ldv<NT>(b2 + gu) : b2[gu];
                if (it == 0) vk0 = vv;
                if (it == 1) vk1 = vv;
            }
            const V xo = xs[u];
            V acc = ons[grow] * xo;
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
                if (it == 0 && k == 0) {
#pragma unroll
                    for (int i = 0; i < KG; ++i) {
                        kli[i] = li[i];
                        kh[i] = h[i];
                    }
                }
#pragma unroll
                for (int i = 0; i < KG; ++i) {
                    if constexpr (CH)
                        unit_mad_cplx<R, VS>(h[i], xs[li[i]], acc);
                    else
                        unit_mad_real<R, VS>(h[i], xs[li[i]], acc);
                }
            }
            const V src = FIRST ? xo : vv;
            V o;
#pragma unroll
            for (int i = 0; i < VS; ++i) {
                const R vr = src[2 * i], vi = src[2 * i + 1];
                const R hr = acc[2 * i], hi = acc[2 * i + 1];
                o[2 * i] = ar * vr - ai * vi + (br * hr - bi * hi);
                o[2 * i + 1] = ar * vi + ai * vr + (br * hi + bi * hr);
            }
            if constexpr (B2_1) o -= bq;
            ys[u] = o;
            if constexpr (!LAST)
                if (own) stv<NT>(out1 + gu, o);
        }
    }
    __syncthreads();

    // order j-1 on own rows
    double dre[VS], dim[VS], nrm[VS];
#pragma unroll
    for (int i = 0; i < VS; ++i) dre[i] = dim[i] = nrm[i] = 0.0;
    {
        const R ar = (R)c2.ar, ai = (R)c2.ai, br = (R)c2.br, bi = (R)c2.bi;
        const uint32_t n_u = n_own << log2u;
        int it = 0;
        for (uint32_t u = threadIdx.x; u < n_u; u += kWG, ++it) {
            const uint32_t lr = u >> log2u;
            const uint32_t row = row0 + lr;
            const uint32_t gu = (row << log2u) + usub;
            uint32_t base;
            int w;
            slots_of(row, base, w);
            V vv;
            if constexpr (FIRST)
                vv = xs[u];
            else
                vv = it == 0 ? vk0 : (it == 1 ? vk1 : v[gu]);
            d2 ph[LAST ? VS : 1];  // phi0 of this unit, loaded before the gathers
            if constexpr (LAST) {
#pragma unroll
                for (int i = 0; i < VS; ++i)
                    ph[i] = ((const d2 *)p.phi0)[(int64_t)row * p.phi0_ld + (usub << LOG2VS) + i];
            }
            V acc = ons[row] * ys[u];
            for (int k = 0; k < w; k += KG) {
                uint32_t li[KG];
                HV h[KG];
                if (it == 0 && k == 0) {  // this unit was the thread's first of order j
#pragma unroll
                    for (int i = 0; i < KG; ++i) {
                        li[i] = kli[i];
                        h[i] = kh[i];
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < KG; ++i) {
                        const bool valid = k + i < w;
                        const uint32_t slot = valid ? base + (uint32_t)(k + i) * kSliceRows : 0u;
                        const uint32_t l = valid ? (uint32_t)p.lidx[slot] : lr;
                        const HV hv = val[slot];
                        li[i] = (l << log2u) + usub;
                        h[i] = valid ? hv : HV{};
                    }
                }
#pragma unroll
                for (int i = 0; i < KG; ++i) {
                    if constexpr (CH)
                        unit_mad_cplx<R, VS>(h[i], ys[li[i]], acc);
                    else
                        unit_mad_real<R, VS>(h[i], ys[li[i]], acc);
                }
            }
            V o;
#pragma unroll
            for (int i = 0; i < VS; ++i) {
                const R vr = vv[2 * i], vi = vv[2 * i + 1];
                const R hr = acc[2 * i], hi = acc[2 * i + 1];
                o[2 * i] = ar * vr - ai * vi + (br * hr - bi * hi);
                o[2 * i + 1] = ar * vi + ai * vr + (br * hi + bi * hr);
            }
            if constexpr (!FIRST) o -= xs[u];  // b_{j+1} on own rows
            stv<NT>(out2 + gu, o);
            if constexpr (LAST) {
#pragma unroll
                for (int i = 0; i < VS; ++i) {
                    const double oxr = (double)o[2 * i], oyi = (double)o[2 * i + 1];
                    dre[i] = fma(ph[i].x, oxr, fma(ph[i].y, oyi, dre[i]));
                    dim[i] = fma(ph[i].x, oyi, fma(-ph[i].y, oxr, dim[i]));
                    nrm[i] = fma(oxr, oxr, fma(oyi, oyi, nrm[i]));
                }
            }
        }
    }
    if constexpr (LAST) {
        __syncthreads();  // the staged rows are dead: their LDS takes the partial sums
        block_unit_partials<VS>(dre, dim, nrm, log2u, p.partials, tile, p.n_tiles,
                                reinterpret_cast<double (*)[64][3]>(pair_mem));
    }
}

template <typename R, bool CH, bool NT, int VS>
hipError_t launch_pair_t(int kind, const FusedParams &p, hipStream_t st) {
    const dim3 grid(p.n_tiles), block(kWG);
    const size_t lds = (size_t)p.lds_units * sizeof(VecT<R, VS>);
    if (kind == kPairFirst)
        hipLaunchKernelGGL((k_pair<R, CH, kPairFirst, NT, VS>), grid, block, lds, st, p);
    else if (kind == kPairMid)
        hipLaunchKernelGGL((k_pair<R, CH, kPairMid, NT, VS>), grid, block, lds, st, p);
    else if (kind == kPairSecond)
        hipLaunchKernelGGL((k_pair<R, CH, kPairSecond, NT, VS>), grid, block, lds, st, p);
    else if (kind == kPairLast)  // the partial sums reuse the LDS: at least kWG/64 x 64 x 3 doubles
        hipLaunchKernelGGL((k_pair<R, CH, kPairLast, NT, VS>), grid, block,
                           std::max(lds, sizeof(double) * kWG * 3), st, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename R, int VS>
hipError_t launch_pair_r(int kind, bool cplx, bool nt, const FusedParams &p, hipStream_t st) {
    if (cplx) return nt ? launch_pair_t<R, true, true, VS>(kind, p, st) : launch_pair_t<R, true, false, VS>(kind, p, st);
    return nt ? launch_pair_t<R, false, true, VS>(kind, p, st) : launch_pair_t<R, false, false, VS>(kind, p, st);
}

}  // namespace

hipError_t launch_pair(int kind, bool fp32, bool cplx, bool nontemporal, int vs, const FusedParams &p,
                       hipStream_t st) {
    if (p.n_tiles <= 0) return hipSuccess;
    if (fp32) {
        if (vs == 4) return launch_pair_r<float, 4>(kind, cplx, nontemporal, p, st);
        if (vs == 2) return launch_pair_r<float, 2>(kind, cplx, nontemporal, p, st);
        return launch_pair_r<float, 1>(kind, cplx, nontemporal, p, st);
    }
    if (vs == 4) return launch_pair_r<double, 4>(kind, cplx, nontemporal, p, st);
    if (vs == 2) return launch_pair_r<double, 2>(kind, cplx, nontemporal, p, st);
    return launch_pair_r<double, 1>(kind, cplx, nontemporal, p, st);
}

}  // namespace tbpm
