// HIP kernels of the TBPM forward path for gfx950 (MI355X).
//
// One time step of the propagation evaluates psi' = sum_{m<M} c_m T_m(H~) psi
// (paper, Sec. "Tight-binding propagation method", Eq. (eq:psi_t) with the
// Jacobi-Anger coefficients c_0 = J_0(z), c_m = 2(-i)^m J_m(z)) by Clenshaw's
// recurrence
//     b_j = c_j psi + 2 H~ b_{j+1} - b_{j+2},   j = M-1 .. 1,  b_M = b_{M+1} = 0
//     psi' = c_0 psi + H~ b_1 - b_2,
// one sparse pass per j.  Every pass is the same streaming kernel,
//     out = alpha * v + beta * (H x) - b2,
// with per-batch-member (alpha, beta) chosen by the host; the last pass also
// accumulates <phi0|psi'> and ||psi'||^2 (Eq. (eq:corr_dos)) in FP64.
//
// The operator is a sparse stencil (arithmetic intensity ~0.4 flop/byte), so
// these kernels are HBM-bound and use no matrix cores: one thread per
// (row, state) element with the S states of a row contiguous, so that the
// gather of x at a neighbour column reads S*16 (FP64) contiguous bytes.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_util.h"
#include "tbpm_internal.h"

namespace tbpm {
namespace {

// ---------------------------------------------------------------------------
// Chebyshev/Clenshaw pass
//
// A thread owns "units" of VS consecutive states of one row (VS = 2 packs two
// complex64 states into one 16-byte access) and handles NE units at a time,
// 256 units apart.  Every load that does not depend on a column index (own
// x, on-site, psi, b2, the slice offsets) is issued first; the stored
// elements of a row are then taken KG at a time, with all their column and
// value loads in flight before the KG gathers of x.  Indices are 32-bit
// (the host keeps rows*S < 2^31 and the ELL size < 2^32).
// ---------------------------------------------------------------------------
template <typename R, bool CH, int KIND, bool NT, int VS, int NE>
__global__ __launch_bounds__(kWG) void k_pass(const PassParams p) {
    using V = VecT<R, VS>;
    using HV = typename HValT<R, CH>::T;
    constexpr int KG = 4;
    constexpr bool X_IS_V = (KIND == kPassFirst);
    constexpr bool HAS_B2 = (KIND == kPassMid || KIND == kPassLast);
    constexpr bool CORR = (KIND == kPassLast || KIND == kPassLastNoB2);
    constexpr int LOG2VS = VS == 4 ? 2 : (VS == 2 ? 1 : 0);

    const int tile = tile_of_block(blockIdx.x, p.n_tiles, p.xcd_remap, p.reverse);
    const TileDesc td = p.tiles[tile];
    const PassCoef pc = p.coef[td.inst];
    const R ar = (R)pc.ar, ai = (R)pc.ai, br = (R)pc.br, bi = (R)pc.bi;
    const int log2s = p.log2s;
    const int log2u = log2s - LOG2VS;
    const uint32_t umask = (1u << log2u) - 1u;
    const uint32_t n_u = (uint32_t)td.rows << log2u;
    const uint32_t row0 = (uint32_t)td.row0;
    const uint32_t u0 = row0 << log2u;

    if (p.bump_counter && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(p.counter, 1);

    const V *__restrict__ x = (const V *)p.x;
    const V *v = (const V *)p.v;
    const V *b2 = (const V *)p.b2;
    V *out = (V *)p.out;
    const R *__restrict__ ons = (const R *)p.onsite;
    const HV *__restrict__ val = (const HV *)p.val;
    const int32_t *__restrict__ col = p.col;
    const uint32_t *__restrict__ soff = p.slice_off;
    const uint32_t usub = threadIdx.x & umask;  // this thread's unit inside a row
    const int32_t uw = p.uniform_w;  // > 0: every slice has this width (no slice-offset load)

    double dre[VS], dim[VS], nrm[VS];
#pragma unroll
    for (int i = 0; i < VS; ++i) dre[i] = dim[i] = nrm[i] = 0.0;
    bool do_ckpt = false;
    uint32_t ckpt_base = 0;
    if constexpr (CORR) {
        if (p.ckpt_slot) {
            // the step counter holds k of the psi(k dt) this pass produces
            const int step = *(volatile const int32_t *)p.counter;
            const int slot = p.ckpt_slot[step];
            do_ckpt = slot >= 0;
            ckpt_base = (uint32_t)(do_ckpt ? slot : 0);
        }
    }

    for (uint32_t ub = threadIdx.x; ub < n_u; ub += kWG * NE) {
        uint32_t row[NE], gu[NE], base[NE];
        int w[NE];
        bool ok[NE];
        V xo[NE], vv[NE], bq[NE];
        R on[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            uint32_t u = ub + q * kWG;
            ok[q] = u < n_u;
            if (!ok[q]) u = ub;  // a valid unit; its result is not stored
            row[q] = row0 + (u >> log2u);
            gu[q] = u0 + u;
            const uint32_t sl = row[q] / kSliceRows;
            if (uw > 0) {
                w[q] = uw;
                base[q] = sl * (uint32_t)(uw * kSliceRows) + row[q] % kSliceRows;
            } else {
                const uint32_t off = soff[sl];
                w[q] = (int)((soff[sl + 1] - off) / kSliceRows);
                base[q] = off + row[q] % kSliceRows;
            }
            xo[q] = x[gu[q]];
            on[q] = ons[row[q]];
            if constexpr (!X_IS_V) vv[q] = ldv<NT>(v + gu[q]);
            if constexpr (HAS_B2) bq[q] = ldv<NT>(b2 + gu[q]);
        }
        V acc[NE];
        int wmax = 0;
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            acc[q] = on[q] * xo[q];
            wmax = max(wmax, w[q]);
        }
        for (int k = 0; k < wmax; k += KG) {
            uint32_t cu[NE][KG];
            HV h[NE][KG];
#pragma unroll
            for (int q = 0; q < NE; ++q) {
#pragma unroll
                for (int i = 0; i < KG; ++i) {
                    const bool valid = k + i < w[q];
                    const uint32_t slot = valid ? base[q] + (uint32_t)(k + i) * kSliceRows : 0u;
                    const int32_t c = col[slot];
                    const HV hv = val[slot];
                    cu[q][i] = ((valid ? (uint32_t)c : row[q]) << log2u) + usub;
                    h[q][i] = valid ? hv : HV{};
                }
            }
            V xc[NE][KG];
#pragma unroll
            for (int q = 0; q < NE; ++q)
#pragma unroll
                for (int i = 0; i < KG; ++i) xc[q][i] = x[cu[q][i]];
#pragma unroll
            for (int q = 0; q < NE; ++q)
#pragma unroll
                for (int i = 0; i < KG; ++i) {
                    if constexpr (CH)
                        unit_mad_cplx<R, VS>(h[q][i], xc[q][i], acc[q]);
                    else
                        unit_mad_real<R, VS>(h[q][i], xc[q][i], acc[q]);
                }
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const V src = X_IS_V ? xo[q] : vv[q];
            V o;
#pragma unroll
            for (int i = 0; i < VS; ++i) {
                const R vr = src[2 * i], vi = src[2 * i + 1];
                const R hr = acc[q][2 * i], hi = acc[q][2 * i + 1];
                o[2 * i] = ar * vr - ai * vi + (br * hr - bi * hi);
                o[2 * i + 1] = ar * vi + ai * vr + (br * hi + bi * hr);
            }
            if constexpr (HAS_B2) o -= bq[q];
            if (!ok[q]) continue;
            if constexpr (CORR) {
                stv<false>(out + gu[q], o);
                const uint32_t s0 = usub << LOG2VS;
#pragma unroll
                for (int i = 0; i < VS; ++i) {
                    const d2 ph = ((const d2 *)p.phi0)[(int64_t)row[q] * p.phi0_ld + s0 + i];
                    const double oxr = (double)o[2 * i], oyi = (double)o[2 * i + 1];
                    dre[i] = fma(ph.x, oxr, fma(ph.y, oyi, dre[i]));
                    dim[i] = fma(ph.x, oyi, fma(-ph.y, oxr, dim[i]));
                    nrm[i] = fma(oxr, oxr, fma(oyi, oyi, nrm[i]));
                    if (do_ckpt && (int)(s0 + i) < p.s_user) {
                        d2 oc;
                        oc.x = oxr;
                        oc.y = oyi;
                        const int64_t crow = p.perm ? (int64_t)p.perm[row[q]] : (int64_t)row[q];
                        ((d2 *)p.ckpt)[(int64_t)ckpt_base * p.ckpt_stride + crow * p.s_user + s0 + i] = oc;
                    }
                }
            } else {
                stv<NT>(out + gu[q], o);
            }
        }
    }
    if constexpr (CORR) block_unit_partials<VS>(dre, dim, nrm, log2u, p.partials, tile, p.n_tiles);
}

// ---------------------------------------------------------------------------
// Clenshaw pass with the gathered vector staged in LDS.  The workgroup of
// tile t first copies the rows of x it will read -- its own rows, then the
// tile's sorted list of external rows -- into LDS (each row is read from
// global memory once per tile instead of once per stored element that
// references it), then evaluates the pass with every neighbour read from
// LDS through the slot's precomputed local index.  Same arithmetic as
// k_pass, so results are identical.  A row's stored elements are taken KG at
// a time (indices and values loaded together, then the LDS reads): 4 for
// narrow rows, 12 for wide ones, where fewer dependent rounds of loads per
// row matter more than the padded slots of the last batch.  Rows wider than
// the LDS row width are taken one block of states (2^log2ub units) per
// workgroup, so the LDS holds rows of one block; the blocks of a tile run on
// one XCD at about the same time, so that the tile's matrix entries come
// from HBM once and the other blocks find them in that XCD's L2.
// ---------------------------------------------------------------------------
template <typename R, bool CH, int KIND, bool NT, int VS, int KG>
__global__ __launch_bounds__(kWG) void k_pass_staged(const PassParams p) {
    extern __shared__ __align__(16) unsigned char stage_mem[];
    using V = VecT<R, VS>;
    using HV = typename HValT<R, CH>::T;
    constexpr bool X_IS_V = (KIND == kPassFirst);
    constexpr bool HAS_B2 = (KIND == kPassMid || KIND == kPassLast);
    constexpr bool CORR = (KIND == kPassLast || KIND == kPassLastNoB2);
    constexpr int LOG2VS = VS == 4 ? 2 : (VS == 2 ? 1 : 0);
    V *xs = reinterpret_cast<V *>(stage_mem);

    const int log2u = p.log2s - LOG2VS;  // units of a whole row
    const int log2ub = p.log2ub;         // units of one state block of a row
    const int n_blk = 1 << (log2u - log2ub);
    // the block of states of this workgroup: with several blocks, workgroup
    // g takes block (g >> 3) % n_blk of tile slot ((g >> 3) / n_blk) * 8 +
    // (g & 7), so the blocks of a tile run on one XCD (workgroups are
    // dispatched to XCD g & 7) at about the same time and the later ones find
    // the tile's matrix entries in that XCD's L2
    int blk = 0, tslot = (int)blockIdx.x;
    if (n_blk > 1) {
        const int r = (int)blockIdx.x >> 3;
        blk = r % n_blk;
        tslot = (r / n_blk) * 8 + ((int)blockIdx.x & 7);
        if (tslot >= p.n_tiles) return;  // the last group of 8 slots is partial
    }
    const uint32_t boff = (uint32_t)blk << log2ub;  // unit offset of the block in a row
    const int tile = tile_of_block(tslot, p.n_tiles, p.xcd_remap, p.reverse);
    const TileDesc td = p.tiles[tile];
    const PassCoef pc = p.coef[td.inst];
    const R ar = (R)pc.ar, ai = (R)pc.ai, br = (R)pc.br, bi = (R)pc.bi;
    const uint32_t umask = (1u << log2ub) - 1u;
    const uint32_t n_own = (uint32_t)td.rows;
    const uint32_t n_u = n_own << log2ub;
    const uint32_t row0 = (uint32_t)td.row0;
    const int32_t x0 = p.uoff[tile], x1 = p.uoff[tile + 1];
    const uint32_t n_stage = (n_own + (uint32_t)(x1 - x0)) << log2ub;

    if (p.bump_counter && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(p.counter, 1);

    const V *__restrict__ x = (const V *)p.x;
    const V *v = (const V *)p.v;
    const V *b2 = (const V *)p.b2;
    V *out = (V *)p.out;
    const R *__restrict__ ons = (const R *)p.onsite;
    const HV *__restrict__ val = (const HV *)p.val;
    const uint16_t *__restrict__ lidx = p.lidx;
    const uint32_t *__restrict__ soff = p.slice_off;
    const uint32_t usub = threadIdx.x & umask;

    bool do_ckpt = false;
    uint32_t ckpt_base = 0;
    if constexpr (CORR) {
        if (p.ckpt_slot) {
            // the step counter holds k of the psi(k dt) this pass produces
            const int step = *(volatile const int32_t *)p.counter;
            const int slot = p.ckpt_slot[step];
            do_ckpt = slot >= 0;
            ckpt_base = (uint32_t)(do_ckpt ? slot : 0);
        }
    }

    // stage the rows: four units per thread in flight, their row indices
    // (the external rows' through the tile's list) loaded first, then the
    // rows, then the LDS writes
    for (uint32_t i0 = threadIdx.x; i0 < n_stage; i0 += 4 * kWG) {
        uint32_t g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t i = i0 + (uint32_t)q * kWG;
            const uint32_t lr = i >> log2ub;
            uint32_t grow = row0 + lr;
            if (i < n_stage && lr >= n_own) grow = (uint32_t)p.ucol[x0 + (int32_t)(lr - n_own)];
            g[q] = (grow << log2u) + boff + (i & umask);
        }
        V t[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (i0 + (uint32_t)q * kWG < n_stage) t[q] = x[g[q]];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t i = i0 + (uint32_t)q * kWG;
            if (i < n_stage) xs[i] = t[q];
        }
    }
    __syncthreads();

    double dre[VS], dim[VS], nrm[VS];
#pragma unroll
    for (int i = 0; i < VS; ++i) dre[i] = dim[i] = nrm[i] = 0.0;

    for (uint32_t u = threadIdx.x; u < n_u; u += kWG) {
        const uint32_t lrow = u >> log2ub;
        const uint32_t row = row0 + lrow;
        const uint32_t gu = (row << log2u) + boff + usub;
        const uint32_t sl = row / kSliceRows;
        const uint32_t off = soff[sl];
        const int w = (int)((soff[sl + 1] - off) / kSliceRows);
        const uint32_t base = off + row % kSliceRows;
        V vv, bq;
        if constexpr (!X_IS_V) vv = ldv<NT>(v + gu);
        if constexpr (HAS_B2) bq = ldv<NT>(b2 + gu);
        const V xo = xs[u];
        V acc = ons[row] * xo;
        for (int k = 0; k < w; k += KG) {
            uint32_t li[KG];
            HV h[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                const bool valid = k + i < w;
                const uint32_t slot = valid ? base + (uint32_t)(k + i) * kSliceRows : 0u;
                const uint32_t l = lidx[slot];
                const HV hv = val[slot];
                li[i] = ((valid ? l : lrow) << log2ub) + usub;
                h[i] = valid ? hv : HV{};
            }
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                if constexpr (CH)
                    unit_mad_cplx<R, VS>(h[i], xs[li[i]], acc);
                else
                    unit_mad_real<R, VS>(h[i], xs[li[i]], acc);
            }
        }
        const V src = X_IS_V ? xo : vv;
        V o;
#pragma unroll
        for (int i = 0; i < VS; ++i) {
            const R vr = src[2 * i], vi = src[2 * i + 1];
            const R hr = acc[2 * i], hi = acc[2 * i + 1];
            o[2 * i] = ar * vr - ai * vi + (br * hr - bi * hi);
            o[2 * i + 1] = ar * vi + ai * vr + (br * hi + bi * hr);
        }
        if constexpr (HAS_B2) o -= bq;
        if constexpr (CORR) {
            stv<false>(out + gu, o);
            const uint32_t s0 = (boff + usub) << LOG2VS;  // first state of the unit
#pragma unroll
            for (int i = 0; i < VS; ++i) {
                const d2 ph = ((const d2 *)p.phi0)[(int64_t)row * p.phi0_ld + s0 + i];
                const double oxr = (double)o[2 * i], oyi = (double)o[2 * i + 1];
                dre[i] = fma(ph.x, oxr, fma(ph.y, oyi, dre[i]));
                dim[i] = fma(ph.x, oyi, fma(-ph.y, oxr, dim[i]));
                nrm[i] = fma(oxr, oxr, fma(oyi, oyi, nrm[i]));
                if (do_ckpt && (int)(s0 + i) < p.s_user) {
                    d2 oc;
                    oc.x = oxr;
                    oc.y = oyi;
                    const int64_t crow = p.perm ? (int64_t)p.perm[row] : (int64_t)row;
                    ((d2 *)p.ckpt)[(int64_t)ckpt_base * p.ckpt_stride + crow * p.s_user + s0 + i] = oc;
                }
            }
        } else {
            stv<NT>(out + gu, o);
        }
    }
    // partials of the block's states: [S][3][n_tiles] from state blk * (units of a block) * VS on
    if constexpr (CORR)
        block_unit_partials<VS>(dre, dim, nrm, log2ub,
                                p.partials + (int64_t)(boff << LOG2VS) * 3 * p.n_tiles, tile, p.n_tiles);
}

// ---------------------------------------------------------------------------
// Initial state: v = psi0 (rounded to the recursion precision), phi0 = psi0
// padded to the power-of-two state count, and the partial sums of C_0.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kWG) void k_init(const InitParams p) {
    using C = typename CxT<R>::T;
    const TileDesc td = p.tiles[blockIdx.x];
    const int log2s = p.log2s;
    const int64_t smask = (1 << log2s) - 1;
    const int64_t n_el = (int64_t)td.rows << log2s;
    const int64_t e0 = td.row0 << log2s;
    const d2 *__restrict__ src = (const d2 *)p.psi0[td.inst];
    const int64_t lrow0 = td.row0 - p.inst_row0[td.inst];
    C *v = (C *)p.v;
    d2 *phi0 = (d2 *)p.phi0;
    double dre = 0.0, dim = 0.0, nrm = 0.0;
    for (int64_t e = threadIdx.x; e < n_el; e += kWG) {
        const int64_t lrow = p.perm ? (int64_t)p.perm[td.row0 + (e >> log2s)] : lrow0 + (e >> log2s);
        const int s = (int)(e & smask);
        d2 a;
        a.x = 0.0;
        a.y = 0.0;
        if (s < p.s_user) a = src[lrow * p.s_user + s];
        C o;
        o.x = (R)a.x;
        o.y = (R)a.y;
        v[e0 + e] = o;
        phi0[e0 + e] = a;
        const double ox = (double)o.x, oy = (double)o.y;
        dre = fma(a.x, ox, fma(a.y, oy, dre));
        dim = fma(a.x, oy, fma(-a.y, ox, dim));
        nrm = fma(ox, ox, fma(oy, oy, nrm));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(p.counter, 0);
    block_state_partials(dre, dim, nrm, log2s, p.partials, blockIdx.x, p.n_tiles);
}

// ---------------------------------------------------------------------------
// Second stage of the correlation: one workgroup per (member, state) sums
// the per-tile partials of that member in a fixed order and writes
// corr[k][s], norm2[k][s] for the current step k.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_reduce(const ReduceParams p) {
    __shared__ double red[3][kWG];
    const int inst = blockIdx.x / p.s_user;
    const int s = blockIdx.x % p.s_user;
    const int t0 = p.inst_tile0[inst], t1 = p.inst_tile0[inst + 1];
    const int64_t nt = p.n_tiles;
    const double *q0 = p.partials + (int64_t)s * 3 * nt;
    // four independent accumulators per component keep several loads in flight;
    // the summation order is fixed
    double a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
    int t = t0 + threadIdx.x;
    for (; t + 3 * kWG < t1; t += 4 * kWG) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] += q0[t + u * kWG];
            b[u] += q0[nt + t + u * kWG];
            c[u] += q0[2 * nt + t + u * kWG];
        }
    }
    for (; t < t1; t += kWG) {
        a[0] += q0[t];
        b[0] += q0[nt + t];
        c[0] += q0[2 * nt + t];
    }
    red[0][threadIdx.x] = (a[0] + a[1]) + (a[2] + a[3]);
    red[1][threadIdx.x] = (b[0] + b[1]) + (b[2] + b[3]);
    red[2][threadIdx.x] = (c[0] + c[1]) + (c[2] + c[3]);
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
            red[2][threadIdx.x] += red[2][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int k = *(volatile const int32_t *)p.counter;
        if (k >= 0 && k < p.n_steps) {
            const int64_t o = (int64_t)k * p.s_user + s;
            d2 cc;
            cc.x = red[0][0];
            cc.y = red[1][0];
            ((d2 *)p.corr[inst])[o] = cc;
            if (p.norm2[inst]) p.norm2[inst][o] = red[2][0];
            if (p.norm2_all) p.norm2_all[(int64_t)inst * p.n_steps * p.s_user + o] = red[2][0];
        }
    }
}

// ---------------------------------------------------------------------------
// DOS by direct windowed Fourier sum (paper, Eq. (dos_tbpm)); the phase
// E_j t_k = pi (j k mod 2N)/N is reduced exactly in integers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double window_w(int k, int n, int window) {
    return window == TBPM_WIN_HANN ? 0.5 * (1.0 + cospi((double)k / (double)n)) : 1.0;
}

// Neumaier-compensated accumulation
__device__ __forceinline__ void kadd(double &sum, double &comp, double x) {
    const double t = sum + x;
    comp += (fabs(sum) >= fabs(x)) ? (sum - t) + x : (x - t) + sum;
    sum = t;
}

__global__ __launch_bounds__(kWG) void k_dos(const double *__restrict__ corr, int nt, int S, double dt,
                                             int window, double *__restrict__ energies,
                                             double *__restrict__ dos) {
    __shared__ double cre[kWG], cim[kWG];
    const int jidx = blockIdx.x * kWG + threadIdx.x;
    const int64_t j = (int64_t)jidx - nt;
    const int64_t two_n = 2 * (int64_t)nt;
    double sum = 0.0, comp = 0.0;
    for (int k0 = 0; k0 < nt; k0 += kWG) {
        const int k = k0 + threadIdx.x;
        double r = 0.0, i = 0.0;
        if (k < nt) {
            const d2 *row = (const d2 *)corr + (int64_t)k * S;
            for (int s = 0; s < S; ++s) {
                r += row[s].x;
                i += row[s].y;
            }
            const double w = window_w(k, nt, window) * (k == 0 ? 1.0 : 2.0) / (double)S;
            r *= w;
            i *= w;
        }
        cre[threadIdx.x] = r;
        cim[threadIdx.x] = i;
        __syncthreads();
        const int kn = min(kWG, nt - k0);
        if (jidx < two_n) {
            for (int kk = 0; kk < kn; ++kk) {
                const int64_t kg = k0 + kk;
                int64_t m = (j * kg) % two_n;
                if (m < 0) m += two_n;
                double sn, cs;
                sincospi((double)m / (double)nt, &sn, &cs);
                kadd(sum, comp, cre[kk] * cs - cim[kk] * sn);
            }
        }
        __syncthreads();
    }
    if (jidx < two_n) {
        energies[jidx] = (double)j * M_PI / ((double)nt * dt);
        dos[jidx] = (sum + comp) * dt / (2.0 * M_PI);
    }
}

// Adjoint of k_dos: gcorr[k][s] = (1/S) (dt/pi) w_k sum_j g_j e^{-i E_j t_k}
// for k >= 1 and (1/S)(dt/2pi) w_0 sum_j g_j for k = 0.
__global__ __launch_bounds__(kWG) void k_dos_backward(const double *__restrict__ gdos, int nt, int S,
                                                      double dt, int window,
                                                      double *__restrict__ gcorr) {
    __shared__ double g[kWG];
    const int k = blockIdx.x * kWG + threadIdx.x;
    const int64_t two_n = 2 * (int64_t)nt;
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    for (int64_t j0 = 0; j0 < two_n; j0 += kWG) {
        const int64_t jj = j0 + threadIdx.x;
        g[threadIdx.x] = jj < two_n ? gdos[jj] : 0.0;
        __syncthreads();
        const int jn = (int)min((int64_t)kWG, two_n - j0);
        if (k < nt) {
            for (int q = 0; q < jn; ++q) {
                const int64_t j = j0 + q - nt;
                int64_t m = (j * (int64_t)k) % two_n;
                if (m < 0) m += two_n;
                double sn, cs;
                sincospi((double)m / (double)nt, &sn, &cs);
                kadd(sr, cr, g[q] * cs);
                kadd(si, ci, -g[q] * sn);
            }
        }
        __syncthreads();
    }
    if (k < nt) {
        const double w = window_w(k, nt, window) * (k == 0 ? 0.5 : 1.0) * dt / M_PI / (double)S;
        d2 o;
        o.x = (sr + cr) * w;
        o.y = (k == 0) ? 0.0 : (si + ci) * w;
        for (int s = 0; s < S; ++s) ((d2 *)gcorr)[(int64_t)k * S + s] = o;
    }
}

// ---------------------------------------------------------------------------
// Value refresh: CSR-ordered values (device) -> sliced-ELL FP64/FP32 copies.
// ---------------------------------------------------------------------------
template <bool CH>
__global__ __launch_bounds__(kWG) void k_convert_values(const int64_t *__restrict__ ell_csr, int64_t ell_size,
                                                        const double *__restrict__ csr_val,
                                                        const double *__restrict__ csr_onsite,
                                                        int64_t n_rows, const int32_t *__restrict__ perm,
                                                        void *val64, void *val32, double *ons64, float *ons32) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t q = (int64_t)blockIdx.x * kWG + threadIdx.x; q < ell_size; q += stride) {
        const int64_t pos = ell_csr[q];
        double re = 0.0, im = 0.0;
        if (pos >= 0) {
            re = csr_val[2 * pos];
            im = csr_val[2 * pos + 1];
        }
        if constexpr (CH) {
            d2 a;
            a.x = re;
            a.y = im;
            f2 b;
            b.x = (float)re;
            b.y = (float)im;
            ((d2 *)val64)[q] = a;
            ((f2 *)val32)[q] = b;
        } else {
            ((double *)val64)[q] = re;
            ((float *)val32)[q] = (float)re;
        }
    }
    for (int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x; r < n_rows; r += stride) {
        const double e = csr_onsite[perm ? perm[r] : r];
        ons64[r] = e;
        ons32[r] = (float)e;
    }
}

// Plain streaming copy (bandwidth calibration).
__global__ __launch_bounds__(kWG) void k_copy(const d2 *__restrict__ src, d2 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename R, bool CH, bool NT, int VS, int NE>
hipError_t launch_pass_t(int kind, const PassParams &p, hipStream_t st) {
    const dim3 grid(p.n_tiles), block(kWG);
    switch (kind) {
        case kPassFirst:
            hipLaunchKernelGGL((k_pass<R, CH, kPassFirst, NT, VS, NE>), grid, block, 0, st, p);
            break;
        case kPassNoB2:
            hipLaunchKernelGGL((k_pass<R, CH, kPassNoB2, NT, VS, NE>), grid, block, 0, st, p);
            break;
        case kPassMid:
            hipLaunchKernelGGL((k_pass<R, CH, kPassMid, NT, VS, NE>), grid, block, 0, st, p);
            break;
        case kPassLast:
            hipLaunchKernelGGL((k_pass<R, CH, kPassLast, NT, VS, NE>), grid, block, 0, st, p);
            break;
        case kPassLastNoB2:
            hipLaunchKernelGGL((k_pass<R, CH, kPassLastNoB2, NT, VS, NE>), grid, block, 0, st, p);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, bool CH, bool NT, int VS>
hipError_t launch_pass_ne(int kind, int ne, const PassParams &p, hipStream_t st) {
    switch (ne) {
        case 1:
            return launch_pass_t<R, CH, NT, VS, 1>(kind, p, st);
        case 2:
            return launch_pass_t<R, CH, NT, VS, 2>(kind, p, st);
        default:
            return hipErrorInvalidValue;
    }
}

template <typename R, int VS>
hipError_t launch_pass_r(int kind, bool cplx, bool nt, int ne, const PassParams &p, hipStream_t st) {
    if (cplx)
        return nt ? launch_pass_ne<R, true, true, VS>(kind, ne, p, st) : launch_pass_ne<R, true, false, VS>(kind, ne, p, st);
    return nt ? launch_pass_ne<R, false, true, VS>(kind, ne, p, st) : launch_pass_ne<R, false, false, VS>(kind, ne, p, st);
}

template <typename R, bool CH, bool NT, int VS, int KG>
hipError_t launch_staged_t(int kind, const PassParams &p, hipStream_t st) {
    constexpr int LOG2VS = VS == 4 ? 2 : (VS == 2 ? 1 : 0);
    const int n_blk = 1 << (p.log2s - LOG2VS - p.log2ub);
    const dim3 grid(n_blk > 1 ? (unsigned)(((p.n_tiles + 7) / 8) * 8 * n_blk) : (unsigned)p.n_tiles), block(kWG);
    const size_t lds = (size_t)p.stage_units * sizeof(VecT<R, VS>);
    switch (kind) {
        case kPassFirst:
            hipLaunchKernelGGL((k_pass_staged<R, CH, kPassFirst, NT, VS, KG>), grid, block, lds, st, p);
            break;
        case kPassNoB2:
            hipLaunchKernelGGL((k_pass_staged<R, CH, kPassNoB2, NT, VS, KG>), grid, block, lds, st, p);
            break;
        case kPassMid:
            hipLaunchKernelGGL((k_pass_staged<R, CH, kPassMid, NT, VS, KG>), grid, block, lds, st, p);
            break;
        case kPassLast:
            hipLaunchKernelGGL((k_pass_staged<R, CH, kPassLast, NT, VS, KG>), grid, block, lds, st, p);
            break;
        case kPassLastNoB2:
            hipLaunchKernelGGL((k_pass_staged<R, CH, kPassLastNoB2, NT, VS, KG>), grid, block, lds, st, p);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, int VS, int KG>
hipError_t launch_staged_k(int kind, bool cplx, bool nt, const PassParams &p, hipStream_t st) {
    if (cplx)
        return nt ? launch_staged_t<R, true, true, VS, KG>(kind, p, st)
                  : launch_staged_t<R, true, false, VS, KG>(kind, p, st);
    return nt ? launch_staged_t<R, false, true, VS, KG>(kind, p, st) : launch_staged_t<R, false, false, VS, KG>(kind, p, st);
}

template <typename R, int VS>
hipError_t launch_staged_r(int kind, bool cplx, bool nt, bool wide, const PassParams &p, hipStream_t st) {
    return wide ? launch_staged_k<R, VS, 12>(kind, cplx, nt, p, st) : launch_staged_k<R, VS, 4>(kind, cplx, nt, p, st);
}

}  // namespace

hipError_t launch_pass(int kind, bool fp32, bool cplx, bool nontemporal, int ne, int vs, const PassParams &p,
                       hipStream_t st) {
    if (p.n_tiles <= 0) return hipSuccess;
    if (fp32) {
        if (vs == 4) return launch_pass_r<float, 4>(kind, cplx, nontemporal, ne, p, st);
        if (vs == 2) return launch_pass_r<float, 2>(kind, cplx, nontemporal, ne, p, st);
        return launch_pass_r<float, 1>(kind, cplx, nontemporal, ne, p, st);
    }
    if (vs == 4) return launch_pass_r<double, 4>(kind, cplx, nontemporal, ne, p, st);
    if (vs == 2) return launch_pass_r<double, 2>(kind, cplx, nontemporal, ne, p, st);
    return launch_pass_r<double, 1>(kind, cplx, nontemporal, ne, p, st);
}

hipError_t launch_pass_staged(int kind, bool fp32, bool cplx, bool nontemporal, int vs, bool wide,
                              const PassParams &p, hipStream_t st) {
    if (p.n_tiles <= 0) return hipSuccess;
    if (fp32) {
        if (vs == 4) return launch_staged_r<float, 4>(kind, cplx, nontemporal, wide, p, st);
        if (vs == 2) return launch_staged_r<float, 2>(kind, cplx, nontemporal, wide, p, st);
        return launch_staged_r<float, 1>(kind, cplx, nontemporal, wide, p, st);
    }
    if (vs == 4) return launch_staged_r<double, 4>(kind, cplx, nontemporal, wide, p, st);
    if (vs == 2) return launch_staged_r<double, 2>(kind, cplx, nontemporal, wide, p, st);
    return launch_staged_r<double, 1>(kind, cplx, nontemporal, wide, p, st);
}

hipError_t launch_init(bool fp32, const InitParams &p, hipStream_t st) {
    if (p.n_tiles <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_init<float>, dim3(p.n_tiles), dim3(kWG), 0, st, p);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(p.n_tiles), dim3(kWG), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_reduce(int n_inst, int s_pad, const ReduceParams &p, hipStream_t st) {
    (void)s_pad;
    hipLaunchKernelGGL(k_reduce, dim3(n_inst * p.s_user), dim3(kWG), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_dos(const double *corr, int32_t n_steps, int32_t n_states, double dt, int window,
                      double *energies, double *dos, hipStream_t st) {
    const int64_t n_e = 2 * (int64_t)n_steps;
    hipLaunchKernelGGL(k_dos, dim3((unsigned)((n_e + kWG - 1) / kWG)), dim3(kWG), 0, st, corr, n_steps, n_states,
                       dt, window, energies, dos);
    return hipGetLastError();
}

hipError_t launch_dos_backward(const double *gdos, int32_t n_steps, int32_t n_states, double dt,
                               int window, double *gcorr, hipStream_t st) {
    hipLaunchKernelGGL(k_dos_backward, dim3((unsigned)((n_steps + kWG - 1) / kWG)), dim3(kWG), 0, st, gdos,
                       n_steps, n_states, dt, window, gcorr);
    return hipGetLastError();
}

hipError_t launch_convert_values(const DevMatrix &m, const double *csr_val, const double *csr_onsite,
                                 int64_t n_rows, hipStream_t st) {
    const int64_t work = m.ell_size > n_rows ? m.ell_size : n_rows;
    int64_t blocks = (work + kWG - 1) / kWG;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (m.is_complex)
        hipLaunchKernelGGL(k_convert_values<true>, dim3((unsigned)blocks), dim3(kWG), 0, st, m.ell_csr, m.ell_size,
                           csr_val, csr_onsite, n_rows, m.perm, m.val64, m.val32, m.onsite64, m.onsite32);
    else
        hipLaunchKernelGGL(k_convert_values<false>, dim3((unsigned)blocks), dim3(kWG), 0, st, m.ell_csr, m.ell_size,
                           csr_val, csr_onsite, n_rows, m.perm, m.val64, m.val32, m.onsite64, m.onsite32);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st) {
    const int64_t n = (int64_t)(bytes / 16);
    int64_t blocks = (n + kWG - 1) / kWG;
    if (blocks > 1 << 20) blocks = 1 << 20;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kWG), 0, st, (const d2 *)src, (d2 *)dst, n);
    return hipGetLastError();
}

}  // namespace tbpm
