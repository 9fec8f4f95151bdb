// Haydock recursion (paper, Sec. "Local density of states", the recursion
// method): one Lanczos chain per state of a block [rows][S] (S a power of
// two, S <= 64), all chains advanced together so that the matrix is read once
// per iteration for all of them.
//
// The normalised Lanczos vector l_i is never stored: the buffers hold
// u_i = b_i l_i (the unnormalised m_i of the recursion, or psi0 for i = 0),
// and a per-state scalar table hs[s] = {1/b_i, b_i/b_{i-1}, a_i/b_i, -}
// carries the normalisation (1/b_0 = 1/||psi0||).  One iteration is
//   k_hay_spmv : y = (H u_i)/b_i - (b_i/b_{i-1}) u_{i-1}   (= H l_i - b_i l_{i-1}),
//                partials of Re <u_i|y>/b_i                 (-> a_i)
//   k_hay_reduce(kA): a_i, hs[s].2 = a_i/b_i
//   k_hay_axpy : u_{i+1} = y - (a_i/b_i) u_i, over u_{i-1}, partials of ||u_{i+1}||^2
//   k_hay_reduce(kB): b_{i+1}, or 0 below the breakdown threshold (the chain
//                stays zero from then on: 1/b = 0 zeroes every later vector)
// so a_i = <l_i|H l_i - b_i l_{i-1}>, which equals <l_i|H|l_i> since l_i is
// orthogonal to l_{i-1} (the form that keeps better orthogonality in
// finite precision).  All reductions are FP64 per-tile partials summed in a
// fixed order, so results are reproducible for a given tiling.
//
// Streams per iteration: gather of u_i, u_{i-1}, y written (spmv); y, u_i
// read and u_{i+1} written (axpy): 6 state vectors plus the matrix.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_util.h"
#include "tbpm_internal.h"

namespace tbpm {
namespace {

enum HayReduce : int { kHayA = 0, kHayB = 1, kHayInit = 2 };

// One thread per (row, state) element: on the headline lattice with 8 chains
// this runs ahead of units of 2 states (+3-7% per iteration) and of 4
// (+30%).  When every slice has the same width (uniform_w > 0) a row's slots
// come without the slice-offset loads.
template <bool CH>
__global__ __launch_bounds__(kWG) void k_hay_spmv(const TileDesc *__restrict__ tiles, int n_tiles, int xcd_remap,
                                                  int log2s, const int32_t *__restrict__ col,
                                                  const void *__restrict__ val, const uint32_t *__restrict__ soff,
                                                  int uniform_w, const double *__restrict__ onsite,
                                                  const d2 *__restrict__ u,
                                                  const d2 *__restrict__ uprev, d2 *__restrict__ y,
                                                  const double *__restrict__ hs, int32_t *counter,
                                                  double *__restrict__ partials) {
    using HV = typename std::conditional<CH, d2, double>::type;
    const HV *hvp = (const HV *)val;
    auto hv_ = [&](uint32_t slot) { return hvp[slot]; };
    const int tile = tile_of_block(blockIdx.x, n_tiles, xcd_remap);
    const TileDesc td = tiles[tile];
    if (counter && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(counter, 1);
    const uint32_t smask = (1u << log2s) - 1u;
    const uint32_t s = threadIdx.x & smask;
    const double inv = hs[4 * s], cprev = hs[4 * s + 1];
    // 32-bit element indices: rows * S < 2^31 (checked by the entry point)
    const uint32_t n_u = (uint32_t)td.rows << log2s;
    const uint32_t row0 = (uint32_t)td.row0;
    constexpr int KG = 4;  // stored elements gathered per batch
    double dre = 0.0;
    for (uint32_t q = threadIdx.x; q < n_u; q += kWG) {
        const uint32_t r = row0 + (q >> log2s);
        const uint32_t sl = r / kSliceRows;
        uint32_t base;
        int w;
        if (uniform_w > 0) {
            w = uniform_w;
            base = sl * (uint32_t)(uniform_w * kSliceRows) + r % kSliceRows;
        } else {
            const uint32_t off = soff[sl];
            w = (int)((soff[sl + 1] - off) / kSliceRows);
            base = off + r % kSliceRows;
        }
        const uint32_t e = (r << log2s) + s;
        const d2 up = __builtin_nontemporal_load(uprev + e);  // read once
        const d2 ur = u[e];
        d2 acc;
        acc.x = onsite[r] * ur.x;
        acc.y = onsite[r] * ur.y;
        for (int k = 0; k < w; k += KG) {
            HV h[KG];
            uint32_t g[KG];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                const bool valid = k + i < w;
                const uint32_t slot = valid ? base + (uint32_t)(k + i) * kSliceRows : base;
                const HV hv = hv_(slot);
                g[i] = ((valid ? (uint32_t)col[slot] : r) << log2s) + s;
                h[i] = valid ? hv : HV{};
            }
#pragma unroll
            for (int i = 0; i < KG; ++i) acc = hmad(h[i], u[g[i]], acc);
        }
        d2 yv;
        yv.x = fma(inv, acc.x, -cprev * up.x);
        yv.y = fma(inv, acc.y, -cprev * up.y);
        __builtin_nontemporal_store(yv, y + e);
        dre = fma(ur.x * inv, yv.x, fma(ur.y * inv, yv.y, dre));
    }
    block_state_partials(dre, 0.0, 0.0, log2s, partials, tile, n_tiles);
}

// unext = y - (a_i/b_i) u  (unext may be the buffer of u_{i-1}), with the
// partials of ||unext||^2; with unext null it only measures ||y||^2.  The
// iteration walks it last tile to first (reverse), so it starts on the tiles
// whose y the product pass wrote last, and the next product pass starts on
// the tiles whose u_{i+1} it wrote last.
__global__ __launch_bounds__(kWG) void k_hay_axpy(const TileDesc *__restrict__ tiles, int n_tiles, int xcd_remap,
                                                  int reverse, int log2s, const d2 *y, const d2 *u, d2 *unext,
                                                  const double *__restrict__ hs, double *__restrict__ partials) {
    const int tile = tile_of_block(blockIdx.x, n_tiles, xcd_remap, reverse);
    const TileDesc td = tiles[tile];
    const uint32_t smask = (1u << log2s) - 1u;
    const uint32_t s = threadIdx.x & smask;
    const double c = unext ? hs[4 * s + 2] : 0.0;
    const uint32_t n_u = (uint32_t)td.rows << log2s;
    const uint32_t u0 = (uint32_t)td.row0 << log2s;
    double nrm = 0.0;
    for (uint32_t q = threadIdx.x; q < n_u; q += kWG) {
        const uint32_t e = u0 + q;
        d2 v = __builtin_nontemporal_load(y + e);  // read once
        if (unext) {
            const d2 ui = u[e];
            v.x = fma(-c, ui.x, v.x);
            v.y = fma(-c, ui.y, v.y);
            unext[e] = v;
        }
        nrm = fma(v.x, v.x, fma(v.y, v.y, nrm));
    }
    block_state_partials(0.0, 0.0, nrm, log2s, partials, tile, n_tiles);
}

// One workgroup per state: the fixed-order sum of the per-tile partials and
// the scalar update.  The iteration index is the device counter minus one
// (k_hay_spmv bumps it).
// First stage of a per-state sum over many per-tile partials: workgroup
// (g, s) adds values [g kFold, (g+1) kFold) of state s (row s of `in`, stride
// in_stride) in a fixed order and writes out[s n_fold + g].  One pass with
// all loads in flight, instead of one workgroup per state walking the whole
// row with dependent rounds of loads.
constexpr int kFold = 4 * kWG;

__global__ __launch_bounds__(kWG) void k_hay_fold(const double *__restrict__ in, int64_t in_stride, int n,
                                                  double *__restrict__ out, int n_fold) {
    __shared__ double red[kWG];
    const int g = blockIdx.x, s = blockIdx.y;
    const double *p = in + (int64_t)s * in_stride + (int64_t)g * kFold;
    const int m = min(kFold, n - g * kFold);
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = (int)threadIdx.x + q * kWG;
        v[q] = i < m ? p[i] : 0.0;
    }
    red[threadIdx.x] = (v[0] + v[1]) + (v[2] + v[3]);
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)s * n_fold + g] = red[0];
}

// Final stage: workgroup s sums row s of `in` (n values, stride in_stride)
// and applies the Lanczos scalar update of `mode`.
__global__ __launch_bounds__(kWG) void k_hay_reduce(const double *__restrict__ in, int64_t in_stride, int n,
                                                    int s_user, int mode, double thr, double *__restrict__ hs,
                                                    int32_t *counter, int n_iter, double *__restrict__ a_out,
                                                    double *__restrict__ b_out) {
    __shared__ double red[kWG];
    const int s = blockIdx.x;
    const double *p = in + (int64_t)s * in_stride;
    // eight independent accumulators keep loads in flight; the order is fixed
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int t = threadIdx.x;
    for (; t + 7 * kWG < n; t += 8 * kWG) {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] += p[t + q * kWG];
    }
    for (; t < n; t += kWG) v[0] += p[t];
    red[threadIdx.x] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double sum = red[0];
    double *h = hs + 4 * s;
    if (mode == kHayInit) {
        const double nrm = sqrt(sum);
        h[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        h[1] = 0.0;
        h[2] = 0.0;
        h[3] = 0.0;
        if (s == 0) *counter = 0;
        return;
    }
    const int k = *(volatile const int32_t *)counter - 1;
    if (mode == kHayA) {
        h[2] = sum * h[0];
        if (k >= 0 && k < n_iter && s < s_user) a_out[(int64_t)k * s_user + s] = sum;
        return;
    }
    double b = sqrt(sum);
    double inv = 0.0;
    if (b > thr && h[0] != 0.0)
        inv = 1.0 / b;
    else
        b = 0.0;
    if (k >= 0 && k < n_iter && s < s_user) b_out[(int64_t)k * s_user + s] = b;
    h[1] = b * h[0];
    h[0] = inv;
}

// d(E_j) = -(1/pi) Im G_0(E_j + i eps), G_0 by the continued fraction from
// the deepest level up; one thread per (energy, state)
__global__ __launch_bounds__(kWG) void k_hay_ldos(const double *__restrict__ a, const double *__restrict__ b,
                                                  int n_iter, int n_states, const double *__restrict__ energies,
                                                  int64_t n_e, double eps, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= n_e * n_states) return;
    const int s = (int)(i % n_states);
    const int64_t j = i / n_states;
    const double zr = energies[j];
    double tr = zr - a[(int64_t)(n_iter - 1) * n_states + s], ti = eps;
    for (int q = n_iter - 2; q >= 0; --q) {
        const double bq = b[(int64_t)q * n_states + s];
        const double d = tr * tr + ti * ti;
        const double f = bq * bq / d;  // b^2 / t = f conj(t)
        tr = zr - a[(int64_t)q * n_states + s] - f * tr;
        ti = eps + f * ti;
    }
    out[i] = ti / (tr * tr + ti * ti) / M_PI;  // -Im(1/t)/pi
}

}  // namespace

hipError_t launch_hay_spmv(bool cplx, const TileDesc *tiles, int32_t n_tiles, int32_t xcd_remap, int32_t log2s,
                           const int32_t *col, const void *val, const uint32_t *slice_off, int32_t uniform_w,
                           const double *onsite, const double *u, const double *uprev, double *y, const double *hs,
                           int32_t *counter, double *partials, hipStream_t st) {
    if (cplx)
        hipLaunchKernelGGL(k_hay_spmv<true>, dim3((unsigned)n_tiles), dim3(kWG), 0, st, tiles, n_tiles, xcd_remap,
                           log2s, col, val, slice_off, uniform_w, onsite, (const d2 *)u, (const d2 *)uprev, (d2 *)y,
                           hs, counter, partials);
    else
        hipLaunchKernelGGL(k_hay_spmv<false>, dim3((unsigned)n_tiles), dim3(kWG), 0, st, tiles, n_tiles, xcd_remap,
                           log2s, col, val, slice_off, uniform_w, onsite, (const d2 *)u, (const d2 *)uprev, (d2 *)y,
                           hs, counter, partials);
    return hipGetLastError();
}

hipError_t launch_hay_axpy(const TileDesc *tiles, int32_t n_tiles, int32_t xcd_remap, int32_t reverse, int32_t log2s,
                           const double *y, const double *u, double *unext, const double *hs, double *partials,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_hay_axpy, dim3((unsigned)n_tiles), dim3(kWG), 0, st, tiles, n_tiles, xcd_remap, reverse, log2s,
                       (const d2 *)y, (const d2 *)u, (d2 *)unext, hs, partials);
    return hipGetLastError();
}

int32_t hay_fold_count(int32_t n_tiles) { return n_tiles > kFold ? (n_tiles + kFold - 1) / kFold : 0; }

hipError_t launch_hay_reduce(const double *partials, int32_t n_tiles, int32_t s_pad, int32_t s_user, int32_t mode,
                             double thr, double *hs, int32_t *counter, int32_t n_iter, double *a_out, double *b_out,
                             double *fold, hipStream_t st) {
    const double *in = partials + (mode == kHayA ? 0 : 2 * (int64_t)n_tiles);
    int64_t stride = 3 * (int64_t)n_tiles;
    int n = n_tiles;
    const int32_t n_fold = hay_fold_count(n_tiles);
    if (n_fold > 0) {
        hipLaunchKernelGGL(k_hay_fold, dim3((unsigned)n_fold, (unsigned)s_pad), dim3(kWG), 0, st, in, stride, n_tiles,
                           fold, n_fold);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        in = fold;
        stride = n_fold;
        n = n_fold;
    }
    hipLaunchKernelGGL(k_hay_reduce, dim3((unsigned)s_pad), dim3(kWG), 0, st, in, stride, n, s_user, (int)mode, thr,
                       hs, counter, n_iter, a_out, b_out);
    return hipGetLastError();
}

hipError_t launch_hay_ldos(const double *a, const double *b, int32_t n_iter, int32_t n_states, const double *energies,
                           int64_t n_e, double eps, double *out, hipStream_t st) {
    const int64_t total = n_e * n_states;
    hipLaunchKernelGGL(k_hay_ldos, dim3((unsigned)((total + kWG - 1) / kWG)), dim3(kWG), 0, st, a, b, n_iter,
                       n_states, energies, n_e, eps, out);
    return hipGetLastError();
}

}  // namespace tbpm
