// Optical conductivity by propagation (paper, Sec. "Optical conductivity"):
// kernels around the Clenshaw passes.
//
//  * k_gather_values: the current operator J (values on H's CSR pattern) in
//    the sliced-ELL layout of H, through the slot -> CSR-position map.
//  * k_join: J psi0 and psi0 (internal row order, [rows][S padded]) side by
//    side in one block [rows][2S padded], so that one Chebyshev series of the
//    Fermi-Dirac operator serves both: f(H) [J psi0 | psi0].
//  * k_pack: from that block B and F = f(H) B, psi1 = (1 - f(H)) J psi0 =
//    B - F in columns 0..S-1 and psi2 = f(H) psi0 in S..2S-1 of one block
//    [n][2S] in the caller's row order, so that one propagation carries both.
//  * k_jcorr: per step, <psi2_s| J |psi1_s> for s < S from the propagated
//    block: J applied to the psi1 columns of each row (gathered over the
//    row's stored elements) and contracted with the row's psi2 columns; FP64
//    per-tile partials in the layout of the correlation, for k_reduce.
//  * k_ac_cond: the windowed sine transform of the Kubo formula, Eq. (AC).
//  * k_ac_kk: the imaginary part from the real part by the Kramers-Kronig
//    relation (the principal-value integral of the piecewise-linear,
//    even extension of Re sigma, as closed-form weights per grid point).
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "tbpm_internal.h"

namespace tbpm {
namespace {

__global__ __launch_bounds__(kWG) void k_gather_values(const int64_t *__restrict__ ell_csr, int64_t ell_size,
                                                       const d2 *__restrict__ csr_val, d2 *__restrict__ ell_val) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t q = (int64_t)blockIdx.x * kWG + threadIdx.x; q < ell_size; q += stride) {
        const int64_t pos = ell_csr[q];
        d2 v;
        v.x = 0.0;
        v.y = 0.0;
        if (pos >= 0) v = csr_val[pos];
        ell_val[q] = v;
    }
}

__global__ __launch_bounds__(kWG) void k_join(const d2 *__restrict__ jpsi, const d2 *__restrict__ psi,
                                              int64_t n_rows, int log2s, int log2s2, int S, d2 *__restrict__ out) {
    const int64_t total = n_rows << log2s2;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    const int m2 = (1 << log2s2) - 1;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < total; i += stride) {
        const int64_t r = i >> log2s2;
        const int c = (int)(i & m2);
        d2 v;
        v.x = 0.0;
        v.y = 0.0;
        if (c < S)
            v = jpsi[(r << log2s) + c];
        else if (c < 2 * S)
            v = psi[(r << log2s) + c - S];
        out[i] = v;
    }
}

__global__ __launch_bounds__(kWG) void k_pack(const d2 *__restrict__ blk, const d2 *__restrict__ fblk,
                                              int64_t n_rows, int log2s2, int S, const int32_t *__restrict__ perm,
                                              d2 *__restrict__ out) {
    const int64_t total = n_rows * 2 * S;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < total; i += stride) {
        const int64_t r = i / (2 * S);
        const int c = (int)(i % (2 * S));
        const int64_t ro = perm ? (int64_t)perm[r] : r;
        const int64_t src = (r << log2s2) + c;
        d2 v = fblk[src];
        if (c < S) {
            const d2 b = blk[src];
            v.x = b.x - v.x;
            v.y = b.y - v.y;
        }
        out[ro * 2 * S + c] = v;
    }
}

// state: the propagated block, [rows][2^log2s2] at precision R; thread t
// handles state t & (SP-1) of its rows (SP = 2^log2sp >= S)
template <typename R>
__global__ __launch_bounds__(kWG) void k_jcorr(const TileDesc *__restrict__ tiles, int n_tiles, int log2sp, int S,
                                               int log2s2, const void *__restrict__ state,
                                               const uint32_t *__restrict__ soff, const int32_t *__restrict__ col,
                                               const d2 *__restrict__ jval, double *__restrict__ partials) {
    using C = typename CxT<R>::T;
    const C *psi = (const C *)state;
    const TileDesc td = tiles[blockIdx.x];
    const uint32_t spm = (1u << log2sp) - 1u;
    const int64_t n_u = (int64_t)td.rows << log2sp;
    double dre = 0.0, dim = 0.0;
    for (int64_t u = threadIdx.x; u < n_u; u += kWG) {
        const int s = (int)(u & spm);
        if (s >= S) continue;
        const int64_t r = td.row0 + (u >> log2sp);
        const int64_t sl = r / kSliceRows;
        const uint32_t off = soff[sl];
        const int w = (int)((soff[sl + 1] - off) / kSliceRows);
        const int64_t base = off + r % kSliceRows;
        double ar = 0.0, ai = 0.0;
        for (int k = 0; k < w; ++k) {
            const int64_t slot = base + (int64_t)k * kSliceRows;
            const d2 j = jval[slot];
            const C x = psi[((int64_t)col[slot] << log2s2) + s];
            const double xr = (double)x.x, xi = (double)x.y;
            ar = fma(j.x, xr, fma(-j.y, xi, ar));
            ai = fma(j.x, xi, fma(j.y, xr, ai));
        }
        const C y = psi[(r << log2s2) + S + s];
        const double yr = (double)y.x, yi = (double)y.y;
        dre = fma(yr, ar, fma(yi, ai, dre));  // conj(y) * (ar + i ai)
        dim = fma(yr, ai, fma(-yi, ar, dim));
    }
    block_state_partials(dre, dim, 0.0, log2sp, partials, blockIdx.x, n_tiles);
}

// sigma(w_j) = (e^{-beta w_j} - 1) / (w_j A) dt sum_k w_k sin(w_j t_k) 2 Im Cbar_k,
// w_j = j pi / (N_t dt), sigma(0) = 0; the phase w_j t_k = pi (j k mod 2N)/N
// is reduced exactly in integers, the sum is compensated.
__global__ __launch_bounds__(kWG) void k_ac_cond(const d2 *__restrict__ corr, int n_steps, int n_states, double dt,
                                                 double beta, double area, int window, double *__restrict__ omegas,
                                                 double *__restrict__ sigma) {
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= n_steps) return;
    const double w_j = M_PI * j / (n_steps * dt);
    omegas[j] = w_j;
    if (j == 0) {
        sigma[0] = 0.0;
        return;
    }
    const int64_t two_n = 2 * (int64_t)n_steps;
    double sum = 0.0, comp = 0.0;
    for (int k = 1; k < n_steps; ++k) {
        double im = 0.0;
        for (int s = 0; s < n_states; ++s) im += corr[(int64_t)k * n_states + s].y;
        im /= n_states;
        const double wk = window == TBPM_WIN_HANN ? 0.5 * (1.0 + cospi((double)k / n_steps)) : 1.0;
        const int64_t m = ((int64_t)j * k) % two_n;
        const double term = wk * sinpi((double)m / n_steps) * 2.0 * im;
        const double t = sum + term;  // Neumaier
        comp += fabs(sum) >= fabs(term) ? (sum - t) + term : (term - t) + sum;
        sum = t;
    }
    sigma[j] = (exp(-beta * w_j) - 1.0) / (w_j * area) * (sum + comp) * dt;
}

// P int phi(u) / (u - m) du for the unit hat phi(u) = max(0, 1 - |u|):
//   g(m) = (1 - m) ln|1 - m| - (1 + m) ln|1 + m| + 2 m ln|m|   (0 ln 0 = 0),
// odd in m; for |m| >= 2 in the form -|m| log1p(-1/m^2) - log1p(2/(|m| - 1)),
// which has no cancellation between terms of size |m| ln|m|.
__device__ __forceinline__ double kk_hat(int64_t m) {
    const double a = (double)(m < 0 ? -m : m);
    double g;
    if (a < 2.0) {
        const double t1 = a == 1.0 ? 0.0 : (1.0 - a) * log(fabs(1.0 - a));
        const double t3 = a == 0.0 ? 0.0 : 2.0 * a * log(a);
        g = t1 - (1.0 + a) * log(1.0 + a) + t3;
    } else {
        g = -a * log1p(-1.0 / (a * a)) - log1p(2.0 / (a - 1.0));
    }
    return m < 0 ? -g : g;
}

// Im sigma_k = -(1/pi) P int Re sigma(|w|)/(w - w_k) dw on the grid w_j = j dw
// with Re sigma = sum_j y_j phi(w/dw - j) (linear between grid points, zero
// one spacing past the last) and its mirror image for w < 0: node 0 gives
// y_0 g(k), node j >= 1 gives y_j (g(k - j) + g(k + j)).  One thread per k;
// the sum over j is compensated (Neumaier) and runs in a fixed order.
__global__ __launch_bounds__(kWG) void k_ac_kk(const double *__restrict__ re, int n, double *__restrict__ im) {
    const int k = blockIdx.x * kWG + threadIdx.x;
    if (k >= n) return;
    double sum = re[0] * kk_hat(k), comp = 0.0;
    for (int j = 1; j < n; ++j) {
        const double term = re[j] * (kk_hat((int64_t)k - j) + kk_hat((int64_t)k + j));
        const double t = sum + term;
        comp += fabs(sum) >= fabs(term) ? (sum - t) + term : (term - t) + sum;
        sum = t;
    }
    im[k] = -(sum + comp) / M_PI;
}

int64_t grid_for_n(int64_t n) {
    int64_t b = (n + kWG - 1) / kWG;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : b;
}

}  // namespace

hipError_t launch_gather_values(const int64_t *ell_csr, int64_t ell_size, const double *csr_val, double *ell_val,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_gather_values, dim3((unsigned)grid_for_n(ell_size)), dim3(kWG), 0, st, ell_csr, ell_size,
                       (const d2 *)csr_val, (d2 *)ell_val);
    return hipGetLastError();
}

hipError_t launch_join(const double *jpsi, const double *psi, int64_t n_rows, int32_t log2s, int32_t log2s2,
                       int32_t S, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_join, dim3((unsigned)grid_for_n(n_rows << log2s2)), dim3(kWG), 0, st, (const d2 *)jpsi,
                       (const d2 *)psi, n_rows, log2s, log2s2, S, (d2 *)out);
    return hipGetLastError();
}

hipError_t launch_pack(const double *blk, const double *fblk, int64_t n_rows, int32_t log2s2, int32_t S,
                       const int32_t *perm, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3((unsigned)grid_for_n(n_rows * 2 * S)), dim3(kWG), 0, st, (const d2 *)blk,
                       (const d2 *)fblk, n_rows, log2s2, S, perm, (d2 *)out);
    return hipGetLastError();
}

hipError_t launch_jcorr(bool fp32, const TileDesc *tiles, int32_t n_tiles, int32_t log2sp, int32_t S, int32_t log2s2,
                        const void *state, const uint32_t *slice_off, const int32_t *col, const double *jval,
                        double *partials, hipStream_t st) {
    if (fp32)
        hipLaunchKernelGGL(k_jcorr<float>, dim3((unsigned)n_tiles), dim3(kWG), 0, st, tiles, n_tiles, log2sp, S, log2s2,
                           state, slice_off, col, (const d2 *)jval, partials);
    else
        hipLaunchKernelGGL(k_jcorr<double>, dim3((unsigned)n_tiles), dim3(kWG), 0, st, tiles, n_tiles, log2sp, S,
                           log2s2, state, slice_off, col, (const d2 *)jval, partials);
    return hipGetLastError();
}

hipError_t launch_ac_kk(const double *re, int32_t n, double *im, hipStream_t st) {
    hipLaunchKernelGGL(k_ac_kk, dim3((unsigned)((n + kWG - 1) / kWG)), dim3(kWG), 0, st, re, n, im);
    return hipGetLastError();
}

hipError_t launch_ac_cond(const double *corr, int32_t n_steps, int32_t n_states, double dt, double beta, double area,
                          int window, double *omegas, double *sigma, hipStream_t st) {
    hipLaunchKernelGGL(k_ac_cond, dim3((unsigned)((n_steps + kWG - 1) / kWG)), dim3(kWG), 0, st, (const d2 *)corr,
                       n_steps, n_states, dt, beta, area, window, omegas, sigma);
    return hipGetLastError();
}

}  // namespace tbpm
