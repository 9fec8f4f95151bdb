// Quasi-eigenstates (paper, Sec. "Quasieigenstates", Eq. (quasi)):
//     Psi(E_j) = sum_k w_|k| e^{i E_j k dt} psi(k dt),  k = -(N_t-1) .. N_t-1,
// accumulated while the states are propagated (forward, then with -dt), and
// normalised per energy and state at the end.
//
// k_qe_accum runs once per time step inside the step graph: it reads the
// current state psi(k dt) (the engine's state buffer, [rows][S] at the
// recursion precision) once and updates n_E FP64 accumulators
// acc[j][rows][S] += coef[k][j] psi, where k is the device step counter and
// coef[k][j] = w_|k| e^{i E_j t_k} is a host-built table.  It is a streaming
// kernel: 8 or 16 bytes read and 32 bytes read and written per energy and
// element.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "tbpm_internal.h"

namespace tbpm {
namespace {

template <typename R>
__global__ __launch_bounds__(kWG) void k_qe_accum(const void *__restrict__ state, d2 *__restrict__ acc, int64_t n_el,
                                                  const d2 *__restrict__ coef, int n_e,
                                                  const int32_t *__restrict__ counter) {
    using C = typename CxT<R>::T;
    const C *psi = (const C *)state;
    const int k = *(volatile const int32_t *)counter;
    const d2 *row = coef + (int64_t)k * n_e;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < n_el; e += stride) {
        const C x = psi[e];
        const double xr = (double)x.x, xi = (double)x.y;
        for (int j = 0; j < n_e; ++j) {
            const d2 c = row[j];
            d2 a = acc[(int64_t)j * n_el + e];
            a.x = fma(c.x, xr, fma(-c.y, xi, a.x));
            a.y = fma(c.x, xi, fma(c.y, xr, a.y));
            acc[(int64_t)j * n_el + e] = a;
        }
    }
}

// Per-block partial sums of |acc|^2 per state: block (b, j) covers rows
// [b * rows_per_block, ...) of energy j; out[j][s][3][n_blk] as written by
// block_state_partials (component 2 holds the squared norm).
__global__ __launch_bounds__(kWG) void k_qe_partials(const d2 *__restrict__ acc, int64_t n_rows, int log2s,
                                                     int64_t rows_per_block, int n_blk, double *__restrict__ out) {
    const int j = blockIdx.y;
    const int S = 1 << log2s;
    const int64_t n_el = n_rows << log2s;
    const int64_t e0 = (int64_t)blockIdx.x * rows_per_block << log2s;
    const int64_t e1 = min(n_el, e0 + (rows_per_block << log2s));
    const d2 *a = acc + (int64_t)j * n_el;
    double nrm = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kWG) nrm = fma(a[e].x, a[e].x, fma(a[e].y, a[e].y, nrm));
    block_state_partials(0.0, 0.0, nrm, log2s, out + (int64_t)j * S * 3 * n_blk, blockIdx.x, n_blk);
}

// norm2[j][s] = sum over blocks of the partials, in a fixed order; one
// workgroup per (energy, state)
__global__ __launch_bounds__(kWG) void k_qe_norms(const double *__restrict__ part, int log2s, int n_blk, int s_user,
                                                  double *__restrict__ norm2) {
    __shared__ double red[kWG];
    const int j = blockIdx.x / s_user, s = blockIdx.x % s_user;
    const int S = 1 << log2s;
    const double *p = part + ((int64_t)j * S + s) * 3 * n_blk + 2 * (int64_t)n_blk;
    double v = 0.0;
    for (int b = threadIdx.x; b < n_blk; b += kWG) v += p[b];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) norm2[(int64_t)j * s_user + s] = red[0];
}

// out[j][perm[r]][s] = acc[j][r][s] / sqrt(norm2[j][s]) for s < s_user
__global__ __launch_bounds__(kWG) void k_qe_scatter(const d2 *__restrict__ acc, const double *__restrict__ norm2,
                                                    int64_t n_rows, int log2s, int s_user, int n_e,
                                                    const int32_t *__restrict__ perm, d2 *__restrict__ out) {
    const int64_t n_el = n_rows << log2s;
    const int64_t total = (int64_t)n_e * n_rows * s_user;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < total; i += stride) {
        const int s = (int)(i % s_user);
        const int64_t r = (i / s_user) % n_rows;
        const int j = (int)(i / ((int64_t)s_user * n_rows));
        const double n2 = norm2[(int64_t)j * s_user + s];
        const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
        const d2 a = acc[(int64_t)j * n_el + (r << log2s) + s];
        d2 o;
        o.x = a.x * inv;
        o.y = a.y * inv;
        const int64_t ro = perm ? (int64_t)perm[r] : r;
        out[((int64_t)j * n_rows + ro) * s_user + s] = o;
    }
}

int64_t grid_of(int64_t n) {
    int64_t b = (n + kWG - 1) / kWG;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : b;
}

}  // namespace

hipError_t launch_qe_accum(bool fp32, const void *state, double *acc, int64_t n_el, const double *coef, int32_t n_e,
                           const int32_t *counter, hipStream_t st) {
    const dim3 grid((unsigned)grid_of(n_el)), block(kWG);
    if (fp32)
        hipLaunchKernelGGL(k_qe_accum<float>, grid, block, 0, st, state, (d2 *)acc, n_el, (const d2 *)coef, n_e,
                           counter);
    else
        hipLaunchKernelGGL(k_qe_accum<double>, grid, block, 0, st, state, (d2 *)acc, n_el, (const d2 *)coef, n_e,
                           counter);
    return hipGetLastError();
}

int32_t qe_partial_blocks(int64_t n_rows) { return (int32_t)std::min<int64_t>(4096, std::max<int64_t>(1, n_rows / 256)); }

hipError_t launch_qe_finalize(const double *acc, int64_t n_rows, int32_t log2s, int32_t s_user, int32_t n_e,
                              const int32_t *perm, double *partials, double *norm2, double *out, hipStream_t st) {
    const int32_t n_blk = qe_partial_blocks(n_rows);
    const int64_t rpb = (n_rows + n_blk - 1) / n_blk;
    hipLaunchKernelGGL(k_qe_partials, dim3((unsigned)n_blk, (unsigned)n_e), dim3(kWG), 0, st, (const d2 *)acc, n_rows,
                       log2s, rpb, n_blk, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qe_norms, dim3((unsigned)(n_e * s_user)), dim3(kWG), 0, st, (const double *)partials, log2s,
                       n_blk, s_user, norm2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qe_scatter, dim3((unsigned)grid_of((int64_t)n_e * n_rows * s_user)), dim3(kWG), 0, st,
                       (const d2 *)acc, (const double *)norm2, n_rows, log2s, s_user, n_e, perm, (d2 *)out);
    return hipGetLastError();
}

}  // namespace tbpm
