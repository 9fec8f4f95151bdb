// Kubo-Bastin conductivity by the kernel polynomial method (paper, Sec.
// "Tight-binding propagation method", the DC conductivity tensor): the
// device side of the energy integral and the split-K reduction of the
// moment products.
//
//  * k_kpm_sum_parts: mu[:, block] = sum_p parts[p] in a fixed order (the
//    per-chunk results of the moment product L^H R).
//  * k_kb_energy: one workgroup per energy E~_k = cos(theta_k) of the
//    midpoint grid in theta: with w_m = g_m / (1 + delta_m0) (Jackson g),
//    c_n = cos(n theta), p_n = (E~ - i n s) e^{i n theta},
//    q_m = (E~ + i m s) e^{-i m theta}, s = sin(theta),
//      F_k = sum_{m,n} Gamma_nm mu~_nm = sum_m w_m [c_m (A p)_m + q_m (A c)_m],
//      (A x)_m = sum_n mu_mn w_n x_n,
//    stored as the integrand weight F_k sin(theta_k) dtheta / (1 - E~_k^2)^2
//    (real part) with the energy E_k = rescale E~_k.
//  * k_kb_sigma: sigma(mu_j) = 4/(pi A rescale^2) sum_k f(E_k; mu_j) weight_k.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "tbpm_internal.h"

namespace tbpm {
namespace {

constexpr int kMaxMomentsLds = 4096;

__global__ __launch_bounds__(kWG) void k_kpm_sum_parts(const d2 *__restrict__ parts, int64_t n_el, int n_parts,
                                                       int64_t part_stride, d2 *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n_el; i += stride) {
        d2 a;
        a.x = 0.0;
        a.y = 0.0;
        for (int p = 0; p < n_parts; ++p) {
            const d2 v = parts[(int64_t)p * part_stride + i];
            a.x += v.x;
            a.y += v.y;
        }
        out[i] = a;
    }
}

__device__ __forceinline__ double jackson_w(int m, int n_mom) {
    const double q = M_PI / (n_mom + 1);
    const double g = ((n_mom - m + 1) * cos(q * m) + sin(q * m) / tan(q)) / (n_mom + 1);
    return m == 0 ? 0.5 * g : g;
}

// mu: [M][M] with mu_mn at m + n*M (column n contiguous over m)
__global__ __launch_bounds__(kWG) void k_kb_energy(const d2 *__restrict__ mu, int n_mom, double th_lo, double dth,
                                                   double rescale, double *__restrict__ energies,
                                                   double *__restrict__ weight) {
    __shared__ double w_s[kMaxMomentsLds];
    __shared__ d2 p_s[kMaxMomentsLds];
    __shared__ double c_s[kMaxMomentsLds];
    __shared__ double red[kWG];
    const int k = blockIdx.x;
    const double th = th_lo + (k + 0.5) * dth;
    double sn, x;
    sincos(th, &sn, &x);
    for (int n = threadIdx.x; n < n_mom; n += kWG) {
        const double w = jackson_w(n, n_mom);
        double sa, ca;
        sincos(n * th, &sa, &ca);
        w_s[n] = w;
        c_s[n] = w * ca;  // w_n cos(n theta)
        // w_n (x - i n s)(cos + i sin)
        d2 pv;
        pv.x = w * (x * ca + n * sn * sa);
        pv.y = w * (x * sa - n * sn * ca);
        p_s[n] = pv;
    }
    __syncthreads();
    double acc = 0.0;  // real part of F
    for (int m = threadIdx.x; m < n_mom; m += kWG) {
        double apx = 0.0, apy = 0.0, acx = 0.0, acy = 0.0;
        for (int n = 0; n < n_mom; ++n) {
            const d2 a = mu[m + (int64_t)n * n_mom];
            const d2 pv = p_s[n];
            const double cv = c_s[n];
            apx = fma(a.x, pv.x, fma(-a.y, pv.y, apx));
            apy = fma(a.x, pv.y, fma(a.y, pv.x, apy));
            acx = fma(a.x, cv, acx);
            acy = fma(a.y, cv, acy);
        }
        const double wm = w_s[m];
        double sa, ca;
        sincos(m * th, &sa, &ca);
        // c_m (A p)_m, real part
        double re = ca * apx;
        // q_m (A c)_m with q_m = (x + i m s)(cos - i sin)
        const double qx = x * ca + m * sn * sa, qy = m * sn * ca - x * sa;
        re += qx * acx - qy * acy;
        acc = fma(wm, re, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double d = (1.0 - x) * (1.0 + x);
        energies[k] = rescale * x;
        weight[k] = red[0] * sn * dth / (d * d);
    }
}

__global__ __launch_bounds__(kWG) void k_kb_sigma(const double *__restrict__ energies,
                                                  const double *__restrict__ weight, int n_energy,
                                                  const double *__restrict__ mus, int n_mu, double beta,
                                                  double scale, double *__restrict__ sigma) {
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= n_mu) return;
    const double mu = mus[j];
    double s = 0.0;
    for (int k = 0; k < n_energy; ++k) {
        const double fd = 0.5 * (1.0 - tanh(0.5 * beta * (energies[k] - mu)));
        s = fma(fd, weight[k], s);
    }
    sigma[j] = scale * s;
}

}  // namespace

int32_t kpm_max_moments_lds() { return kMaxMomentsLds; }

hipError_t launch_kpm_sum_parts(const double *parts, int64_t n_el, int32_t n_parts, int64_t part_stride, double *out,
                                hipStream_t st) {
    int64_t b = (n_el + kWG - 1) / kWG;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_kpm_sum_parts, dim3((unsigned)b), dim3(kWG), 0, st, (const d2 *)parts, n_el, n_parts,
                       part_stride, (d2 *)out);
    return hipGetLastError();
}

hipError_t launch_kubo_bastin(const double *mu, int32_t n_mom, double rescale, double th_lo, double dth,
                              int32_t n_energy, const double *mus, int32_t n_mu, double beta, double scale,
                              double *energies, double *weight, double *sigma, hipStream_t st) {
    hipLaunchKernelGGL(k_kb_energy, dim3((unsigned)n_energy), dim3(kWG), 0, st, (const d2 *)mu, n_mom, th_lo, dth,
                       rescale, energies, weight);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kb_sigma, dim3((unsigned)((n_mu + kWG - 1) / kWG)), dim3(kWG), 0, st, energies, weight,
                       n_energy, mus, n_mu, beta, scale, sigma);
    return hipGetLastError();
}

}  // namespace tbpm
