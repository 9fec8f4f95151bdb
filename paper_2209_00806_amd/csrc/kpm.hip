// Kubo-Bastin conductivity by the kernel polynomial method (paper, Sec.
// "Tight-binding propagation method", the DC conductivity tensor): the
// moment product on the FP64 matrix cores, its fixed-order chunk sum, and
// the device side of the energy integral.
//
//  * k_kpm_product: the moment product L^H R on the FP64 matrix cores,
//    split over chunks of the long inner dimension (rows x states).
//  * k_kpm_sum_parts: mu[:, block] = scale sum_p parts[p] in a fixed order
//    (the per-chunk results of the moment product).
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

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Moment product.  With L_m, R_n complex vectors of K elements stored as 2K
// interleaved doubles Lf, Rf (len = 2K doubles, rows `stride` doubles apart:
// the stores pad their vectors so that the rows a wave reads at once do not
// all fall at the same offset of a power-of-two stride),
//   Re <L_m|R_n> = sum_k' Lf[m][k'] Rf[n][k'],
//   Im <L_m|R_n> = sum_k' Lf[m][k'] Rf'[n][k'],  Rf'[2k] = Rf[2k+1], Rf'[2k+1] = -Rf[2k],
// so both parts are real products over k', taken with
// v_mfma_f64_16x16x4f64: D[i][j] += sum_{s<4} A[i][s] B[s][j], where lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and holds D[4r + l/16][l%16] in
// its result register r.  Lane (g = l/16, i = l%16) of a wave takes rows
// m = m0 + 16t + i of L and n = n0 + 16u + i of R; in a step of 32 doubles
// it loads the pairs at k' + 8q + 2g (q < 4) of each of its rows, and its
// k-slot g of the q-th pair of instructions is k' + 8q + 2g + h (h < 2), the
// same for A and B, so every k' of the step is summed once; the pair
// (2g, 2g+1) it holds is one complex element, which gives Rf' in registers.
// A workgroup is WM x (4/WM) waves, each with TM x TN tiles of 16 x 16
// (with PF, the next step's operands are loaded before the current step's
// products); at most 256 registers per lane, so that the products
// accumulate in ordinary vector registers (two waves per SIMD or more);
// blocks take tiles of one chunk of K' (kchunk doubles, a multiple of 32),
// chunk-major, XCD-contiguous, and write
//   parts[chunk][n][m] = sum_{k' in chunk} (Re, Im) as complex128.
// Rows past n_mom or cnt load a valid row (the last) and store nothing.
// ---------------------------------------------------------------------------
template <int TM, int TN, int WM, bool PF>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2))) void k_kpm_product(const double *__restrict__ L, const double *__restrict__ R,
                                                     int64_t stride, int64_t ld, int32_t n_mom, int32_t cnt, int64_t kchunk,
                                                     int32_t m_groups, int32_t n_groups, int32_t n_blocks,
                                                     d2 *__restrict__ parts) {
    constexpr int WN = 4 / WM;
    const int b = tile_of_block(blockIdx.x, n_blocks, 1);
    const int per_chunk = m_groups * n_groups;
    const int ch = b / per_chunk;
    const int rem = b - ch * per_chunk;
    const int mg = rem % m_groups, ng = rem / m_groups;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave % WM, wn = wave / WM;
    const int g = lane >> 4, i = lane & 15;
    const int m0 = (mg * WM + wm) * TM * 16;
    const int n0 = (ng * WN + wn) * TN * 16;
    if (m0 >= n_mom || n0 >= cnt) return;  // no barrier below: a wave may leave
    const int64_t k0 = (int64_t)ch * kchunk;
    const int64_t k1 = k0 + kchunk < ld ? k0 + kchunk : ld;
    const int64_t kfull = k0 + ((k1 - k0) & ~(int64_t)31);

    const double *lp[TM];
    const double *rp[TN];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        const int m = m0 + 16 * t + i;
        lp[t] = L + (int64_t)(m < n_mom ? m : n_mom - 1) * stride + 2 * g;
    }
#pragma unroll
    for (int u = 0; u < TN; ++u) {
        const int n = n0 + 16 * u + i;
        rp[u] = R + (int64_t)(n < cnt ? n : cnt - 1) * stride + 2 * g;
    }
    d4 cre[TM][TN], cim[TM][TN];
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int u = 0; u < TN; ++u) {
            cre[t][u] = d4{0.0, 0.0, 0.0, 0.0};
            cim[t][u] = d4{0.0, 0.0, 0.0, 0.0};
        }

    d2 a[TM][4], bv[TN][4];
    auto mma = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int t = 0; t < TM; ++t) {
                    const double av = h ? a[t][q].y : a[t][q].x;
#pragma unroll
                    for (int u = 0; u < TN; ++u) {
                        const double br = h ? bv[u][q].y : bv[u][q].x;
                        const double bi = h ? -bv[u][q].x : bv[u][q].y;
                        cre[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, br, cre[t][u], 0, 0, 0);
                        cim[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bi, cim[t][u], 0, 0, 0);
                    }
                }
    };
    auto load = [&](int64_t kk) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int t = 0; t < TM; ++t) a[t][q] = *(const d2 *)(lp[t] + kk + 8 * q);
#pragma unroll
            for (int u = 0; u < TN; ++u) bv[u][q] = *(const d2 *)(rp[u] + kk + 8 * q);
        }
    };
    int64_t k = k0;
    if constexpr (!PF) {
        for (; k < kfull; k += 32) {
            load(k);
            mma();
        }
    }
    if (PF && k < kfull) load(k);
    for (; PF && k < kfull; k += 32) {
        // the next step's operands (the current step again on the last one)
        const int64_t kn = k + 32 < kfull ? k + 32 : k;
        d2 na[TM][4], nb[TN][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int t = 0; t < TM; ++t) na[t][q] = *(const d2 *)(lp[t] + kn + 8 * q);
#pragma unroll
            for (int u = 0; u < TN; ++u) nb[u][q] = *(const d2 *)(rp[u] + kn + 8 * q);
        }
        // keep the next step's loads ahead of this step's products (the
        // scheduler would otherwise sink them to shorten their live ranges)
        __builtin_amdgcn_sched_barrier(0);
        mma();
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int t = 0; t < TM; ++t) a[t][q] = na[t][q];
#pragma unroll
            for (int u = 0; u < TN; ++u) bv[u][q] = nb[u][q];
        }
    }
    if (kfull < k1) {
        // last partial step: pairs at or past k1 are zero (k1 and every pair
        // offset are even, so a pair is wholly inside or wholly outside)
        const d2 z = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool in = kfull + 8 * q + 2 * g < k1;
#pragma unroll
            for (int t = 0; t < TM; ++t) a[t][q] = in ? *(const d2 *)(lp[t] + kfull + 8 * q) : z;
#pragma unroll
            for (int u = 0; u < TN; ++u) bv[u][q] = in ? *(const d2 *)(rp[u] + kfull + 8 * q) : z;
        }
        mma();
    }
    d2 *out = parts + (int64_t)ch * cnt * n_mom;
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int u = 0; u < TN; ++u) {
            const int n = n0 + 16 * u + i;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + 16 * t + 4 * r + g;
                if (m < n_mom && n < cnt) {
                    d2 v;
                    v.x = cre[t][u][r];
                    v.y = cim[t][u][r];
                    out[(int64_t)n * n_mom + m] = v;
                }
            }
        }
}

__global__ __launch_bounds__(kWG) void k_kpm_sum_parts(const d2 *__restrict__ parts, int64_t n_el, int n_parts,
                                                       int64_t part_stride, double scale, d2 *__restrict__ out) {
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
        a.x *= scale;
        a.y *= scale;
        out[i] = a;
    }
}

template <int TM, int TN, int WM, bool PF>
hipError_t launch_product_t(const double *L, const double *R, int64_t stride, int64_t ld, int32_t n_mom,
                            int32_t cnt, int64_t kchunk, int32_t n_chunks, double *parts, hipStream_t st) {
    constexpr int WN = 4 / WM;
    const int32_t m_groups = (n_mom + WM * TM * 16 - 1) / (WM * TM * 16);
    const int32_t n_groups = (cnt + WN * TN * 16 - 1) / (WN * TN * 16);
    const int64_t blocks = (int64_t)m_groups * n_groups * n_chunks;
    if (blocks >= INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_kpm_product<TM, TN, WM, PF>), dim3((unsigned)blocks), dim3(kWG), 0, st, L, R, stride, ld,
                       n_mom, cnt, kchunk, m_groups, n_groups, (int32_t)blocks, (d2 *)parts);
    return hipGetLastError();
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

// Tilings, measured on 512 moments x 128 of R x 2.1M elements: 2 x 4 tiles
// per wave, 2 x 2 waves (shape 0) 51.9 TFLOP/s; 4 x 2 tiles 50.4; 2 x 2 tiles
// with the next step's operands prefetched (three waves per SIMD) 46.8.  The
// bound is the operand stream, not the matrix cores (a product loop with no
// loads issues at 98% of their peak): bigger tiles read less per product.
KpmProductShape kpm_product_shape(int32_t shape) {
    switch (shape) {
        case 1: return {4, 2, 2, 0};
        case 2: return {2, 2, 2, 1};
        default: return {2, 4, 2, 0};
    }
}

hipError_t launch_kpm_product(int32_t shape, const double *L, const double *R, int64_t stride, int64_t ld,
                              int32_t n_mom, int32_t cnt, int64_t kchunk, int32_t n_chunks, double *parts,
                              hipStream_t st) {
    if (kchunk <= 0 || (kchunk & 31) || n_chunks < 1 || n_mom < 1 || cnt < 1 || ld < 2 || (ld & 1) || stride < ld ||
        (stride & 1) || (int64_t)(n_chunks - 1) * kchunk >= ld || (int64_t)n_chunks * kchunk < ld)
        return hipErrorInvalidValue;
    switch (shape) {
        case 1: return launch_product_t<4, 2, 2, false>(L, R, stride, ld, n_mom, cnt, kchunk, n_chunks, parts, st);
        case 2: return launch_product_t<2, 2, 2, true>(L, R, stride, ld, n_mom, cnt, kchunk, n_chunks, parts, st);
        default: return launch_product_t<2, 4, 2, false>(L, R, stride, ld, n_mom, cnt, kchunk, n_chunks, parts, st);
    }
}

hipError_t launch_kpm_sum_parts(const double *parts, int64_t n_el, int32_t n_parts, int64_t part_stride, double scale,
                                double *out, hipStream_t st) {
    int64_t b = (n_el + kWG - 1) / kWG;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_kpm_sum_parts, dim3((unsigned)b), dim3(kWG), 0, st, (const d2 *)parts, n_el, n_parts,
                       part_stride, scale, (d2 *)out);
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
