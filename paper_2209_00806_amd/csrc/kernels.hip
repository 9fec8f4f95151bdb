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

#include "tbpm_internal.h"

namespace tbpm {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

template <typename R>
struct CxT;
template <>
struct CxT<double> {
    using T = d2;
};
template <>
struct CxT<float> {
    using T = f2;
};

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// acc += h * x for a real or complex matrix element h
template <typename C, typename R>
__device__ __forceinline__ C hmad(R h, C x, C acc) {
    acc.x = fma(h, x.x, acc.x);
    acc.y = fma(h, x.y, acc.y);
    return acc;
}
template <typename C>
__device__ __forceinline__ C hmad(C h, C x, C acc) {
    acc.x = fma(h.x, x.x, acc.x);
    acc.x = fma(-h.y, x.y, acc.x);
    acc.y = fma(h.x, x.y, acc.y);
    acc.y = fma(h.y, x.x, acc.y);
    return acc;
}

template <bool NT, typename T>
__device__ __forceinline__ T ldv(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void stv(T *p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Blocks are dispatched round-robin over the 8 XCDs; remap so that XCD x
// works through one contiguous range of tiles (the neighbour rows gathered
// by a tile were then most likely brought into the same XCD's L2).
__device__ __forceinline__ int tile_of_block(int b, int n_tiles, int remap) {
    if (!remap) return b;
    const int q = n_tiles >> 3, r = n_tiles & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Sum (dre, dim, nrm) over the threads of the workgroup that hold the same
// state (thread t holds state t & (S-1)) in a fixed order, and write the
// workgroup's partial sums for each state.
__device__ __forceinline__ void block_state_partials(double dre, double dim, double nrm, int log2s,
                                                     double *__restrict__ out /* [S][3] */) {
    __shared__ double red[kWG / 64][64][3];
    const int S = 1 << log2s;
    for (int off = 32; off >= S; off >>= 1) {
        dre += __shfl_xor(dre, off);
        dim += __shfl_xor(dim, off);
        nrm += __shfl_xor(nrm, off);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < S) {
        red[wave][lane][0] = dre;
        red[wave][lane][1] = dim;
        red[wave][lane][2] = nrm;
    }
    __syncthreads();
    if (threadIdx.x < S) {
        double a = 0, b = 0, c = 0;
#pragma unroll
        for (int w = 0; w < kWG / 64; ++w) {
            a += red[w][threadIdx.x][0];
            b += red[w][threadIdx.x][1];
            c += red[w][threadIdx.x][2];
        }
        out[threadIdx.x * 3 + 0] = a;
        out[threadIdx.x * 3 + 1] = b;
        out[threadIdx.x * 3 + 2] = c;
    }
}

// ---------------------------------------------------------------------------
// Chebyshev/Clenshaw pass
// ---------------------------------------------------------------------------
template <typename R, bool CH, int KIND, bool NT>
__global__ __launch_bounds__(kWG) void k_pass(const PassParams p) {
    using C = typename CxT<R>::T;
    using HV = std::conditional_t<CH, C, R>;
    constexpr bool X_IS_V = (KIND == kPassFirst);
    constexpr bool HAS_B2 = (KIND == kPassMid || KIND == kPassLast);
    constexpr bool CORR = (KIND == kPassLast || KIND == kPassLastNoB2);

    const int tile = tile_of_block(blockIdx.x, p.n_tiles, p.xcd_remap);
    const TileDesc td = p.tiles[tile];
    const PassCoef pc = p.coef[td.inst];
    C alpha, beta;
    alpha.x = (R)pc.ar;
    alpha.y = (R)pc.ai;
    beta.x = (R)pc.br;
    beta.y = (R)pc.bi;
    const int log2s = p.log2s;
    const int64_t smask = (1 << log2s) - 1;
    const int64_t n_el = (int64_t)td.rows << log2s;
    const int64_t e0 = td.row0 << log2s;

    if (p.bump_counter && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(p.counter, 1);

    const C *__restrict__ x = (const C *)p.x;
    const C *v = (const C *)p.v;
    const C *b2 = (const C *)p.b2;
    C *out = (C *)p.out;
    const R *__restrict__ ons = (const R *)p.onsite;
    const HV *__restrict__ val = (const HV *)p.val;
    const int32_t *__restrict__ col = p.col;
    const int64_t *__restrict__ soff = p.slice_off;

    double dre = 0.0, dim = 0.0, nrm = 0.0;
    bool do_ckpt = false;
    int64_t ckpt_base = 0;
    if constexpr (CORR) {
        if (p.ckpt_every > 0) {
            const int step = *(volatile const int32_t *)p.counter;
            do_ckpt = (step % p.ckpt_every == 0) && step <= p.ckpt_max && step > 0;
            ckpt_base = (int64_t)(step / p.ckpt_every - 1);
        }
    }

    for (int64_t e = threadIdx.x; e < n_el; e += kWG) {
        const int64_t row = td.row0 + (e >> log2s);
        const int s = (int)(e & smask);
        const int64_t g = e0 + e;
        const int64_t sl = row / kSliceRows;
        const int64_t off = soff[sl];
        const int w = (int)((soff[sl + 1] - off) / kSliceRows);
        const int64_t base = off + (row % kSliceRows);
        const C xo = x[g];
        C acc;
        acc.x = ons[row] * xo.x;
        acc.y = ons[row] * xo.y;
        for (int k = 0; k < w; ++k) {
            const int c = col[base + (int64_t)k * kSliceRows];
            const HV h = val[base + (int64_t)k * kSliceRows];
            const C xc = x[((int64_t)c << log2s) + s];
            acc = hmad(h, xc, acc);
        }
        C vv;
        if constexpr (X_IS_V)
            vv = xo;
        else
            vv = ldv<NT>(v + g);
        C o = cmul(alpha, vv) + cmul(beta, acc);
        if constexpr (HAS_B2) o -= ldv<NT>(b2 + g);
        if constexpr (CORR) {
            stv<false>(out + g, o);
            const d2 ph = ((const d2 *)p.phi0)[row * p.phi0_ld + s];
            const double oxr = (double)o.x, oyi = (double)o.y;
            dre = fma(ph.x, oxr, fma(ph.y, oyi, dre));
            dim = fma(ph.x, oyi, fma(-ph.y, oxr, dim));
            nrm = fma(oxr, oxr, fma(oyi, oyi, nrm));
            if (do_ckpt && s < p.s_user) {
                d2 oc;
                oc.x = oxr;
                oc.y = oyi;
                ((d2 *)p.ckpt)[ckpt_base * p.ckpt_stride + row * p.s_user + s] = oc;
            }
        } else {
            stv<NT>(out + g, o);
        }
    }
    if constexpr (CORR) block_state_partials(dre, dim, nrm, log2s, p.partials + (int64_t)tile * (3 << log2s));
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
        const int64_t lrow = lrow0 + (e >> log2s);
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
    block_state_partials(dre, dim, nrm, log2s, p.partials + (int64_t)blockIdx.x * (3 << log2s));
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
    const int S = 1 << p.log2s;
    const int t0 = p.inst_tile0[inst], t1 = p.inst_tile0[inst + 1];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int t = t0 + threadIdx.x; t < t1; t += kWG) {
        const double *q = p.partials + ((int64_t)t * S + s) * 3;
        a += q[0];
        b += q[1];
        c += q[2];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    red[2][threadIdx.x] = c;
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
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
            p.norm2_all[(int64_t)inst * p.n_steps * p.s_user + o] = red[2][0];
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
                                                        int64_t n_rows, void *val64, void *val32,
                                                        double *ons64, float *ons32) {
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
        ons64[r] = csr_onsite[r];
        ons32[r] = (float)csr_onsite[r];
    }
}

// Plain streaming copy (bandwidth calibration).
__global__ __launch_bounds__(kWG) void k_copy(const d2 *__restrict__ src, d2 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename R, bool CH, bool NT>
hipError_t launch_pass_t(int kind, const PassParams &p, hipStream_t st) {
    const dim3 grid(p.n_tiles), block(kWG);
    switch (kind) {
        case kPassFirst:
            hipLaunchKernelGGL((k_pass<R, CH, kPassFirst, NT>), grid, block, 0, st, p);
            break;
        case kPassNoB2:
            hipLaunchKernelGGL((k_pass<R, CH, kPassNoB2, NT>), grid, block, 0, st, p);
            break;
        case kPassMid:
            hipLaunchKernelGGL((k_pass<R, CH, kPassMid, NT>), grid, block, 0, st, p);
            break;
        case kPassLast:
            hipLaunchKernelGGL((k_pass<R, CH, kPassLast, NT>), grid, block, 0, st, p);
            break;
        case kPassLastNoB2:
            hipLaunchKernelGGL((k_pass<R, CH, kPassLastNoB2, NT>), grid, block, 0, st, p);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pass(int kind, bool fp32, bool cplx, bool nontemporal, const PassParams &p,
                       hipStream_t st) {
    if (p.n_tiles <= 0) return hipSuccess;
    if (fp32) {
        if (cplx) return nontemporal ? launch_pass_t<float, true, true>(kind, p, st) : launch_pass_t<float, true, false>(kind, p, st);
        return nontemporal ? launch_pass_t<float, false, true>(kind, p, st) : launch_pass_t<float, false, false>(kind, p, st);
    }
    if (cplx) return nontemporal ? launch_pass_t<double, true, true>(kind, p, st) : launch_pass_t<double, true, false>(kind, p, st);
    return nontemporal ? launch_pass_t<double, false, true>(kind, p, st) : launch_pass_t<double, false, false>(kind, p, st);
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
                           csr_val, csr_onsite, n_rows, m.val64, m.val32, m.onsite64, m.onsite32);
    else
        hipLaunchKernelGGL(k_convert_values<false>, dim3((unsigned)blocks), dim3(kWG), 0, st, m.ell_csr, m.ell_size,
                           csr_val, csr_onsite, n_rows, m.val64, m.val32, m.onsite64, m.onsite32);
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
