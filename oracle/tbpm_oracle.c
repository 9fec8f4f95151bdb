/*
 * TBPM oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 implementation of the TBPM DOS
 * propagation and of its discrete adjoint.  It exists to check the HIP
 * library; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code with the library.
 *
 * Method (paper, Sec. "Tight-binding propagation method"):
 *   H~ = H / f                                  (rescaling, ||H|| -> f)
 *   psi(t + dt) = [J_0(z) T^_0 + 2 sum_{m>=1} J_m(z) T^_m] psi(t),  z = f dt
 *   T^_0 psi = psi,  T^_1 psi = -i H~ psi,
 *   T^_{m+1} psi = -2i H~ T^_m psi + T^_{m-1} psi       (modified recurrence)
 *   C(t) = <psi(0)|psi(t)>                       (DOS correlation, Eq. corr_dos)
 * The series is truncated after M terms (m = 0..M-1); the Bessel values are
 * computed by the Python side of the oracle and passed in.
 *
 * Matrix: CSR of the off-diagonal elements (row_ptr, col, val as interleaved
 * re/im) plus the real on-site energies eps_i on the diagonal.
 * States: psi0[i*S + s] (orbital-major, S states interleaved), complex.
 *
 * Sums over orbitals use Neumaier compensation so that the oracle's
 * reductions are accurate to a few ulps independently of N.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Neumaier-compensated accumulator */
typedef struct {
    double sum, comp;
} ksum;

static void ksum_add(ksum *k, double x) {
    double t = k->sum + x;
    if (fabs(k->sum) >= fabs(x))
        k->comp += (k->sum - t) + x;
    else
        k->comp += (x - t) + k->sum;
    k->sum = t;
}

static double ksum_value(const ksum *k) { return k->sum + k->comp; }

/* y = H~ x = (eps .* x + H_off x) / f */
static void apply_scaled_h(int64_t n, const int64_t *row_ptr, const int32_t *col, const cplx *val,
                           const double *onsite, double f, const cplx *x, cplx *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        cplx acc = onsite[i] * x[i];
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) acc += val[p] * x[col[p]];
        y[i] = acc / f;
    }
}

/* <a|b> and ||b||^2 with compensated sums */
static void inner_and_norm(int64_t n, const cplx *a, const cplx *b, cplx *dot, double *nrm) {
    ksum re = {0, 0}, im = {0, 0}, nn = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        cplx p = conj(a[i]) * b[i];
        ksum_add(&re, creal(p));
        ksum_add(&im, cimag(p));
        ksum_add(&nn, creal(b[i]) * creal(b[i]));
        ksum_add(&nn, cimag(b[i]) * cimag(b[i]));
    }
    *dot = ksum_value(&re) + I * ksum_value(&im);
    *nrm = ksum_value(&nn);
}

/* One time step: out = [J_0 T^_0 + 2 sum_{m=1}^{M-1} J_m T^_m] psi.
 * If 'T' is non-NULL it receives all M vectors T^_m psi (T[m*n + i]). */
static void time_step(int64_t n, const int64_t *row_ptr, const int32_t *col, const cplx *val,
                      const double *onsite, double f, int32_t M, const double *J, const cplx *psi,
                      cplx *out, cplx *T, cplx *w0, cplx *w1, cplx *w2, cplx *h) {
    cplx *tm1 = w0, *tm = w1, *tp = w2;
    for (int64_t i = 0; i < n; ++i) {
        tm1[i] = psi[i];
        out[i] = J[0] * psi[i];
    }
    if (T) memcpy(T, psi, (size_t)n * sizeof(cplx));
    if (M < 2) return;
    apply_scaled_h(n, row_ptr, col, val, onsite, f, psi, h);
    for (int64_t i = 0; i < n; ++i) {
        tm[i] = -I * h[i];
        out[i] += 2.0 * J[1] * tm[i];
    }
    if (T) memcpy(T + n, tm, (size_t)n * sizeof(cplx));
    for (int32_t m = 2; m < M; ++m) {
        apply_scaled_h(n, row_ptr, col, val, onsite, f, tm, h);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            tp[i] = -2.0 * I * h[i] + tm1[i];
            out[i] += 2.0 * J[m] * tp[i];
        }
        if (T) memcpy(T + (size_t)m * n, tp, (size_t)n * sizeof(cplx));
        cplx *r = tm1;
        tm1 = tm;
        tm = tp;
        tp = r;
    }
}

/*
 * Propagate S states for n_steps correlation samples.
 *   corr[k*S + s]  = <phi0_s | psi_s(k dt)>,   k = 0 .. n_steps-1
 *   norm2[k*S + s] = ||psi_s(k dt)||^2
 * psi_s(0) = phi0_s; n_steps-1 time steps are taken.
 * Returns 0 on success, -1 on allocation failure.
 */
int oracle_propagate(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_ri,
                     const double *onsite, double f, int32_t S, const double *phi0_ri, int32_t n_steps,
                     int32_t M, const double *J, double *corr_ri, double *norm2) {
    const cplx *val = (const cplx *)val_ri;
    const cplx *phi0 = (const cplx *)phi0_ri;
    cplx *corr = (cplx *)corr_ri;
    cplx *buf = malloc(sizeof(cplx) * (size_t)n * 7);
    if (!buf) return -1;
    cplx *p0 = buf, *psi = buf + n, *nxt = buf + 2 * n, *w0 = buf + 3 * n, *w1 = buf + 4 * n,
         *w2 = buf + 5 * n, *h = buf + 6 * n;
    for (int32_t s = 0; s < S; ++s) {
        for (int64_t i = 0; i < n; ++i) p0[i] = psi[i] = phi0[i * S + s];
        for (int32_t k = 0; k < n_steps; ++k) {
            cplx c;
            double nn;
            inner_and_norm(n, p0, psi, &c, &nn);
            corr[(int64_t)k * S + s] = c;
            if (norm2) norm2[(int64_t)k * S + s] = nn;
            if (k == n_steps - 1) break;
            time_step(n, row_ptr, col, val, onsite, f, M, J, psi, nxt, NULL, w0, w1, w2, h);
            cplx *t = psi;
            psi = nxt;
            nxt = t;
        }
    }
    free(buf);
    return 0;
}

/*
 * Snapshots of the propagated states (the wave-function propagation of the
 * paper's usage section): snaps[(q*n + i)*S + s] = psi_s(steps[q] dt)_i for
 * q = 0 .. n_snap-1, with the same time step as oracle_propagate.  steps must
 * be non-negative; they need not be sorted.
 * Returns 0 on success, -1 on allocation failure or a negative step.
 */
int oracle_psi_t(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_ri,
                 const double *onsite, double f, int32_t S, const double *phi0_ri, int32_t n_snap,
                 const int32_t *steps, int32_t M, const double *J, double *snaps_ri) {
    const cplx *val = (const cplx *)val_ri;
    const cplx *phi0 = (const cplx *)phi0_ri;
    cplx *snaps = (cplx *)snaps_ri;
    int32_t last = 0;
    for (int32_t q = 0; q < n_snap; ++q) {
        if (steps[q] < 0) return -1;
        if (steps[q] > last) last = steps[q];
    }
    cplx *buf = malloc(sizeof(cplx) * (size_t)n * 6);
    if (!buf) return -1;
    cplx *psi = buf, *nxt = buf + n, *w0 = buf + 2 * n, *w1 = buf + 3 * n, *w2 = buf + 4 * n, *h = buf + 5 * n;
    for (int32_t s = 0; s < S; ++s) {
        for (int64_t i = 0; i < n; ++i) psi[i] = phi0[i * S + s];
        for (int32_t k = 0; k <= last; ++k) {
            for (int32_t q = 0; q < n_snap; ++q)
                if (steps[q] == k)
                    for (int64_t i = 0; i < n; ++i) snaps[((int64_t)q * n + i) * S + s] = psi[i];
            if (k == last) break;
            time_step(n, row_ptr, col, val, onsite, f, M, J, psi, nxt, NULL, w0, w1, w2, h);
            cplx *t = psi;
            psi = nxt;
            nxt = t;
        }
    }
    free(buf);
    return 0;
}

/*
 * Chebyshev series of an operator (Sec. "Tight-binding propagation method",
 * decomposition of other operators): out_s = sum_{k<K} a[k] T_k(H~) psi_s with
 * H~ = H/f, by the forward recurrence T_0 psi = psi, T_1 psi = H~ psi,
 * T_{k+1} psi = 2 H~ T_k psi - T_{k-1} psi.  Returns 0, or -1 on allocation failure.
 */
int oracle_apply_cheb(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_ri,
                      const double *onsite, double f, int32_t S, const double *psi_ri, int32_t K, const double *a,
                      double *out_ri) {
    const cplx *val = (const cplx *)val_ri;
    const cplx *psi = (const cplx *)psi_ri;
    cplx *out = (cplx *)out_ri;
    cplx *buf = malloc(sizeof(cplx) * (size_t)n * 4);
    if (!buf) return -1;
    cplx *tm1 = buf, *tm = buf + n, *tp = buf + 2 * n, *h = buf + 3 * n;
    for (int32_t s = 0; s < S; ++s) {
        for (int64_t i = 0; i < n; ++i) {
            tm1[i] = psi[i * S + s];
            out[i * S + s] = a[0] * tm1[i];
        }
        if (K > 1) {
            apply_scaled_h(n, row_ptr, col, val, onsite, f, tm1, tm);
            for (int64_t i = 0; i < n; ++i) out[i * S + s] += a[1] * tm[i];
        }
        for (int32_t k = 2; k < K; ++k) {
            apply_scaled_h(n, row_ptr, col, val, onsite, f, tm, h);
            for (int64_t i = 0; i < n; ++i) {
                tp[i] = 2.0 * h[i] - tm1[i];
                out[i * S + s] += a[k] * tp[i];
            }
            cplx *r = tm1;
            tm1 = tm;
            tm = tp;
            tp = r;
        }
    }
    free(buf);
    return 0;
}

/*
 * Optical-conductivity correlation (Sec. "Optical conductivity"): both
 * states are propagated with the series of oracle_propagate and
 *   corr[k*S + s] = <psi2_s(k dt)| J_a |psi1_s(k dt)>,  k = 0 .. n_steps-1,
 * where J_a has the sparsity pattern of H (values ja_ri, no diagonal).
 * Returns 0, or -1 on allocation failure.
 */
int oracle_ac_corr(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_ri, const double *onsite,
                   double f, int32_t S, const double *psi1_ri, const double *psi2_ri, int32_t n_steps, int32_t M,
                   const double *J, const double *ja_ri, double *corr_ri) {
    const cplx *val = (const cplx *)val_ri;
    const cplx *ja = (const cplx *)ja_ri;
    const cplx *psi1 = (const cplx *)psi1_ri, *psi2 = (const cplx *)psi2_ri;
    cplx *corr = (cplx *)corr_ri;
    cplx *buf = malloc(sizeof(cplx) * (size_t)n * 9);
    if (!buf) return -1;
    cplx *p1 = buf, *p2 = buf + n, *nx1 = buf + 2 * n, *nx2 = buf + 3 * n, *w0 = buf + 4 * n, *w1 = buf + 5 * n,
         *w2 = buf + 6 * n, *h = buf + 7 * n, *jp = buf + 8 * n;
    for (int32_t s = 0; s < S; ++s) {
        for (int64_t i = 0; i < n; ++i) {
            p1[i] = psi1[i * S + s];
            p2[i] = psi2[i * S + s];
        }
        for (int32_t k = 0; k < n_steps; ++k) {
            for (int64_t i = 0; i < n; ++i) {
                cplx acc = 0;
                for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) acc += ja[q] * p1[col[q]];
                jp[i] = acc;
            }
            ksum re = {0, 0}, im = {0, 0};
            for (int64_t i = 0; i < n; ++i) {
                const cplx c = conj(p2[i]) * jp[i];
                ksum_add(&re, creal(c));
                ksum_add(&im, cimag(c));
            }
            corr[(int64_t)k * S + s] = ksum_value(&re) + I * ksum_value(&im);
            if (k == n_steps - 1) break;
            time_step(n, row_ptr, col, val, onsite, f, M, J, p1, nx1, NULL, w0, w1, w2, h);
            time_step(n, row_ptr, col, val, onsite, f, M, J, p2, nx2, NULL, w0, w1, w2, h);
            cplx *t = p1;
            p1 = nx1;
            nx1 = t;
            t = p2;
            p2 = nx2;
            nx2 = t;
        }
    }
    free(buf);
    return 0;
}

/*
 * Discrete adjoint of oracle_propagate (reverse-mode differentiation of the
 * recurrence above, written out by hand).
 *
 * Input  gcorr[k*S + s] = G_k with dL = Re sum_k conj(G_k) dC_k  (complex).
 * Output grad_val[p]    = G_pq with dL = Re sum_pq conj(G_pq) dH_pq for every
 *                         stored off-diagonal entry p = (row, col) (complex),
 *        grad_onsite[i] = dL/d eps_i (real),
 * summed over the S states.  f and dt are held fixed.
 *
 * All psi_k are stored (n_steps * n complex per state): tiny systems only.
 */
int oracle_backward(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_ri,
                    const double *onsite, double f, int32_t S, const double *phi0_ri, int32_t n_steps,
                    int32_t M, const double *J, const double *gcorr_ri, double *grad_val_ri,
                    double *grad_onsite) {
    const cplx *val = (const cplx *)val_ri;
    const cplx *phi0 = (const cplx *)phi0_ri;
    const cplx *gcorr = (const cplx *)gcorr_ri;
    cplx *grad_val = (cplx *)grad_val_ri;
    const int64_t nnz = row_ptr[n];
    cplx *gdiag = calloc((size_t)n, sizeof(cplx));
    cplx *gacc = calloc((size_t)nnz > 0 ? (size_t)nnz : 1, sizeof(cplx));
    cplx *hist = malloc(sizeof(cplx) * (size_t)n * (size_t)n_steps);
    cplx *T = malloc(sizeof(cplx) * (size_t)n * (size_t)(M > 0 ? M : 1));
    cplx *Tb = malloc(sizeof(cplx) * (size_t)n * (size_t)(M > 0 ? M : 1));
    cplx *buf = malloc(sizeof(cplx) * (size_t)n * 8);
    if (!gdiag || !gacc || !hist || !T || !Tb || !buf) {
        free(gdiag); free(gacc); free(hist); free(T); free(Tb); free(buf);
        return -1;
    }
    cplx *p0 = buf, *lam = buf + n, *w0 = buf + 2 * n, *w1 = buf + 3 * n, *w2 = buf + 4 * n,
         *h = buf + 5 * n, *nxt = buf + 6 * n, *tmp = buf + 7 * n;

    for (int32_t s = 0; s < S; ++s) {
        for (int64_t i = 0; i < n; ++i) p0[i] = hist[i] = phi0[i * S + s];
        /* forward sweep, keeping every psi_k */
        for (int32_t k = 0; k + 1 < n_steps; ++k)
            time_step(n, row_ptr, col, val, onsite, f, M, J, hist + (size_t)k * n,
                      hist + (size_t)(k + 1) * n, NULL, w0, w1, w2, h);
        if (n_steps < 2) continue;
        /* lambda_{N-1} = G_{N-1} phi0 */
        for (int64_t i = 0; i < n; ++i) lam[i] = gcorr[(int64_t)(n_steps - 1) * S + s] * p0[i];
        for (int32_t l = n_steps - 2; l >= 0; --l) {
            /* recompute T^_m psi_l, m = 0..M-1 */
            time_step(n, row_ptr, col, val, onsite, f, M, J, hist + (size_t)l * n, nxt, T, w0, w1,
                      w2, h);
            /* psi_{l+1} = sum_m a_m T_m with a_0 = J_0, a_m = 2 J_m */
            for (int32_t m = 0; m < M; ++m) {
                double a = (m == 0) ? J[0] : 2.0 * J[m];
                for (int64_t i = 0; i < n; ++i) Tb[(size_t)m * n + i] = a * lam[i];
            }
            /* T_m = -2i H~ T_{m-1} + T_{m-2},  m = M-1 .. 2 */
            for (int32_t m = M - 1; m >= 2; --m) {
                const cplx *tb = Tb + (size_t)m * n;
                const cplx *tprev = T + (size_t)(m - 1) * n;
                for (int64_t i = 0; i < n; ++i) {
                    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                        gacc[p] += 2.0 * I * tb[i] * conj(tprev[col[p]]);
                    gdiag[i] += 2.0 * I * tb[i] * conj(tprev[i]);
                }
                apply_scaled_h(n, row_ptr, col, val, onsite, f, tb, tmp);
                for (int64_t i = 0; i < n; ++i) {
                    Tb[(size_t)(m - 1) * n + i] += 2.0 * I * tmp[i];
                    Tb[(size_t)(m - 2) * n + i] += tb[i];
                }
            }
            /* T_1 = -i H~ T_0 */
            if (M >= 2) {
                const cplx *tb = Tb + n;
                for (int64_t i = 0; i < n; ++i) {
                    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                        gacc[p] += I * tb[i] * conj(T[col[p]]);
                    gdiag[i] += I * tb[i] * conj(T[i]);
                }
                apply_scaled_h(n, row_ptr, col, val, onsite, f, tb, tmp);
                for (int64_t i = 0; i < n; ++i) Tb[i] += I * tmp[i];
            }
            /* lambda_l = (adjoint of psi_l through the step) + G_l phi0 */
            for (int64_t i = 0; i < n; ++i) lam[i] = Tb[i] + gcorr[(int64_t)l * S + s] * p0[i];
        }
    }
    /* the recurrence is in H~ = H/f: dL/dH = dL/dH~ / f */
    for (int64_t p = 0; p < nnz; ++p) grad_val[p] = gacc[p] / f;
    for (int64_t i = 0; i < n; ++i) grad_onsite[i] = creal(gdiag[i]) / f;
    free(gdiag); free(gacc); free(hist); free(T); free(Tb); free(buf);
    return 0;
}
