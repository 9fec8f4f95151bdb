/*
 * libtbpm -- TBPM (tight-binding propagation method) on AMD Instinct MI355X.
 *
 * C ABI over hand-written HIP kernels for gfx950.  The library evolves
 * random initial states under a sparse Hermitian tight-binding Hamiltonian
 * with the Chebyshev/Bessel expansion of exp(-i H dt), records the DOS
 * correlation C(t) = <psi(0)|psi(t)> at every step, and turns the
 * sample-averaged correlation into a density of states (paper: Sec.
 * "Tight-binding propagation method", Eq. (eq:psi_t); Sec. "Density of
 * states", Eq. (eq:corr_dos) and Eq. (dos_tbpm)).  It also provides the
 * exact adjoint of that computation (gradients of a loss on the DOS with
 * respect to the hoppings and on-site energies), a batched form that
 * propagates many Hamiltonians in one launch sequence, and an FP32
 * recursion with FP64 reductions.
 *
 * General conventions
 *   - Every function returns a tbpm_status and never throws; on error
 *     tbpm_last_error() gives a message (thread-local).
 *   - Complex numbers are interleaved (re, im) pairs of double, i.e. the
 *     memory layout of complex128 / double2.
 *   - State vectors are orbital-major with the states interleaved:
 *     psi[(i * n_states + s) * 2 + {0: re, 1: im}], i.e. [n_orb][n_states]
 *     complex128.  Correlations are [n_steps][n_states] complex128.
 *   - "device" pointers are HIP device memory on the current device;
 *     "host" pointers are ordinary host memory.  The caller owns every
 *     buffer it passes in; the library owns only what its handles hold.
 *   - A handle lives on the device that was current when it was created;
 *     every call that uses it must be made with that device current
 *     (TBPM_E_ARG otherwise, before any work is enqueued).
 *   - Work is enqueued on the caller's HIP stream (a hipStream_t passed as
 *     void*; NULL means the default stream).
 *   - Inputs are validated on the host before any device work.
 *   - Limits: n_orb < 2^31 per Hamiltonian and in total per batch.
 */
#ifndef TBPM_H
#define TBPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tbpm_hamiltonian tbpm_hamiltonian; /* opaque, library-owned device copy of H */
typedef struct tbpm_batch tbpm_batch;             /* opaque, several Hamiltonians concatenated */

typedef enum {
    TBPM_OK = 0,
    TBPM_E_ARG = 1,           /* bad argument: NULL pointer, size out of range, non-finite value */
    TBPM_E_CSR = 2,           /* malformed CSR: row_ptr not monotone, column out of range, diagonal entry */
    TBPM_E_NOT_HERMITIAN = 3, /* |H_ij - conj(H_ji)| > 1e-13 max|H| for some stored pair */
    TBPM_E_OOM = 4,           /* device or host allocation failed */
    TBPM_E_DEVICE = 5,        /* HIP runtime error (no device, launch or copy failure) */
    TBPM_E_DIVERGED = 6       /* norm check failed: the spectrum is not inside [-rescale, rescale] */
} tbpm_status;

typedef enum {
    TBPM_FP64 = 0,      /* complex128 states, FP64 matrix and arithmetic */
    TBPM_FP32_MIXED = 1 /* complex64 states and FP32 recursion; correlation, norm and DOS in FP64 */
} tbpm_precision;

typedef enum {
    TBPM_WIN_HANN = 0, /* w_k = (1 + cos(pi k / n_steps)) / 2 */
    TBPM_WIN_NONE = 1  /* w_k = 1 */
} tbpm_window;

/* flags */
#define TBPM_FLAG_HOST_PTRS 0x0u   /* create, set_values: the arrays are host memory (the default) */
#define TBPM_FLAG_DEVICE_PTRS 0x1u /* create, set_values: the arrays are device memory of the current device */
#define TBPM_FLAG_ASYNC 0x2u       /* propagate: do not synchronise; skip the norm check */
#define TBPM_FLAG_NO_GRAPH 0x4u    /* propagate: plain kernel launches instead of a replayed HIP graph */

/* ------------------------------------------------------------------------
 * Hamiltonian
 * ------------------------------------------------------------------------ */

/*
 * Build the device Hamiltonian H_ij = eps_i delta_ij + (off-diagonal
 * element)_ij of a tight-binding model (paper: Sec. "Tight-binding models",
 * Eq. (hal) and Eq. (eq:ham_mat_finite)).
 *
 *   n_orb    number of orbitals (rows), 1 <= n_orb < 2^31.
 *   row_ptr  [n_orb + 1], row_ptr[0] = 0, non-decreasing; nnz = row_ptr[n_orb].
 *   col_idx  [nnz], column of each stored off-diagonal element, in [0, n_orb),
 *            never equal to its row.  Order inside a row is free; repeated
 *            (row, col) pairs are summed.
 *   val      [2 * nnz] doubles, the complex matrix elements H_ij (not -t_ij:
 *            a hopping written "t = -2.7 eV" is passed as -2.7).  The FULL Hermitian
 *            pattern is required (both (i,j) and (j,i)); the paper's half list with
 *            t_ij(R) = t_ji(-R)^* must be expanded by the caller.
 *   onsite   [n_orb], real on-site energies eps_i (eV).
 *   flags    TBPM_FLAG_HOST_PTRS (0): the four arrays are host memory.
 *            TBPM_FLAG_DEVICE_PTRS: they are device memory of the current
 *            device (TBPM_E_ARG otherwise); the library reads them into its
 *            own host copy (row_ptr first, then the rest; synchronous), so
 *            the caller keeps no host copy.  Every check below then runs on
 *            that copy, exactly as for host pointers.
 *   out      receives the handle; release with tbpm_hamiltonian_destroy.
 * The caller keeps ownership of the arrays; the library copies them.
 * Errors: TBPM_E_ARG, TBPM_E_CSR, TBPM_E_NOT_HERMITIAN (checked on the host
 * before the device copy of H is built), TBPM_E_OOM, TBPM_E_DEVICE.  On
 * error *out is NULL.  If every stored element has zero imaginary part the
 * device copy is real.
 * Host work: the checks, the merge and the internal row order run on up to
 * 16 host threads for large inputs (from 2^20 stored elements, or 2^16 rows
 * for the row order), started and joined inside the call; the handle and
 * every error are the same on any number of threads.
 */
tbpm_status tbpm_hamiltonian_create(int64_t n_orb, const int64_t *row_ptr, const int32_t *col_idx,
                                    const double *val, const double *onsite, uint32_t flags,
                                    tbpm_hamiltonian **out);

/*
 * Replace the values of H on the same pattern: val [2 * nnz] in the merged
 * CSR order (rows in order, columns ascending inside a row, duplicates merged;
 * see tbpm_hamiltonian_pattern -- for an input that is already sorted and
 * duplicate-free this is the input order), onsite [n_orb].  With
 * TBPM_FLAG_DEVICE_PTRS both are device pointers, the copy is enqueued on
 * 'stream' and Hermiticity is NOT re-checked; otherwise host pointers,
 * validated like create.  A real H stays real: the imaginary parts of val
 * are ignored unless H was created complex.  Values set from device pointers
 * never reach the host, so the Gershgorin bound of the new values is not
 * known: until host values are set again (or the row order is set, which
 * re-uploads the last host values), every call on H that would take that
 * bound (rescale <= 0) returns TBPM_E_ARG, and tbpm_hamiltonian_info reports
 * the bound of the last host values.
 */
tbpm_status tbpm_hamiltonian_set_values(tbpm_hamiltonian *H, const double *val, const double *onsite,
                                        uint32_t flags, void *stream);

/*
 * Row order used on the device.  The library may renumber the orbitals
 * internally so that rows coupled by H sit close together (recursive
 * bisection of the graph of H: compact groups of rows, which the two-order
 * launch shape needs for small halos); every array crossing this interface
 * (states, checkpoints, values, gradients) stays in the caller's order.
 *   order  -1: automatic (the default): renumber Hamiltonians of at least
 *              16384 orbitals when it shrinks the rows a 128-row tile
 *              references outside itself by 15% or more
 *           0: keep the caller's order;  1: always renumber
 * Setting it re-uploads H from the values last given on the host (at
 * creation or by a host-pointer tbpm_hamiltonian_set_values) and drops
 * cached launch state; the launch configurations are kept.  A batch takes
 * the order of each member's handle at tbpm_batch_create.
 * tbpm_hamiltonian_get_row_order reports the order in use (0 or 1).
 */
tbpm_status tbpm_hamiltonian_set_row_order(tbpm_hamiltonian *H, int32_t order);
tbpm_status tbpm_hamiltonian_get_row_order(const tbpm_hamiltonian *H, int32_t *order);

/*
 * Query H.  Any output pointer may be NULL.
 *   n_orb, nnz   sizes of the stored pattern (nnz after merging duplicates)
 *   gershgorin   max_i (|eps_i| + sum_j |H_ij|), an upper bound of ||H|| used
 *                when a propagate call passes rescale <= 0 (paper, Sec. "Tight-
 *                binding propagation method": rescaling H~ = H/||H||)
 *   is_complex   1 if the device copy holds complex elements
 *   max_row      largest number of stored off-diagonal elements in a row
 */
tbpm_status tbpm_hamiltonian_info(const tbpm_hamiltonian *H, int64_t *n_orb, int64_t *nnz,
                                  double *gershgorin, int32_t *is_complex, int32_t *max_row);

/* The CSR pattern after merging duplicates (host arrays of n_orb+1 and nnz). */
tbpm_status tbpm_hamiltonian_pattern(const tbpm_hamiltonian *H, int64_t *row_ptr, int32_t *col_idx);

tbpm_status tbpm_hamiltonian_destroy(tbpm_hamiltonian *H);

/* ------------------------------------------------------------------------
 * Chebyshev/Bessel coefficients (host only; no device needed)
 * ------------------------------------------------------------------------ */

/*
 * Number of terms M of the expansion exp(-i z x) = J_0(z) + 2 sum_{m>=1}
 * (-i)^m J_m(z) T_m(x) (paper, Sec. "Tight-binding propagation method",
 * Jacobi-Anger expansion): the smallest m > |z| with |J_m(z)| < tol, and at
 * least 3.  Terms m = 0..M-1 are kept.  0 < tol < 1, |z| <= 1e4.
 */
tbpm_status tbpm_num_terms(double z, double tol, int32_t *M);

/* J_0(z) .. J_{M-1}(z) into J[M] (host), by Miller's backward recurrence
 * normalised with J_0 + 2 sum_k J_2k = 1 (Abramowitz & Stegun 9.1.46, 9.12). */
tbpm_status tbpm_bessel_j(double z, int32_t M, double *J);

/* ------------------------------------------------------------------------
 * Propagation and DOS
 * ------------------------------------------------------------------------ */

/*
 * Propagate n_states initial states and record the DOS correlation
 * (paper, Eq. (eq:psi_t) and Eq. (eq:corr_dos)):
 *   psi(0) = psi0,  psi((k+1) dt) = P psi(k dt),  P = sum_{m<M} c_m T_m(H/f),
 *   c_0 = J_0(z), c_m = 2 (-i)^m J_m(z),  z = f dt,
 *   corr[k][s]  = <psi0_s | psi_s(k dt)>,   k = 0 .. n_steps-1,
 *   norm2[k][s] = ||psi_s(k dt)||^2.
 * The series is evaluated by Clenshaw's recurrence on the GPU.
 *
 *   psi0        device, [n_orb][n_states] complex128; read only.
 *   n_states    1 .. 64.
 *   n_steps     number of correlation samples N_t >= 1 (N_t - 1 time steps).
 *   dt          time step in hbar/eV (> 0); the paper uses dt = pi / f.
 *   rescale     f in eV (> 0); <= 0 selects the Gershgorin bound.  The
 *               spectrum of H must lie in [-f, f].
 *   bessel_tol  truncation threshold of the series (e.g. 1e-12), see tbpm_num_terms.
 *   prec        TBPM_FP64 or TBPM_FP32_MIXED.
 *   corr        device, [n_steps][n_states] complex128, written.
 *   norm2       device, [n_steps][n_states] double, written; may be NULL.
 *   ckpt_every  K > 0 to store checkpoints for tbpm_backward, else 0.
 *   ckpt        device, [max(0, (n_steps - 2) / K)][n_orb][n_states] complex128:
 *               ckpt[m-1] = psi(m K dt) for m K <= n_steps - 2 (TBPM_FP64 only).
 *   flags       TBPM_FLAG_ASYNC, TBPM_FLAG_NO_GRAPH.
 *   stream      hipStream_t or NULL.
 * Unless TBPM_FLAG_ASYNC is set, the call synchronises the stream and
 * returns TBPM_E_DIVERGED if some ||psi_s(k dt)||^2 / ||psi0_s||^2 leaves
 * [1 - 1e-3, 1 + 1e-3] or is not finite (H outside [-f, f]).
 * Calls on the same H must not overlap (they share its work buffers).
 */
tbpm_status tbpm_propagate(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps,
                           double dt, double rescale, double bessel_tol, tbpm_precision prec,
                           double *corr, double *norm2, int32_t ckpt_every, double *ckpt,
                           uint32_t flags, void *stream);

/*
 * tbpm_propagate for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same propagation and correlation, corr[k][s] = <psi0_s|psi_s(k dt)> and
 * norm2[k][s] = ||psi_s(k dt)||^2, with the same kernels in the plain launch
 * shape (one Clenshaw order per launch, the handle's configuration for prec;
 * the fused and staged shapes are not used), launched directly.
 *   Arguments as tbpm_propagate (no checkpoints, no flags); norm2 may be NULL.
 * Work memory: every work buffer lives in one fixed device array of 64 MiB
 * per device, reserved by the library when its code is loaded onto the
 * device and held until the process ends.  A call needs about
 * 4096 + (3 b + 16) n_orb S_pad + 32 n_orb bytes (b = 16 for TBPM_FP64,
 * 8 for TBPM_FP32_MIXED; S_pad = n_states rounded up to a power of two);
 * beyond 64 MiB it returns TBPM_E_ARG before any work is enqueued, and the
 * series may have at most 65 terms.  All calls on one device share that
 * array: calls that overlap on one device race (serialise them, e.g. on one
 * stream).  The call allocates nothing, copies nothing from the host and
 * never synchronises: it only enqueues kernels on 'stream' and returns, so
 * it performs no norm check (read norm2 to check).  The caller's buffers
 * must stay valid until the work has finished.
 */
tbpm_status tbpm_propagate_noalloc(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps,
                                   double dt, double rescale, double bessel_tol, tbpm_precision prec, double *corr,
                                   double *norm2, void *stream);

/*
 * Wave-function propagation with snapshots (the paper's usage section,
 * propagation of a wave packet; Sec. "Tight-binding propagation method",
 * Eq. (eq:psi_t)): propagate psi0 with the same series and time step as
 * tbpm_propagate and store psi(k dt) for every k in steps.
 *   steps   host, n_snap distinct step indices >= 0 (any order); step 0 is
 *           psi0 itself.  The propagation runs to max(steps).
 *   snaps   device, [n_snap][n_orb][n_states] complex128, written:
 *           snaps[q] = psi(steps[q] dt), orbitals in the caller's order.
 *   corr    device [max(steps)+1][n_states] complex128 receiving
 *           <psi0|psi(k dt)> as in tbpm_propagate, or NULL.
 *   prec    TBPM_FP64 or TBPM_FP32_MIXED (snapshots are stored in FP64).
 * Other arguments, errors and the norm check as for tbpm_propagate.  The
 * snapshot buffer is the caller's; the library keeps nothing of it.
 */
tbpm_status tbpm_propagate_snapshots(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, const int32_t *steps,
                                     int32_t n_snap, double dt, double rescale, double bessel_tol,
                                     tbpm_precision prec, double *snaps, double *corr, uint32_t flags,
                                     void *stream);

/*
 * Quasi-eigenstates (Sec. "Quasieigenstates", Eq. (quasi)): for each energy
 * E_j and state s,
 *   Psi_s(E_j) = sum_{k=-(n_steps-1)}^{n_steps-1} w_|k| e^{i E_j k dt} psi_s(k dt),
 * normalised to unit norm, where psi_s(t) propagates psi0_s with the series
 * of tbpm_propagate (negative times with the time step -dt) and w is the
 * window of tbpm_dos (Hann, or none).  Energies are in eV, the units of H.
 *   energies  host, n_energies values (1 .. 256)
 *   states    device, [n_energies][n_orb][n_states] complex128, written,
 *             orbitals in the caller's order
 *   norm2     device [n_energies][n_states] f64 receiving ||Psi_s(E_j)||^2
 *             before normalisation, or NULL.  A zero norm (an energy far
 *             outside the spectrum) leaves that state zero.
 * The library keeps n_energies * n_orb * (n_states padded to a power of 2)
 * complex128 accumulators.  Other arguments and errors as tbpm_propagate.
 */
tbpm_status tbpm_quasi_eigenstates(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps,
                                   double dt, double rescale, double bessel_tol, tbpm_precision prec,
                                   const double *energies, int32_t n_energies, tbpm_window win, double *states,
                                   double *norm2, uint32_t flags, void *stream);

/*
 * Optical conductivity by propagation (Sec. "Optical conductivity"; the
 * Fermi-Dirac operator by its Chebyshev series, Sec. "Tight-binding
 * propagation method").  With f(H) = 1/(exp(beta (H - mu)) + 1),
 *   psi1 = [1 - f(H)] J_beta psi0,   psi2 = f(H) psi0,
 * both propagated with the series of tbpm_propagate, and
 *   corr[k][s] = <psi2_s(k dt)| J_alpha |psi1_s(k dt)>,  k = 0 .. n_steps-1.
 *   j_alpha, j_beta  host, 2*nnz doubles: the current operators (complex,
 *             Hermitian; J = -i sum H_ij (r_j - r_i) c_i^+ c_j in units
 *             e = hbar = 1) as values on H's merged pattern, in the order of
 *             tbpm_hamiltonian_pattern; they may be the same array
 *   psi0      device, [n_orb][n_states] complex128 (caller's row order)
 *   n_states  1 .. 32 (both states are propagated as one block of 2 S)
 *   beta      1/(k_B T) in 1/eV (> 0), mu the chemical potential in eV
 *   fermi_tol truncation of the Fermi-Dirac series (last |a_k| kept >= tol),
 *             in (0, 1e-2); the series (coefficients of tbpm_fermi_cheb) is
 *             evaluated once, in FP64, on the block [J_beta psi0 | psi0], and
 *             psi1 = J_beta psi0 - f(H) J_beta psi0; prec applies to the
 *             propagation only
 *   corr      device, [n_steps][n_states] complex128, written
 * Other arguments as tbpm_propagate.  TBPM_E_ARG also when the series needs
 * more than 2^19 terms (beta times the rescale factor too large).
 */
tbpm_status tbpm_ac_corr(tbpm_hamiltonian *H, const double *j_alpha, const double *j_beta, const double *psi0,
                         int32_t n_states, int32_t n_steps, double dt, double rescale, double bessel_tol, double beta,
                         double mu, double fermi_tol, tbpm_precision prec, double *corr, uint32_t flags, void *stream);

/*
 * Moments of the Kubo-Bastin conductivity by the kernel polynomial method
 * (Sec. "Tight-binding propagation method", the DC conductivity tensor):
 *   mu_mn = (1/S) sum_s <r_s| v_alpha T_m(H/f) v_beta T_n(H/f) |r_s>,  m, n < M,
 * with no kernel factors (tbpm_kubo_bastin applies them).  With
 * L_m = T_m(H/f) v_alpha r and R_n = v_beta T_n(H/f) r the moments are the
 * matrix product L^H R, computed on the matrix cores; all M vectors L_m are
 * held in device memory (M x n_orb x S_pad x 16 bytes, S_pad the power of two
 * >= S, plus 128 vectors of R): TBPM_E_OOM if they do not fit.
 *   v_alpha, v_beta host, 2*nnz doubles: Hermitian operators (velocity or
 *             current; the sign cancels in sigma) as complex values on H's
 *             merged pattern (tbpm_hamiltonian_pattern order)
 *   psi0      device [n_orb][n_states] complex128 random vectors (unit norm
 *             estimates Tr/N), n_states 1 .. 64
 *   n_moments 2 .. 16384;  rescale f > 0 must bound the spectrum of H
 *             (<= 0: the Gershgorin bound); the moments are not checked
 *   mu        device [M][M] complex128, written: mu[n*M + m] = mu_mn
 *   timing_ms host [4] or NULL: milliseconds of the L recursion, the R
 *             recursion and the products, and the number of chunks the product's
 *             inner dimension is split into
 * Returns after the work has finished.
 */
tbpm_status tbpm_kpm_moments(tbpm_hamiltonian *H, const double *v_alpha, const double *v_beta, const double *psi0,
                             int32_t n_states, int32_t n_moments, double rescale, double *mu, double *timing_ms,
                             void *stream);

/*
 * Kubo-Bastin conductivity from the moments (Sec. "Tight-binding propagation
 * method", the DC conductivity tensor), units e = hbar = 1:
 *   sigma(mu_c) = 4/(pi A f^2) int dE~ f_FD(E~)/(1 - E~^2)^2 sum_{m,n} Gamma_nm(E~) g_m g_n mu_mn
 *                 / ((1 + delta_m0)(1 + delta_n0)),
 *   Gamma_nm = T_m(E~)(E~ - i n sin t) e^{i n t} + T_n(E~)(E~ + i m sin t) e^{-i m t},
 * E~ = cos t, g the Jackson kernel of M moments, f_FD the Fermi-Dirac
 * function at chemical potential mu_c (eV) and 1/k_B T = beta (1/eV).  The
 * integral is the midpoint rule on n_energy points uniform in t over
 * E = f E~ in [e_lo, e_hi] (a window holding the spectrum, strictly inside
 * (-f, f); outside the spectrum the integrand's delta-function factor
 * vanishes).  With unit-norm random vectors pass the area per orbital.
 *   mu        device [M][M] complex128 from tbpm_kpm_moments (M <= 4096)
 *   mus       device [n_mu] f64 chemical potentials (eV)
 *   energies  device [n_energy] f64, written: the grid E_k (eV, descending)
 *   weight    device [n_energy] f64, written: the real integrand times its
 *             quadrature weight at E_k (sum_k f_FD(E_k) weight_k is the integral)
 *   sigma     device [n_mu] f64, written (units e^2/hbar)
 */
tbpm_status tbpm_kubo_bastin(const double *mu, int32_t n_moments, double rescale, double e_lo, double e_hi,
                             int32_t n_energy, double beta, const double *mus, int32_t n_mu, double area,
                             double *energies, double *weight, double *sigma, void *stream);

/*
 * Haydock recursion (Sec. "Local density of states", the recursion method):
 * one Lanczos chain per column of psi0, all chains advanced together,
 *   l_0 = psi0_s / ||psi0_s||,  a_i = <l_i|H|l_i>,
 *   m_{i+1} = (H - a_i) l_i - b_i l_{i-1},  b_{i+1} = ||m_{i+1}||,
 *   l_{i+1} = m_{i+1} / b_{i+1}   (l_{-1} = 0),
 * so that <l_0|(z - H)^{-1}|l_0> is the continued fraction of
 * tbpm_haydock_ldos.  A unit vector on orbital i gives the LDOS of i.
 *   psi0      device, [n_orb][n_states] complex128 start vectors (caller's
 *             row order); a zero column gives zero coefficients
 *   n_states  1 .. 64;  n_iter  1 .. 2^24
 *   a, b      device, [n_iter][n_states] f64, written: a[i] = a_i and
 *             b[i] = b_{i+1}.  When b_{i+1} falls to 1e-11 times the
 *             Gershgorin bound of H or below, the chain has reached an
 *             invariant subspace: b_{i+1} is written as 0 and every later
 *             coefficient of that chain is 0.
 * Unscaled H (energies in eV), FP64.  Returns after the work has finished
 * (flags: TBPM_FLAG_NO_GRAPH launches every iteration directly).
 */
tbpm_status tbpm_haydock(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_iter, double *a,
                         double *b, uint32_t flags, void *stream);

/*
 * LDOS from Haydock coefficients: d(E) = -(1/pi) Im G_0(E + i eps) with
 *   G_0(z) = 1/(z - a_0 - b_1^2/(z - a_1 - b_2^2/( ... /(z - a_{n-1})))),
 * the continued fraction cut after n_iter levels (no terminator).
 *   a, b      device [n_iter][n_states] f64 as written by tbpm_haydock
 *   energies  device [n_e] f64 (eV), n_e * n_states <= 2^31;  eps > 0 the broadening (eV)
 *   ldos      device [n_e][n_states] f64, written (per eV)
 */
tbpm_status tbpm_haydock_ldos(const double *a, const double *b, int32_t n_iter, int32_t n_states,
                              const double *energies, int64_t n_e, double eps, double *ldos, void *stream);

/*
 * Chebyshev coefficients of the Fermi-Dirac function (Sec. "Tight-binding
 * propagation method": the expansion of a function of H by a discrete
 * Fourier sum over Chebyshev nodes), as tbpm_ac_corr uses them:
 *   f(H) = sum_{k<K} a[k] T_k(H / rescale),  f(x) = 1/(exp(beta (x - mu)) + 1),
 * kept up to the last |a[k]| >= tol.  Host call, no GPU.
 *   a    host, capacity cap doubles: the first min(cap, K) coefficients
 *        (cap = 0 and a = NULL query K)
 *   K    host, written: the number of coefficients
 * TBPM_E_ARG for beta <= 0, rescale <= 0, tol outside (0, 1e-2), or an
 * expansion longer than 2^19 terms.
 */
tbpm_status tbpm_fermi_cheb(double beta, double mu, double rescale, double tol, double *a, int32_t cap, int32_t *K);

/*
 * Real part of the optical conductivity (Eq. (AC)) from tbpm_ac_corr's
 * correlation averaged over the states, by a rectangle rule on t_k = k dt
 * with the window of tbpm_dos in place of e^{-Et}:
 *   sigma(w_j) = (e^{-beta w_j} - 1) / (w_j area) dt sum_k w_k sin(w_j t_k) 2 Im Cbar_k
 * on w_j = j pi / (n_steps dt), j = 0 .. n_steps-1 (sigma(0) = 0: the Drude
 * part is omitted).  Units e = hbar = 1: energies in eV, area in the square
 * of the length unit of the current operator.  The state average stands for
 * a trace: with unit-norm random states (which estimate Tr/N) pass the
 * sample's area divided by its number of orbitals, giving the conductivity
 * in units of e^2/hbar per spin.
 *   corr          device [n_steps][n_states] complex128
 *   omegas, sigma device [n_steps] f64, written
 */
tbpm_status tbpm_ac_cond(const double *corr, int32_t n_steps, int32_t n_states, double dt, double beta, double area,
                         tbpm_window win, double *omegas, double *sigma, void *stream);

/*
 * Imaginary part of the optical conductivity from its real part by the
 * Kramers-Kronig relation (Sec. "Optical conductivity"):
 *   Im sigma(w) = -(1/pi) P int_{-inf}^{inf} Re sigma(w') / (w' - w) dw',
 * on the uniform grid w_j = j dw, j = 0 .. n-1, that tbpm_ac_cond writes (the
 * spacing drops out).  Re sigma(-w) = Re sigma(w) (sigma(-w) = sigma(w)^* for
 * a real response); between grid points Re sigma is taken linear, and it
 * falls linearly to zero one spacing past the last point; the principal
 * value of that function is integrated exactly (closed-form weights per
 * grid point, a direct O(n^2) sum in FP64 with compensation, fixed order).
 * Like the real part it omits the Drude weight at w = 0.
 *   re_sigma  device [n] f64 (e.g. the sigma of tbpm_ac_cond)
 *   n         1 .. 2^17
 *   im_sigma  device [n] f64, written; must not alias re_sigma
 */
tbpm_status tbpm_ac_cond_imag(const double *re_sigma, int32_t n, double *im_sigma, void *stream);

/*
 * DOS from the correlations (paper, Eq. (dos_tbpm), with C(-t) = C(t)^*):
 *   Cbar_k = (1/S) sum_s corr[k][s],
 *   E_j = j pi / (N_t dt),  j = -N_t .. N_t - 1   (2 N_t energies),
 *   D(E_j) = dt/(2 pi) [w_0 Re Cbar_0 + 2 sum_{k=1}^{N_t-1} w_k Re(Cbar_k e^{i E_j k dt})].
 * corr device [n_steps][n_states] complex128; energies, dos device [2 n_steps].
 * The sum is direct (no FFT), in FP64 with compensated summation, in a
 * fixed order.
 */
tbpm_status tbpm_dos(const double *corr, int32_t n_steps, int32_t n_states, double dt, tbpm_window win,
                     double *energies, double *dos, void *stream);

/*
 * Adjoint of tbpm_dos: given grad_dos[j] = dL/dD(E_j) (device, [2 n_steps]),
 * writes grad_corr (device, [n_steps][n_states] complex128) such that
 * dL = Re sum_{k,s} conj(grad_corr[k][s]) d corr[k][s].
 */
tbpm_status tbpm_dos_backward(const double *grad_dos, int32_t n_steps, int32_t n_states, double dt,
                              tbpm_window win, double *grad_corr, void *stream);

/*
 * Gradient of a loss L(corr) with respect to the Hamiltonian, through the
 * propagation of tbpm_propagate (exact discrete adjoint of the Clenshaw
 * evaluation; f and dt fixed).
 *   grad_corr   device, [n_steps][n_states] complex128, with
 *               dL = Re sum conj(grad_corr) d corr  (PyTorch's convention).
 *   ckpt_every, ckpt  the checkpoints written by tbpm_propagate with the same
 *               psi0, n_steps, dt, rescale and bessel_tol (K > 0 required).
 *   grad_val    device, [2 * nnz] complex128 in the merged CSR order
 *               (tbpm_hamiltonian_pattern): G_pq with dL = Re sum conj(G_pq) dH_pq.
 *   grad_onsite device, [n_orb] double: dL/d eps_i.
 * Both gradients are summed over the states.  FP64 only.  Device memory of
 * about K * (M - 1) + 8 state-sized vectors is used for the segment replay.
 */
tbpm_status tbpm_backward(tbpm_hamiltonian *H, const double *psi0, int32_t n_states, int32_t n_steps,
                          double dt, double rescale, double bessel_tol, const double *grad_corr,
                          int32_t ckpt_every, const double *ckpt, double *grad_val,
                          double *grad_onsite, void *stream);

/* ------------------------------------------------------------------------
 * Batched propagation of several Hamiltonians of uneven size
 * ------------------------------------------------------------------------ */

/*
 * Concatenate n_ham Hamiltonians into one block-diagonal device operator
 * so that every Chebyshev pass of all of them is one kernel launch.  The
 * handles must stay alive while the batch is used; later set_values calls
 * on them are not seen by the batch.
 */
tbpm_status tbpm_batch_create(tbpm_hamiltonian *const *Hs, int32_t n_ham, tbpm_batch **out);
tbpm_status tbpm_batch_destroy(tbpm_batch *B);

/*
 * tbpm_propagate for every member of the batch at once (paper: samples and
 * Hamiltonians are independent, Sec. "TBPM" of the parallelisation part).
 *   psi0[i], corr[i], norm2[i]: host arrays of n_ham device pointers, laid
 *   out as in tbpm_propagate for member i (norm2 may be NULL, or contain NULLs).
 *   dt[i], rescale[i]: host arrays; each member has its own z_i = f_i dt_i
 *   and coefficient set.  n_states is common.  Flags as tbpm_propagate; the
 *   norm check covers every member.
 */
tbpm_status tbpm_propagate_batched(tbpm_batch *B, const double *const *psi0, int32_t n_states,
                                   int32_t n_steps, const double *dt, const double *rescale,
                                   double bessel_tol, tbpm_precision prec, double *const *corr,
                                   double *const *norm2, uint32_t flags, void *stream);

/* ------------------------------------------------------------------------
 * Launch configuration and autotuning
 * ------------------------------------------------------------------------ */

/*
 * Launch shape of the Chebyshev pass kernels:
 *   wg_chunks   row chunks handled by one workgroup (1, 2, 4, 8, 16 or 32);
 *               one chunk is 256 state elements
 *   xcd_remap   order in which the 8 XCDs take the tiles.  0: workgroup b
 *               takes tile b (consecutive tiles on different XCDs);
 *               1: each XCD a contiguous range of tiles; 2 .. 6: runs of
 *               2^xcd_remap (4 .. 64) consecutive tiles per XCD, the runs
 *               dealt to the XCDs in turn
 *   nontemporal 1: stream the read-once vectors with non-temporal hints
 *   unroll      elements each thread handles at once (1 or 2)
 *   staged      1 .. 6: each workgroup first copies the distinct rows of x
 *               that its tile reads into LDS and gathers from there (pays off
 *               for rows with many stored elements); the value t is the LDS
 *               tier, as for fused below: a tile's staged rows use at most
 *               1/(t+2) of a CU's 160 KiB.  wg_chunks and unroll are then
 *               unused.  0: gather from global memory
 *   vec         states of a row each thread holds (1, 2 or 4; capped by the
 *               padded state count)
 *   fused       1 .. 6: evaluate two Clenshaw orders per launch: each tile
 *               stages its rows and their two-hop neighbourhood in LDS and
 *               computes the first order on its rows and their neighbours,
 *               the second on its own rows.  The value t is the LDS tier: a
 *               tile uses at most 1/(t+2) of a CU's 160 KiB (bigger tiles and
 *               smaller halos, or more resident workgroups).  Two
 *               extra state-sized work vectors are allocated; staged and
 *               wg_chunks are unused and unroll applies to the orders left
 *               unpaired.  When only the correlation is taken from each
 *               psi(k dt) (no checkpoints, snapshots, quasi-eigenstates or
 *               current correlation) the last middle order and the final
 *               order share a launch, and with an even number of middle
 *               orders the first order runs alone; otherwise the final order
 *               runs alone, and a middle one when their count is odd.  Falls
 *               back to the plain shape when the series has fewer than 4
 *               terms or no tile fits.  0: one order per launch.
 */
typedef struct {
    int32_t wg_chunks;
    int32_t xcd_remap;
    int32_t nontemporal;
    int32_t unroll;
    int32_t staged;
    int32_t vec;
    int32_t fused;
} tbpm_launch_config;

/* Each handle keeps one launch configuration per precision. */
tbpm_status tbpm_get_launch_config(const tbpm_hamiltonian *H, tbpm_precision prec, tbpm_launch_config *cfg);
tbpm_status tbpm_set_launch_config(tbpm_hamiltonian *H, tbpm_precision prec, const tbpm_launch_config *cfg);
tbpm_status tbpm_batch_set_launch_config(tbpm_batch *B, tbpm_precision prec, const tbpm_launch_config *cfg);
tbpm_status tbpm_batch_get_launch_config(const tbpm_batch *B, tbpm_precision prec, tbpm_launch_config *cfg);

/*
 * Autotune the launch configuration of H (or of a batch) for n_states and
 * prec by timing every candidate on three Chebyshev time steps of scratch
 * states, then the three fastest on eight, on 'stream' (synchronises).  The
 * best configuration is stored in the handle for that precision and returned
 * in *best (may be NULL); its mean step time in ms over the eight steps in
 * *best_ms (may be NULL).  Candidates with more elements
 * per thread than chunks per workgroup are skipped (they idle threads).
 */
tbpm_status tbpm_autotune(tbpm_hamiltonian *H, int32_t n_states, tbpm_precision prec,
                          tbpm_launch_config *best, double *best_ms, void *stream);
tbpm_status tbpm_batch_autotune(tbpm_batch *B, int32_t n_states, tbpm_precision prec,
                                tbpm_launch_config *best, double *best_ms, void *stream);

/* ------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------ */

/* Plain streaming copy of 'bytes' (multiple of 16) from src to dst (device),
 * used to calibrate achievable HBM bandwidth and the profiler's byte counters. */
tbpm_status tbpm_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/*
 * Enqueue n_launch back-to-back launches of the interior Clenshaw pass kernel
 * (b_j = c_j v + 2 H~ b_{j+1} - b_{j+2}), or of the two-order launch when the
 * fused shape is configured, on H's work buffers, for timing the dominant
 * kernel in isolation.  The launches chain as in a time step: each reads what
 * the one before wrote, and consecutive launches walk the tiles in opposite
 * directions.  A tbpm_propagate call with the same n_states and prec must
 * have been made on H first (it sizes and fills the buffers); the buffers'
 * contents stay bounded but are overwritten.
 */
tbpm_status tbpm_bench_pass(tbpm_hamiltonian *H, int32_t n_states, tbpm_precision prec, int32_t n_launch,
                            void *stream);

/* Message of the last error on this thread ("" if none). */
const char *tbpm_last_error(void);

/* Library version string. */
const char *tbpm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TBPM_H */
