"""TBPM oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct FP64 CPU implementation of the TBPM DOS
path of the paper (Sec. "Tight-binding propagation method" and Sec.
"Density of states", Eq. (eq:psi_t), Eq. (eq:corr_dos), Eq. (dos_tbpm)).
It checks the HIP library and shares no code with it.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the product path never does.

Pieces:
  * :func:`bessel_j` -- J_m(z) by the power series, summed in 60+-digit
    decimal arithmetic (Abramowitz & Stegun 9.1.10);
  * :func:`n_terms` -- truncation of the Chebyshev/Bessel series;
  * :func:`propagate` -- the paper's modified Chebyshev recurrence (plain C,
    ``tbpm_oracle.c``), recording C_k = <phi0|psi_k> and ||psi_k||^2;
  * :func:`psi_t` -- the same propagation, returning psi at chosen steps
    (wave-packet snapshots);
  * :func:`quasi_eigenstates` -- windowed Fourier transform of psi(t) over
    positive and negative times at chosen energies;
  * :func:`fermi_coeffs`, :func:`apply_cheb` -- Chebyshev series of the
    Fermi-Dirac operator (forward recurrence);
  * :func:`ac_corr`, :func:`ac_cond` -- optical-conductivity correlation and
    its windowed sine transform (Kubo formula);
  * :func:`ac_cond_imag` -- the imaginary part of the optical conductivity
    from the real part by the Kramers-Kronig relation;
  * :func:`haydock`, :func:`haydock_ldos` -- the Lanczos recursion of the
    Haydock method and the continued fraction of the Green's function;
  * :func:`jackson`, :func:`kpm_moments`, :func:`kubo_bastin` -- the
    Kubo-Bastin conductivity tensor by the kernel polynomial method;
  * :func:`dos` -- Hann-windowed Fourier transform of the sample-averaged
    correlation, summed directly (no FFT);
  * :func:`dos_adjoint`, :func:`backward` -- the discrete adjoints used to
    check gradients.

Readings of the paper that the oracle fixes (the paper is silent on them):
  * the Chebyshev series keeps terms m = 0..M-1 where M is the smallest
    m > z with |J_m(z)| < tol, and at least 3 terms;
  * the Hann window is w_k = (1 + cos(pi k / N_t)) / 2 over the N_t samples;
  * DOS grid E_j = j pi / (N_t dt), j = -N_t .. N_t - 1.
Every function here is pinned by the ``-m "not gpu"`` tests against exact
diagonalisation, closed forms and identities.
"""
from __future__ import annotations

import ctypes
import math
import os
from decimal import Decimal, localcontext

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_propagate.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                                         P, ctypes.c_int32, ctypes.c_int32, P, P, P]
        lib.oracle_propagate.restype = ctypes.c_int
        lib.oracle_backward.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                                        P, ctypes.c_int32, ctypes.c_int32, P, P, P, P]
        lib.oracle_backward.restype = ctypes.c_int
        lib.oracle_psi_t.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                                     P, ctypes.c_int32, P, ctypes.c_int32, P, P]
        lib.oracle_psi_t.restype = ctypes.c_int
        lib.oracle_apply_cheb.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_int32, P,
                                          ctypes.c_int32, P, P]
        lib.oracle_apply_cheb.restype = ctypes.c_int
        lib.oracle_ac_corr.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_int32, P, P,
                                       ctypes.c_int32, ctypes.c_int32, P, P, P]
        lib.oracle_ac_corr.restype = ctypes.c_int
        _lib = lib
    return _lib


# ----------------------------------------------------------------------------
# Bessel coefficients (Jacobi-Anger expansion of exp(-i z x))
# ----------------------------------------------------------------------------

def bessel_j(m: int, z: float) -> float:
    """J_m(z) for integer m >= 0 from the power series
    J_m(z) = sum_k (-1)^k (z/2)^(2k+m) / (k! (k+m)!), summed in decimal
    arithmetic with enough digits to absorb the cancellation for large z."""
    if m < 0:
        raise ValueError("order must be >= 0")
    if z == 0.0:
        return 1.0 if m == 0 else 0.0
    digits = 60 + int(abs(z) * 0.45)
    with localcontext() as ctx:
        ctx.prec = digits
        x = Decimal(z) / 2
        x2 = x * x
        term = x ** m / Decimal(math.factorial(m))
        total = term
        k = 0
        tiny = Decimal(10) ** (-45)
        while True:
            k += 1
            term = -term * x2 / (k * (k + m))
            total += term
            if k > abs(x) and abs(term) < tiny:
                break
        return float(total)


def n_terms(z: float, tol: float = 1e-12) -> int:
    """Number M of Chebyshev terms kept: the smallest m > |z| with
    |J_m(z)| < tol (terms m = 0..M-1 are used), and at least 3."""
    m = int(math.floor(abs(z))) + 1
    while abs(bessel_j(m, z)) >= tol:
        m += 1
    return max(3, m)


def gershgorin(row_ptr, val, onsite) -> float:
    """Gershgorin bound max_i (|eps_i| + sum_j |H_ij|) of the spectral radius."""
    n = onsite.shape[0]
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    radius = np.zeros(n)
    np.add.at(radius, rows, np.abs(val))
    return float(np.max(np.abs(onsite) + radius))


def _prep(row_ptr, col, val, onsite, psi0):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.complex128)
    onsite = np.ascontiguousarray(onsite, dtype=np.float64)
    psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
    if psi0.ndim == 1:
        psi0 = psi0[:, None].copy()
    return row_ptr, col, val, onsite, psi0


def _scale_and_coeffs(row_ptr, val, onsite, dt, rescale, tol):
    f = float(rescale) if rescale > 0 else gershgorin(row_ptr, val, onsite)
    z = f * dt
    M = n_terms(z, tol)
    J = np.array([bessel_j(m, z) for m in range(M)], dtype=np.float64)
    return f, M, J


def propagate(row_ptr, col, val, onsite, psi0, n_steps: int, dt: float, rescale: float,
              tol: float = 1e-12):
    """C_k = <phi0|psi_k> and ||psi_k||^2 for k = 0..n_steps-1 (paper, Eq. eq:psi_t).

    Returns (corr [n_steps, S] complex128, norm2 [n_steps, S] float64, info dict).
    """
    row_ptr, col, val, onsite, psi0 = _prep(row_ptr, col, val, onsite, psi0)
    n, S = psi0.shape
    f, M, J = _scale_and_coeffs(row_ptr, val, onsite, dt, rescale, tol)
    corr = np.zeros((n_steps, S), dtype=np.complex128)
    norm2 = np.zeros((n_steps, S), dtype=np.float64)
    rc = _load().oracle_propagate(n, row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data,
                                  onsite.ctypes.data, f, S, psi0.ctypes.data, n_steps, M,
                                  J.ctypes.data, corr.ctypes.data, norm2.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_propagate failed")
    return corr, norm2, {"rescale": f, "z": f * dt, "M": M, "J": J}


def psi_t(row_ptr, col, val, onsite, psi0, steps, dt: float, rescale: float, tol: float = 1e-12):
    """psi(k dt) for each k in ``steps`` (the wave-function propagation of the
    paper's usage section, same series as :func:`propagate`).

    Returns snapshots [len(steps), n, S] complex128 and the info dict.
    """
    row_ptr, col, val, onsite, psi0 = _prep(row_ptr, col, val, onsite, psi0)
    n, S = psi0.shape
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    f, M, J = _scale_and_coeffs(row_ptr, val, onsite, dt, rescale, tol)
    snaps = np.zeros((steps.shape[0], n, S), dtype=np.complex128)
    rc = _load().oracle_psi_t(n, row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data, onsite.ctypes.data, f, S,
                              psi0.ctypes.data, steps.shape[0], steps.ctypes.data, M, J.ctypes.data,
                              snaps.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_psi_t failed (negative step or allocation failure)")
    return snaps, {"rescale": f, "z": f * dt, "M": M, "J": J}


def quasi_eigenstates(row_ptr, col, val, onsite, psi0, n_steps: int, dt: float, rescale: float, energies_ev,
                      tol: float = 1e-12, kind: str = "hann"):
    """Quasi-eigenstates (paper, Sec. "Quasieigenstates", Eq. (quasi)): the
    windowed inverse Fourier transform of psi(t) over positive and negative
    times,
        Psi(E) = sum_{k=-(N_t-1)}^{N_t-1} w_|k| e^{i E k dt} psi(k dt),
    with psi(-k dt) propagated with the time step -dt, normalised to unit norm
    per energy and state.

    Returns (states [n_E, n, S] complex128, norm2 [n_E, S] = ||Psi(E)||^2
    before normalisation).
    """
    row_ptr, col, val, onsite, psi0 = _prep(row_ptr, col, val, onsite, psi0)
    n, S = psi0.shape
    steps = np.arange(n_steps)
    fwd, _ = psi_t(row_ptr, col, val, onsite, psi0, steps, dt, rescale, tol)
    bwd, _ = psi_t(row_ptr, col, val, onsite, psi0, steps, -dt, rescale, tol)
    w = window(n_steps, kind)
    e = np.atleast_1d(np.asarray(energies_ev, dtype=np.float64))
    out = np.zeros((e.shape[0], n, S), dtype=np.complex128)
    norm2 = np.zeros((e.shape[0], S))
    for j in range(e.shape[0]):
        ph = w * np.exp(1j * e[j] * steps * dt)
        acc = np.tensordot(ph, fwd, axes=(0, 0)) + np.tensordot(np.conj(ph[1:]), bwd[1:], axes=(0, 0))
        norm2[j] = np.sum(np.abs(acc) ** 2, axis=0)
        out[j] = acc / np.sqrt(norm2[j])
    return out, norm2


def fermi(x, beta: float, mu: float):
    """Fermi-Dirac occupation 1 / (exp(beta (x - mu)) + 1), written with tanh
    so that large |beta (x - mu)| does not overflow."""
    return 0.5 * (1.0 - np.tanh(0.5 * beta * (np.asarray(x, dtype=np.float64) - mu)))


def fermi_coeffs(beta: float, mu: float, rescale: float, tol: float = 1e-14, n_max: int = 1 << 16) -> np.ndarray:
    """Chebyshev coefficients a_k with f(H) = sum_k a_k T_k(H/rescale) for the
    Fermi-Dirac operator (Sec. "Tight-binding propagation method",
    Eq. (ck_coef) evaluated as the discrete Fourier sum the paper gives:
    c_k = Re[(2/N) sum_n g(cos(2 pi n/N)) e^{i 2 pi n k/N}], a_0 = c_0/2,
    a_k = c_k), for g(x) = f(rescale * x).  Kept up to the last |a_k| >= tol."""
    n = 1024
    while True:
        theta = 2.0 * np.pi * np.arange(n) / n
        g = fermi(rescale * np.cos(theta), beta, mu)
        c = np.real(np.fft.ifft(g) * n) * 2.0 / n  # sum_n g_n e^{+i 2 pi n k / N}
        a = c[: n // 2].copy()
        a[0] *= 0.5
        big = np.flatnonzero(np.abs(a) >= tol)
        K = int(big[-1]) + 1 if big.size else 1
        if K < n // 8 or n >= n_max:
            return a[:K]
        n *= 2


def apply_cheb(row_ptr, col, val, onsite, rescale: float, coeffs, psi):
    """sum_k coeffs[k] T_k(H/rescale) psi (plain forward recurrence, C)."""
    row_ptr, col, val, onsite, psi = _prep(row_ptr, col, val, onsite, psi)
    n, S = psi.shape
    a = np.ascontiguousarray(coeffs, dtype=np.float64)
    out = np.zeros_like(psi)
    rc = _load().oracle_apply_cheb(n, row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data, onsite.ctypes.data,
                                   float(rescale), S, psi.ctypes.data, a.shape[0], a.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_apply_cheb failed")
    return out


def _sparse_apply(row_ptr, col, vals, psi):
    n = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    out = np.zeros_like(psi)
    np.add.at(out, rows, vals[:, None] * psi[col])
    return out


def ac_corr(row_ptr, col, val, onsite, j_alpha, j_beta, psi0, n_steps: int, dt: float, rescale: float,
            beta: float, mu: float, tol: float = 1e-12, fermi_tol: float = 1e-14):
    """Optical-conductivity correlation (Sec. "Optical conductivity"):
    psi1 = [1 - f(H)] J_beta psi0, psi2 = f(H) psi0, both propagated, and
    C_k = <psi2(k dt)| J_alpha |psi1(k dt)>.  J_alpha, J_beta: values on the
    CSR pattern of H.  Returns (corr [n_steps, S], psi1(0), psi2(0))."""
    row_ptr, col, val, onsite, psi0 = _prep(row_ptr, col, val, onsite, psi0)
    n, S = psi0.shape
    ja = np.ascontiguousarray(j_alpha, dtype=np.complex128)
    jb = np.ascontiguousarray(j_beta, dtype=np.complex128)
    f, M, J = _scale_and_coeffs(row_ptr, val, onsite, dt, rescale, tol)
    a = fermi_coeffs(beta, mu, f, fermi_tol)
    one_minus = -a.copy()
    one_minus[0] += 1.0
    psi2 = apply_cheb(row_ptr, col, val, onsite, f, a, psi0)
    psi1 = apply_cheb(row_ptr, col, val, onsite, f, one_minus, _sparse_apply(row_ptr, col, jb, psi0))
    psi1 = np.ascontiguousarray(psi1)
    psi2 = np.ascontiguousarray(psi2)
    corr = np.zeros((n_steps, S), dtype=np.complex128)
    rc = _load().oracle_ac_corr(n, row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data, onsite.ctypes.data, f, S,
                                psi1.ctypes.data, psi2.ctypes.data, n_steps, M, J.ctypes.data, ja.ctypes.data,
                                corr.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_ac_corr failed")
    return corr, psi1, psi2


def ac_cond(corr, dt: float, beta: float, area: float, kind: str = "hann"):
    """Real part of the optical conductivity (Sec. "Optical conductivity",
    Eq. (AC)) from the state-averaged correlation, by a rectangle rule on
    t_k = k dt with the DOS window in place of e^{-Et}:
        sigma(w_j) = (e^{-beta w_j} - 1) / (w_j A) * dt * sum_k w_k sin(w_j t_k) 2 Im Cbar_k,
    on w_j = j pi / (N_t dt), j = 0 .. N_t-1 (sigma(0) = 0: the Drude part is
    omitted).  Units e = hbar = 1 (energies in eV, lengths in A).  With
    unit-norm random states (an estimate of Tr/N) ``area`` is the sample's
    area per orbital."""
    corr = np.asarray(corr)
    if corr.ndim == 1:
        corr = corr[:, None]
    nt = corr.shape[0]
    cbar = corr.mean(axis=1)
    w = window(nt, kind)
    tk = np.arange(nt) * dt
    omega = np.arange(nt) * np.pi / (nt * dt)
    sigma = np.zeros(nt)
    for j in range(1, nt):
        s = np.sum(w * np.sin(omega[j] * tk) * 2.0 * np.imag(cbar)) * dt
        sigma[j] = (np.exp(-beta * omega[j]) - 1.0) / (omega[j] * area) * s
    return omega, sigma


def ac_cond_imag(re_sigma):
    """Imaginary part of the optical conductivity by the Kramers-Kronig
    relation (Sec. "Optical conductivity"):
        Im sigma(w) = -(1/pi) P int_{-inf}^{inf} Re sigma(w') / (w' - w) dw',
    on the uniform grid w_k = k dw of ``re_sigma`` (the grid of ac_cond;
    the spacing cancels).  Readings: Re sigma(-w) = Re sigma(w), since
    sigma(-w) = sigma(w)^* for a real response; Re sigma is piecewise linear
    between grid points and falls linearly to zero one spacing past the last
    one.  The principal value is the exact integral of that function,
    segment by segment over the whole line: on a segment [x0, x1] with
    Re sigma = y(x) linear,
        int y(x)/(x - w) dx = y(w) (ln|x1 - w| - ln|x0 - w|) + (y1 - y0),
    where y(w) extends the segment's line; at w = x0 or x1 the logarithm of
    zero is left out, since the two segments that meet at w contribute it
    with opposite signs and the same y(w)."""
    y = np.asarray(re_sigma, dtype=np.float64)
    n = y.shape[0]
    # nodes on the whole line in units of the spacing: -n .. n, value 0 at +-n
    xs = np.arange(-n, n + 1, dtype=np.float64)
    ys = np.concatenate([[0.0], y[:0:-1], y, [0.0]])
    x0, x1, y0, y1 = xs[:-1], xs[1:], ys[:-1], ys[1:]
    slope = y1 - y0  # segments have unit length
    out = np.zeros(n)
    for k in range(n):
        w = float(k)
        yw = y0 + slope * (w - x0)
        d1 = np.abs(x1 - w)
        d0 = np.abs(x0 - w)
        l1 = np.where(d1 > 0, np.log(np.where(d1 > 0, d1, 1.0)), 0.0)
        l0 = np.where(d0 > 0, np.log(np.where(d0 > 0, d0, 1.0)), 0.0)
        out[k] = -np.sum(yw * (l1 - l0) + slope) / np.pi
    return out


def haydock(row_ptr, col, val, onsite, psi0, n_iter: int, breakdown: float = 1e-11):
    """Lanczos recursion of the Haydock method (Sec. "Local density of
    states", the recursion method), one chain per column of psi0:
        l_0 = psi0 / ||psi0||,  l_{-1} = 0,
        a_i = <l_i|H|l_i>,
        m_{i+1} = (H - a_i) l_i - b_i l_{i-1},
        b_{i+1} = ||m_{i+1}||,  l_{i+1} = m_{i+1} / b_{i+1}.
    Returns (a [n_iter, S], b [n_iter, S]) with b[i] = b_{i+1}.  A chain whose
    b_{i+1} falls to ``breakdown`` times the Gershgorin bound or below has
    reached an invariant subspace: b_{i+1} is set to 0 and the chain stays
    zero (its continued fraction ends there).  The sparse product is SciPy's
    CSR matrix-vector product."""
    import scipy.sparse as sp

    row_ptr, col, val, onsite, psi0 = _prep(row_ptr, col, val, onsite, psi0)
    n, S = psi0.shape
    h = sp.csr_matrix((val, col, row_ptr), shape=(n, n)) + sp.diags(onsite)
    thr = breakdown * gershgorin(row_ptr, val, onsite)
    a = np.zeros((n_iter, S))
    b = np.zeros((n_iter, S))
    for s in range(S):
        nrm = np.linalg.norm(psi0[:, s])
        if nrm == 0.0:
            continue
        l_prev = np.zeros(n, dtype=np.complex128)
        l_cur = psi0[:, s] / nrm
        b_cur = 0.0
        for i in range(n_iter):
            hl = h @ l_cur
            a[i, s] = np.real(np.vdot(l_cur, hl))
            m = hl - a[i, s] * l_cur - b_cur * l_prev
            b_next = np.linalg.norm(m)
            if b_next <= thr:
                break
            b[i, s] = b_next
            l_prev, l_cur, b_cur = l_cur, m / b_next, b_next
    return a, b


def haydock_ldos(a, b, energies_ev, eps: float):
    """d(E) = -(1/pi) Im G_0(E + i eps) with the continued fraction
    G_0(z) = 1/(z - a_0 - b_1^2/(z - a_1 - b_2^2/(... /(z - a_{n-1})))),
    evaluated from the deepest level up (a zero terminator).  Returns
    [n_E, S]."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    n, S = a.shape
    out = np.zeros((len(energies_ev), S))
    for j, e in enumerate(energies_ev):
        z = complex(e, eps)
        for s in range(S):
            t = z - a[n - 1, s]
            for i in range(n - 2, -1, -1):
                t = z - a[i, s] - b[i, s] ** 2 / t
            out[j, s] = -(1.0 / t).imag / math.pi
    return out


def jackson(n_moments: int) -> np.ndarray:
    """Jackson kernel g_m, m = 0..N-1, for N moments (the closed form of the
    kernel polynomial method):
    g_m = [(N - m + 1) cos(pi m/(N+1)) + sin(pi m/(N+1)) cot(pi/(N+1))]/(N+1)."""
    N = n_moments
    m = np.arange(N)
    q = math.pi / (N + 1)
    return ((N - m + 1) * np.cos(q * m) + np.sin(q * m) / math.tan(q)) / (N + 1)


def kpm_moments(row_ptr, col, val, onsite, v_alpha, v_beta, psi0, n_moments: int, rescale: float):
    """mu[m, n] = (1/S) sum_s <r_s| v_alpha T_m(H~) v_beta T_n(H~) |r_s>,
    H~ = H/rescale, m, n < n_moments (Sec. "Tight-binding propagation method",
    the Kubo-Bastin formula; no kernel factors).  v_alpha, v_beta: values on
    the CSR pattern of H (Hermitian).  With L_m = T_m(H~) v_alpha r and
    R_n = v_beta T_n(H~) r, mu = L^H R, a matrix product."""
    import scipy.sparse as sp

    row_ptr, col, val, onsite, psi0 = _prep(row_ptr, col, val, onsite, psi0)
    n, S = psi0.shape
    ht = (sp.csr_matrix((val, col, row_ptr), shape=(n, n)) + sp.diags(onsite)) / rescale
    va = sp.csr_matrix((np.asarray(v_alpha, dtype=np.complex128), col, row_ptr), shape=(n, n))
    vb = sp.csr_matrix((np.asarray(v_beta, dtype=np.complex128), col, row_ptr), shape=(n, n))
    M = n_moments
    mu = np.zeros((M, M), dtype=np.complex128)
    for s in range(S):
        r = psi0[:, s]
        L = np.zeros((n, M), dtype=np.complex128)
        R = np.zeros((n, M), dtype=np.complex128)
        t_prev, t_cur = None, va @ r
        for m in range(M):  # T_0 = 1, T_1 = x, T_{m+1} = 2 x T_m - T_{m-1}
            L[:, m] = t_cur
            t_next = ht @ t_cur if m == 0 else 2.0 * (ht @ t_cur) - t_prev
            t_prev, t_cur = t_cur, t_next
        t_prev, t_cur = None, r.copy()
        for m in range(M):
            R[:, m] = vb @ t_cur
            t_next = ht @ t_cur if m == 0 else 2.0 * (ht @ t_cur) - t_prev
            t_prev, t_cur = t_cur, t_next
        mu += L.conj().T @ R
    return mu / S


def kubo_bastin(mu, rescale: float, e_lo: float, e_hi: float, n_energy: int, beta: float, mus, area: float):
    """sigma_ab(mu_c, T) of the Kubo-Bastin formula by the kernel polynomial
    method (Sec. "Tight-binding propagation method", DC conductivity tensor),
    units e = hbar = 1:
        sigma = 4/(pi A) (4/dE^2) int dE~ f(E~)/(1 - E~^2)^2 sum_{m,n} Gamma_nm(E~) mu~_nm
    with dE = 2 rescale, mu~_nm = g_m g_n mu_mn / ((1 + d_n0)(1 + d_m0)) (Jackson
    g), E~ = cos(theta),
        Gamma_nm = T_m(E~)(E~ - i n sin theta) e^{i n theta}
                 + T_n(E~)(E~ + i m sin theta) e^{-i m theta},
    f the Fermi-Dirac function at chemical potential mu_c (eV) and 1/k_B T =
    beta (1/eV).  The integral is the midpoint rule in theta over
    E~ in [e_lo, e_hi]/rescale (the window holding the spectrum; outside it
    the delta-function factor of the integrand vanishes), dE~ = sin theta
    dtheta.  mu: [M, M] state averages of kpm_moments, so ``area`` is the
    area per orbital.  Returns the real part for each mu_c."""
    mu = np.asarray(mu, dtype=np.complex128)
    M = mu.shape[0]
    g = jackson(M)
    w = g / np.where(np.arange(M) == 0, 2.0, 1.0)
    mut = w[:, None] * w[None, :] * mu
    th_hi = math.acos(e_lo / rescale)
    th_lo = math.acos(e_hi / rescale)
    dth = (th_hi - th_lo) / n_energy
    m = np.arange(M)
    acc = np.zeros(len(mus))
    for k in range(n_energy):
        th = th_lo + (k + 0.5) * dth
        x, sn = math.cos(th), math.sin(th)
        tm = np.cos(m * th)
        gam = (tm[:, None] * ((x - 1j * m[None, :] * sn) * np.exp(1j * m[None, :] * th))
               + tm[None, :] * ((x + 1j * m[:, None] * sn) * np.exp(-1j * m[:, None] * th)))
        # gam[m, n] = Gamma_nm; the sum runs over both indices
        val = np.sum(gam * mut).real / (1.0 - x * x) ** 2
        e = x * rescale
        fd = fermi(e, beta, np.asarray(mus, dtype=np.float64))
        acc += fd * val * sn * dth
    return 4.0 / (math.pi * area) / rescale ** 2 * acc


def energies(n_steps: int, dt: float) -> np.ndarray:
    """DOS grid E_j = j pi / (N_t dt), j = -N_t .. N_t-1."""
    j = np.arange(-n_steps, n_steps)
    return j * np.pi / (n_steps * dt)


def window(n_steps: int, kind: str = "hann") -> np.ndarray:
    k = np.arange(n_steps)
    if kind == "hann":
        return 0.5 * (1.0 + np.cos(np.pi * k / n_steps))
    if kind == "none":
        return np.ones(n_steps)
    raise ValueError(kind)


def dos(corr, dt: float, kind: str = "hann"):
    """D(E) = (1/S) sum_p (1/2pi) int e^{iEt} C_p(t) dt  (paper, Eq. dos_tbpm).

    Using C(-t) = conj C(t), the integral over the sampled times t_k = k dt is
    D(E_j) = dt/(2 pi) [w_0 Re Cbar_0 + 2 sum_{k>=1} w_k Re(Cbar_k e^{i E_j t_k})].
    Summed directly over k for every energy (no FFT).
    """
    corr = np.asarray(corr, dtype=np.complex128)
    if corr.ndim == 1:
        corr = corr[:, None]
    n_steps = corr.shape[0]
    cbar = corr.mean(axis=1)
    w = window(n_steps, kind)
    E = energies(n_steps, dt)
    t = np.arange(n_steps) * dt
    out = np.empty(E.shape[0])
    for a in range(0, E.shape[0], 256):
        ph = np.exp(1j * np.outer(E[a:a + 256], t))
        terms = (w * cbar)[None, :] * ph
        out[a:a + 256] = w[0] * cbar[0].real + 2.0 * terms[:, 1:].real.sum(axis=1)
    return E, out * dt / (2.0 * np.pi)


def dos_adjoint(gdos, n_steps: int, n_states: int, dt: float, kind: str = "hann"):
    """Adjoint of :func:`dos` with respect to the per-state correlations.

    Given gdos_j = dL/dD_j, returns G[k, s] with dL = Re sum conj(G) dC.
    From D_j above: dD_j/dRe C_k = (dt/pi) w_k cos(E_j t_k)/S,
    dD_j/dIm C_k = -(dt/pi) w_k sin(E_j t_k)/S for k >= 1, and only Re C_0
    enters with weight dt/(2 pi) w_0 / S.
    """
    gdos = np.asarray(gdos, dtype=np.float64)
    w = window(n_steps, kind)
    E = energies(n_steps, dt)
    t = np.arange(n_steps) * dt
    g = np.zeros(n_steps, dtype=np.complex128)
    for k in range(n_steps):
        s = np.sum(gdos * np.exp(-1j * E * t[k]))
        g[k] = (dt / np.pi) * w[k] * s if k > 0 else (dt / (2 * np.pi)) * w[0] * s.real
    return np.repeat((g / n_states)[:, None], n_states, axis=1)


def backward(row_ptr, col, val, onsite, psi0, n_steps: int, dt: float, rescale: float,
             gcorr, tol: float = 1e-12):
    """Gradient of L through C_k (dL = Re sum conj(gcorr) dC) with respect to the
    stored off-diagonal entries (complex, dL = Re sum conj(G_pq) dH_pq) and the
    on-site energies (real).  Rescale f and dt are fixed.  Tiny systems only."""
    row_ptr, col, val, onsite, psi0 = _prep(row_ptr, col, val, onsite, psi0)
    n, S = psi0.shape
    gcorr = np.ascontiguousarray(gcorr, dtype=np.complex128).reshape(n_steps, S)
    f, M, J = _scale_and_coeffs(row_ptr, val, onsite, dt, rescale, tol)
    gval = np.zeros(col.shape[0], dtype=np.complex128)
    gons = np.zeros(n, dtype=np.float64)
    rc = _load().oracle_backward(n, row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data,
                                 onsite.ctypes.data, f, S, psi0.ctypes.data, n_steps, M,
                                 J.ctypes.data, gcorr.ctypes.data, gval.ctypes.data, gons.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_backward failed")
    return gval, gons
