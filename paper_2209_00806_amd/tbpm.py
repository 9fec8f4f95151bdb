"""Thin Python binding of libtbpm (argument marshalling only).

Every step of the TBPM path runs in the library's HIP kernels; this module
only converts numpy arrays / torch tensors to pointers, picks the current
torch stream, and turns status codes into exceptions.  It raises
:class:`TBPMError` if the compiled library is missing -- there is no
fallback implementation.

Layouts (see ``include/tbpm.h``): states ``[n_orb, n_states]`` complex128,
correlations ``[n_steps, n_states]`` complex128, DOS on ``2*n_steps``
energies.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtbpm.so")

STATUS = {0: "TBPM_OK", 1: "TBPM_E_ARG", 2: "TBPM_E_CSR", 3: "TBPM_E_NOT_HERMITIAN", 4: "TBPM_E_OOM",
          5: "TBPM_E_DEVICE", 6: "TBPM_E_DIVERGED"}
FP64, FP32_MIXED = 0, 1
WIN = {"hann": 0, "none": 1}
FLAG_DEVICE_PTRS, FLAG_ASYNC, FLAG_NO_GRAPH = 1, 2, 4


class TBPMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class LaunchConfig(ctypes.Structure):
    _fields_ = [("wg_chunks", ctypes.c_int32), ("xcd_remap", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("staged", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("fused", ctypes.c_int32)]

    def as_dict(self):
        return {"wg_chunks": self.wg_chunks, "xcd_remap": self.xcd_remap, "nontemporal": self.nontemporal,
                "unroll": self.unroll, "staged": self.staged, "vec": self.vec, "fused": self.fused}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libtbpm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TBPMError(5, f"{LIB_PATH} not found: build it with paper_2209_00806_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, U32, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_uint32, ctypes.c_size_t)
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "tbpm_hamiltonian_create": [I64, P, P, P, P, U32, PP],
        "tbpm_hamiltonian_set_values": [P, P, P, U32, P],
        "tbpm_hamiltonian_info": [P, P, P, P, P, P],
        "tbpm_hamiltonian_pattern": [P, P, P],
        "tbpm_hamiltonian_destroy": [P],
        "tbpm_hamiltonian_set_row_order": [P, I32],
        "tbpm_hamiltonian_get_row_order": [P, P],
        "tbpm_num_terms": [D, D, P],
        "tbpm_bessel_j": [D, I32, P],
        "tbpm_propagate": [P, P, I32, I32, D, D, D, ctypes.c_int, P, P, I32, P, U32, P],
        "tbpm_propagate_noalloc": [P, P, I32, I32, D, D, D, ctypes.c_int, P, P, P],
        "tbpm_propagate_snapshots": [P, P, I32, P, I32, D, D, D, ctypes.c_int, P, P, U32, P],
        "tbpm_quasi_eigenstates": [P, P, I32, I32, D, D, D, ctypes.c_int, P, I32, ctypes.c_int, P, P, U32, P],
        "tbpm_ac_corr": [P, P, P, P, I32, I32, D, D, D, D, D, D, ctypes.c_int, P, U32, P],
        "tbpm_ac_cond": [P, I32, I32, D, D, D, ctypes.c_int, P, P, P],
        "tbpm_ac_cond_imag": [P, I32, P, P],
        "tbpm_fermi_cheb": [D, D, D, D, P, I32, P],
        "tbpm_kpm_moments": [P, P, P, P, I32, I32, D, P, P, P],
        "tbpm_kubo_bastin": [P, I32, D, D, D, I32, D, P, I32, D, P, P, P, P],
        "tbpm_haydock": [P, P, I32, I32, P, P, U32, P],
        "tbpm_haydock_ldos": [P, P, I32, I32, P, ctypes.c_int64, D, P, P],
        "tbpm_dos": [P, I32, I32, D, ctypes.c_int, P, P, P],
        "tbpm_dos_backward": [P, I32, I32, D, ctypes.c_int, P, P],
        "tbpm_backward": [P, P, I32, I32, D, D, D, P, I32, P, P, P, P],
        "tbpm_batch_create": [P, I32, PP],
        "tbpm_batch_destroy": [P],
        "tbpm_propagate_batched": [P, P, I32, I32, P, P, D, ctypes.c_int, P, P, U32, P],
        "tbpm_get_launch_config": [P, ctypes.c_int, P],
        "tbpm_set_launch_config": [P, ctypes.c_int, P],
        "tbpm_batch_get_launch_config": [P, ctypes.c_int, P],
        "tbpm_batch_set_launch_config": [P, ctypes.c_int, P],
        "tbpm_autotune": [P, I32, ctypes.c_int, P, P, P],
        "tbpm_batch_autotune": [P, I32, ctypes.c_int, P, P, P],
        "tbpm_stream_copy": [P, P, SZ, P],
        "tbpm_bench_pass": [P, I32, ctypes.c_int, I32, P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.tbpm_last_error.argtypes = []
    L.tbpm_last_error.restype = ctypes.c_char_p
    L.tbpm_version.argtypes = []
    L.tbpm_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise TBPMError(status, lib().tbpm_last_error().decode())


def _ptr(a) -> int:
    """Data pointer of a contiguous numpy array or torch tensor."""
    if a is None:
        return 0
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return a.ctypes.data


def _stream(stream=None) -> int:
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _require_cuda(t, dtype, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def version() -> str:
    return lib().tbpm_version().decode()


def num_terms(z: float, tol: float = 1e-12) -> int:
    m = ctypes.c_int32()
    _check(lib().tbpm_num_terms(float(z), float(tol), ctypes.byref(m)))
    return m.value


def bessel_j(z: float, M: int) -> np.ndarray:
    out = np.zeros(M)
    _check(lib().tbpm_bessel_j(float(z), int(M), out.ctypes.data))
    return out


class Hamiltonian:
    """Library-owned device copy of a tight-binding Hamiltonian."""

    def __init__(self, n_orb: int, row_ptr, col, val, onsite):
        """CSR arrays as numpy arrays (host), or all four as CUDA tensors on the
        current device (int64, int32, complex128, float64), which the library
        reads from device memory (TBPM_FLAG_DEVICE_PTRS)."""
        h = ctypes.c_void_p()
        if hasattr(row_ptr, "is_cuda") and row_ptr.is_cuda:
            import torch

            for t, dt, name in ((row_ptr, torch.int64, "row_ptr"), (col, torch.int32, "col"),
                                (val, torch.complex128, "val"), (onsite, torch.float64, "onsite")):
                _require_cuda(t, dt, name)
            _check(lib().tbpm_hamiltonian_create(int(n_orb), _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(onsite),
                                                 FLAG_DEVICE_PTRS, ctypes.byref(h)))
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
            ci = np.ascontiguousarray(col, dtype=np.int32)
            va = np.ascontiguousarray(val, dtype=np.complex128)
            on = np.ascontiguousarray(onsite, dtype=np.float64)
            _check(lib().tbpm_hamiltonian_create(int(n_orb), rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                                                 on.ctypes.data, 0, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_lattice(cls, lat) -> "Hamiltonian":
        return cls(lat.n_orb, lat.row_ptr, lat.col, lat.val, lat.onsite)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("Hamiltonian has been closed")
        return self._h

    def info(self) -> dict:
        n, nnz, g, c, mr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().tbpm_hamiltonian_info(self.handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(g),
                                           ctypes.byref(c), ctypes.byref(mr)))
        return {"n_orb": n.value, "nnz": nnz.value, "gershgorin": g.value, "is_complex": bool(c.value),
                "max_row": mr.value}

    def pattern(self):
        inf = self.info()
        rp = np.zeros(inf["n_orb"] + 1, dtype=np.int64)
        ci = np.zeros(max(inf["nnz"], 1), dtype=np.int32)
        _check(lib().tbpm_hamiltonian_pattern(self.handle, rp.ctypes.data, ci.ctypes.data))
        return rp, ci[: inf["nnz"]]

    def set_values(self, val, onsite, stream=None):
        """New values on the same (merged) pattern: numpy (host, validated) or
        CUDA torch tensors (device, complex128 [nnz] and float64 [n_orb])."""
        if hasattr(val, "is_cuda") and val.is_cuda:
            _check(lib().tbpm_hamiltonian_set_values(self.handle, _ptr(val), _ptr(onsite), FLAG_DEVICE_PTRS,
                                                     _stream(stream)))
        else:
            va = np.ascontiguousarray(val, dtype=np.complex128)
            on = np.ascontiguousarray(onsite, dtype=np.float64)
            _check(lib().tbpm_hamiltonian_set_values(self.handle, va.ctypes.data, on.ctypes.data, 0, 0))

    def set_row_order(self, order: int):
        """-1: automatic, 0: the caller's orbital order, 1: bisection order on
        the device (re-uploads the matrix from its host values)."""
        _check(lib().tbpm_hamiltonian_set_row_order(self.handle, int(order)))

    def row_order(self) -> int:
        o = ctypes.c_int32()
        _check(lib().tbpm_hamiltonian_get_row_order(self.handle, ctypes.byref(o)))
        return o.value

    def launch_config(self, precision: str = "fp64") -> dict:
        c = LaunchConfig()
        _check(lib().tbpm_get_launch_config(self.handle, _prec(precision), ctypes.byref(c)))
        return c.as_dict()

    def set_launch_config(self, wg_chunks=2, xcd_remap=1, nontemporal=1, unroll=1, staged=0, vec=None,
                          precision=None, fused=0):
        """Launch shape for one precision, or for both when precision is None
        (vec=None: 1 state per thread in FP64, 2 in FP32)."""
        for p in ((FP64, FP32_MIXED) if precision is None else (_prec(precision),)):
            c = LaunchConfig(wg_chunks, xcd_remap, nontemporal, unroll, staged,
                             vec if vec is not None else (2 if p == FP32_MIXED else 1), fused)
            _check(lib().tbpm_set_launch_config(self.handle, p, ctypes.byref(c)))

    def autotune(self, n_states: int, precision: str = "fp64", stream=None):
        c = LaunchConfig()
        ms = ctypes.c_double()
        _check(lib().tbpm_autotune(self.handle, int(n_states), _prec(precision), ctypes.byref(c),
                                   ctypes.byref(ms), _stream(stream)))
        return c.as_dict(), ms.value

    def close(self):
        if getattr(self, "_h", None):
            lib().tbpm_hamiltonian_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _prec(precision: str) -> int:
    if precision in ("fp64", FP64):
        return FP64
    if precision in ("fp32", "fp32_mixed", FP32_MIXED):
        return FP32_MIXED
    raise ValueError(f"unknown precision {precision!r}")


def propagate(H: Hamiltonian, psi0, n_steps: int, dt: float, rescale: float = 0.0, tol: float = 1e-12,
              precision: str = "fp64", return_norm: bool = False, ckpt_every: int = 0, graph: bool = True,
              sync: bool = True, stream=None, out=None):
    """C_k = <psi0|psi(k dt)>, k < n_steps, for psi0 a CUDA complex128 tensor [n_orb, S].

    Returns corr [n_steps, S] (and norm2 [n_steps, S] if return_norm, and the
    checkpoint tensor if ckpt_every > 0).
    """
    import torch

    _require_cuda(psi0, torch.complex128, "psi0")
    if psi0.dim() == 1:
        psi0 = psi0.reshape(-1, 1)
    n, S = psi0.shape
    corr = out if out is not None else torch.empty((n_steps, S), dtype=torch.complex128, device=psi0.device)
    norm2 = torch.empty((n_steps, S), dtype=torch.float64, device=psi0.device) if return_norm else None
    ckpt = None
    if ckpt_every > 0:
        n_ck = max(0, (n_steps - 2) // ckpt_every)
        ckpt = torch.empty((max(n_ck, 1), n, S), dtype=torch.complex128, device=psi0.device)
    flags = (0 if graph else FLAG_NO_GRAPH) | (0 if sync else FLAG_ASYNC)
    _check(lib().tbpm_propagate(H.handle, _ptr(psi0), S, int(n_steps), float(dt), float(rescale), float(tol),
                                _prec(precision), _ptr(corr), _ptr(norm2), int(ckpt_every), _ptr(ckpt), flags,
                                _stream(stream)))
    res = [corr]
    if return_norm:
        res.append(norm2)
    if ckpt_every > 0:
        res.append(ckpt)
    return res[0] if len(res) == 1 else tuple(res)


def propagate_noalloc(H: Hamiltonian, psi0, n_steps: int, dt: float, rescale: float = 0.0, tol: float = 1e-12,
                      precision: str = "fp64", corr=None, norm2=None, stream=None):
    """tbpm_propagate_noalloc: C_k = <psi0|psi(k dt)> into the caller's CUDA
    tensors corr [n_steps, S] complex128 (and norm2 [n_steps, S] float64 if
    given), with no device allocation by the library; enqueued on the stream
    and not synchronised.  Returns corr (allocated here if not given)."""
    import torch

    _require_cuda(psi0, torch.complex128, "psi0")
    if psi0.dim() == 1:
        psi0 = psi0.reshape(-1, 1)
    n, S = psi0.shape
    if corr is None:
        corr = torch.empty((n_steps, S), dtype=torch.complex128, device=psi0.device)
    _require_cuda(corr, torch.complex128, "corr")
    if tuple(corr.shape) != (n_steps, S):
        raise ValueError(f"corr must have shape {(n_steps, S)}")
    if norm2 is not None:
        _require_cuda(norm2, torch.float64, "norm2")
        if tuple(norm2.shape) != (n_steps, S):
            raise ValueError(f"norm2 must have shape {(n_steps, S)}")
    _check(lib().tbpm_propagate_noalloc(H.handle, _ptr(psi0), S, int(n_steps), float(dt), float(rescale),
                                        float(tol), _prec(precision), _ptr(corr), _ptr(norm2), _stream(stream)))
    return corr


def propagate_snapshots(H: Hamiltonian, psi0, steps, dt: float, rescale: float = 0.0, tol: float = 1e-12,
                        precision: str = "fp64", return_corr: bool = False, stream=None):
    """psi(k dt) for every k in ``steps`` (distinct, >= 0), for psi0 a CUDA
    complex128 tensor [n_orb, S] (or [n_orb]).  Returns snapshots
    [len(steps), n_orb, S] complex128 (and corr [max(steps)+1, S] if asked)."""
    import torch

    _require_cuda(psi0, torch.complex128, "psi0")
    squeeze = psi0.dim() == 1
    if squeeze:
        psi0 = psi0.reshape(-1, 1)
    n, S = psi0.shape
    st = np.ascontiguousarray(np.asarray(steps, dtype=np.int64).reshape(-1).astype(np.int32))
    if st.size == 0:
        raise ValueError("steps must not be empty")
    snaps = torch.empty((st.size, n, S), dtype=torch.complex128, device=psi0.device)
    corr = torch.empty((int(st.max()) + 1, S), dtype=torch.complex128, device=psi0.device) if return_corr else None
    _check(lib().tbpm_propagate_snapshots(H.handle, _ptr(psi0), S, st.ctypes.data, int(st.size), float(dt),
                                          float(rescale), float(tol), _prec(precision), _ptr(snaps), _ptr(corr), 0,
                                          _stream(stream)))
    if squeeze:
        snaps = snaps[:, :, 0]
    return (snaps, corr) if return_corr else snaps


def quasi_eigenstates(H: Hamiltonian, psi0, energies, n_steps: int, dt: float, rescale: float = 0.0,
                      tol: float = 1e-12, precision: str = "fp64", window: str = "hann", return_norm: bool = False,
                      stream=None):
    """Quasi-eigenstates at ``energies`` (eV) from the CUDA complex128 state(s)
    psi0 [n_orb, S] (or [n_orb]): windowed Fourier transform of psi(t) over
    -(n_steps-1) dt .. (n_steps-1) dt, normalised.  Returns [n_E, n_orb, S]
    (or [n_E, n_orb]) complex128, and ||Psi(E)||^2 [n_E, S] if asked."""
    import torch

    _require_cuda(psi0, torch.complex128, "psi0")
    squeeze = psi0.dim() == 1
    if squeeze:
        psi0 = psi0.reshape(-1, 1)
    n, S = psi0.shape
    e = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).reshape(-1))
    out = torch.empty((e.size, n, S), dtype=torch.complex128, device=psi0.device)
    n2 = torch.empty((e.size, S), dtype=torch.float64, device=psi0.device) if return_norm else None
    _check(lib().tbpm_quasi_eigenstates(H.handle, _ptr(psi0), S, int(n_steps), float(dt), float(rescale), float(tol),
                                        _prec(precision), e.ctypes.data, int(e.size), WIN[window], _ptr(out), _ptr(n2), 0,
                                        _stream(stream)))
    if squeeze:
        out = out[:, :, 0]
        n2 = n2[:, 0] if n2 is not None else None
    return (out, n2) if return_norm else out


def ac_corr(H: Hamiltonian, j_alpha, j_beta, psi0, n_steps: int, dt: float, beta: float, mu: float,
            rescale: float = 0.0, tol: float = 1e-12, fermi_tol: float = 1e-12, precision: str = "fp64", stream=None):
    """Optical-conductivity correlation <psi2(t)|J_alpha|psi1(t)> (numpy
    complex128 current operators on H's merged pattern; psi0 a CUDA
    complex128 tensor [n_orb, S], S <= 32).  Returns corr [n_steps, S]."""
    import torch

    _require_cuda(psi0, torch.complex128, "psi0")
    if psi0.dim() == 1:
        psi0 = psi0.reshape(-1, 1)
    nnz = H.info()["nnz"]
    ja = np.ascontiguousarray(j_alpha, dtype=np.complex128)
    jb = np.ascontiguousarray(j_beta, dtype=np.complex128)
    if ja.shape != (nnz,) or jb.shape != (nnz,):
        raise ValueError(f"current operators must hold one value per stored element ({nnz})")
    n, S = psi0.shape
    corr = torch.empty((n_steps, S), dtype=torch.complex128, device=psi0.device)
    _check(lib().tbpm_ac_corr(H.handle, ja.ctypes.data, jb.ctypes.data, _ptr(psi0), S, int(n_steps), float(dt),
                              float(rescale), float(tol), float(beta), float(mu), float(fermi_tol), _prec(precision),
                              _ptr(corr), 0, _stream(stream)))
    return corr


def kpm_moments(H: Hamiltonian, v_alpha, v_beta, psi0, n_moments: int, rescale: float = 0.0,
                return_timing: bool = False, stream=None):
    """Kubo-Bastin moments mu[m, n] = (1/S) sum_s <r_s| v_alpha T_m(H/f) v_beta
    T_n(H/f) |r_s> (numpy complex128 operators on H's merged pattern; psi0 a
    CUDA complex128 tensor [n_orb, S], S <= 64).  Returns a CUDA complex128
    [M, M] tensor indexed [m, n] (a transposed view of the library's layout),
    and the timing dict if asked."""
    import torch

    _require_cuda(psi0, torch.complex128, "psi0")
    if psi0.dim() == 1:
        psi0 = psi0.reshape(-1, 1)
    nnz = H.info()["nnz"]
    va = np.ascontiguousarray(v_alpha, dtype=np.complex128)
    vb = np.ascontiguousarray(v_beta, dtype=np.complex128)
    if va.shape != (nnz,) or vb.shape != (nnz,):
        raise ValueError(f"operators must hold one value per stored element ({nnz})")
    n, S = psi0.shape
    M = int(n_moments)
    out = torch.empty((M, M), dtype=torch.complex128, device=psi0.device)  # [n][m]
    t = np.zeros(4, dtype=np.float64)
    _check(lib().tbpm_kpm_moments(H.handle, va.ctypes.data, vb.ctypes.data, _ptr(psi0), S, M, float(rescale),
                                  _ptr(out), t.ctypes.data if return_timing else None, _stream(stream)))
    mu = out.transpose(0, 1)
    if return_timing:
        return mu, {"l_ms": float(t[0]), "r_ms": float(t[1]), "product_ms": float(t[2]), "chunks": int(t[3])}
    return mu


def kubo_bastin(mu, rescale: float, e_lo: float, e_hi: float, n_energy: int, beta: float, mus, area: float,
                stream=None):
    """sigma(mu_c) of the Kubo-Bastin formula from kpm_moments' mu (indexed
    [m, n]); returns (sigma [n_mu], energies [n_energy], weight [n_energy]) as
    CUDA float64 tensors."""
    import torch

    if not isinstance(mu, torch.Tensor) or not mu.is_cuda or mu.dtype != torch.complex128 or mu.dim() != 2:
        raise TypeError("mu must be a CUDA complex128 [M, M] tensor")
    M = mu.shape[0]
    mc = mu.transpose(0, 1).contiguous()  # the library's layout [n][m]
    m_t = mus if isinstance(mus, torch.Tensor) else torch.as_tensor(np.asarray(mus, dtype=np.float64))
    m_t = m_t.to(device=mu.device, dtype=torch.float64).contiguous().reshape(-1)
    en = torch.empty(int(n_energy), dtype=torch.float64, device=mu.device)
    w = torch.empty(int(n_energy), dtype=torch.float64, device=mu.device)
    sg = torch.empty(m_t.numel(), dtype=torch.float64, device=mu.device)
    _check(lib().tbpm_kubo_bastin(_ptr(mc), M, float(rescale), float(e_lo), float(e_hi), int(n_energy), float(beta),
                                  _ptr(m_t), m_t.numel(), float(area), _ptr(en), _ptr(w), _ptr(sg), _stream(stream)))
    return sg, en, w


def haydock(H: Hamiltonian, psi0, n_iter: int, graph: bool = True, stream=None):
    """Haydock (Lanczos) coefficients of every column of psi0 (CUDA
    complex128 [n_orb, S], S <= 64): returns (a, b), each [n_iter, S] float64
    with b[i] = b_{i+1}."""
    import torch

    _require_cuda(psi0, torch.complex128, "psi0")
    if psi0.dim() == 1:
        psi0 = psi0.reshape(-1, 1)
    n, S = psi0.shape
    a = torch.empty((n_iter, S), dtype=torch.float64, device=psi0.device)
    b = torch.empty((n_iter, S), dtype=torch.float64, device=psi0.device)
    _check(lib().tbpm_haydock(H.handle, _ptr(psi0), S, int(n_iter), _ptr(a), _ptr(b),
                              0 if graph else FLAG_NO_GRAPH, _stream(stream)))
    return a, b


def haydock_ldos(a, b, energies, eps: float, stream=None):
    """-(1/pi) Im G_0(E + i eps) by the continued fraction of Haydock
    coefficients (CUDA float64 [n_iter, S]); energies a sequence or a CUDA
    float64 tensor.  Returns [n_E, S]."""
    import torch

    _require_cuda(a, torch.float64, "a")
    _require_cuda(b, torch.float64, "b")
    if a.dim() == 1:
        a, b = a.reshape(-1, 1), b.reshape(-1, 1)
    if a.shape != b.shape:
        raise ValueError("a and b must have the same shape")
    en = energies if isinstance(energies, torch.Tensor) else torch.as_tensor(
        np.asarray(energies, dtype=np.float64), device=a.device)
    en = en.to(device=a.device, dtype=torch.float64).contiguous()
    n_iter, S = a.shape
    out = torch.empty((en.numel(), S), dtype=torch.float64, device=a.device)
    _check(lib().tbpm_haydock_ldos(_ptr(a.contiguous()), _ptr(b.contiguous()), n_iter, S, _ptr(en), en.numel(),
                                   float(eps), _ptr(out), _stream(stream)))
    return out


def ldos_haydock(H: Hamiltonian, orbitals, n_iter: int, energies, eps: float, stream=None):
    """LDOS averaged over ``orbitals`` by the recursion method (unit-vector
    start states, one Lanczos chain each, up to 64 per launch)."""
    import torch

    orbitals = np.asarray(orbitals, dtype=np.int64)
    n = H.info()["n_orb"]
    total = None
    for c0 in range(0, orbitals.size, 64):
        chunk = orbitals[c0:c0 + 64]
        st = torch.zeros((n, chunk.size), dtype=torch.complex128, device="cuda")
        st[torch.as_tensor(chunk, device="cuda"), torch.arange(chunk.size, device="cuda")] = 1.0
        a, b = haydock(H, st, n_iter, stream=stream)
        d = haydock_ldos(a, b, energies, eps, stream=stream).sum(dim=1)
        total = d if total is None else total + d
    return total / orbitals.size


def fermi_coeffs(beta: float, mu: float, rescale: float, tol: float = 1e-12) -> np.ndarray:
    """Chebyshev coefficients a_k of the Fermi-Dirac function on [-rescale,
    rescale] (f(H) = sum_k a_k T_k(H/rescale)), as ac_corr uses them."""
    K = ctypes.c_int32(0)
    _check(lib().tbpm_fermi_cheb(float(beta), float(mu), float(rescale), float(tol), None, 0, ctypes.byref(K)))
    a = np.zeros(K.value, dtype=np.float64)
    _check(lib().tbpm_fermi_cheb(float(beta), float(mu), float(rescale), float(tol), a.ctypes.data, K.value,
                                 ctypes.byref(K)))
    return a


def ac_cond(corr, dt: float, beta: float, area: float, window: str = "hann", stream=None):
    """(omegas, Re sigma) on w_j = j pi/(n_steps dt), j = 0..n_steps-1, from
    ac_corr's correlation (CUDA complex128 [n_steps, S])."""
    import torch

    _require_cuda(corr, torch.complex128, "corr")
    if corr.dim() == 1:
        corr = corr.reshape(-1, 1)
    nt, S = corr.shape
    om = torch.empty(nt, dtype=torch.float64, device=corr.device)
    sg = torch.empty(nt, dtype=torch.float64, device=corr.device)
    _check(lib().tbpm_ac_cond(_ptr(corr), nt, S, float(dt), float(beta), float(area), WIN[window], _ptr(om), _ptr(sg),
                              _stream(stream)))
    return om, sg


def ac_cond_imag(re_sigma, stream=None):
    """Im sigma on the same grid from Re sigma (a CUDA float64 tensor [n], e.g.
    ac_cond's second output) by the Kramers-Kronig relation."""
    import torch

    _require_cuda(re_sigma, torch.float64, "re_sigma")
    if re_sigma.dim() != 1:
        raise ValueError("re_sigma must be one-dimensional")
    im = torch.empty_like(re_sigma)
    _check(lib().tbpm_ac_cond_imag(_ptr(re_sigma), int(re_sigma.shape[0]), _ptr(im), _stream(stream)))
    return im


def ldos(H: Hamiltonian, orbitals, n_steps: int, dt: float, rescale: float = 0.0, tol: float = 1e-12,
         precision: str = "fp64", window: str = "hann", stream=None):
    """Local density of states by propagation (Sec. "Local density of
    states"): each listed orbital's unit vector is propagated, and the DOS
    transform of the correlations, averaged over the orbitals, is returned
    as (energies, ldos) CUDA float64 tensors.  Orbitals go 64 per launch."""
    import torch

    orbs = np.asarray(orbitals, dtype=np.int64).reshape(-1)
    n = H.info()["n_orb"]
    if orbs.size == 0 or orbs.min() < 0 or orbs.max() >= n:
        raise ValueError("orbitals must be non-empty and inside [0, n_orb)")
    corr_all = []
    for c0 in range(0, orbs.size, 64):
        chunk = orbs[c0:c0 + 64]
        psi0 = torch.zeros((n, chunk.size), dtype=torch.complex128, device="cuda")
        psi0[torch.from_numpy(chunk).cuda(), torch.arange(chunk.size, device="cuda")] = 1.0
        corr_all.append(propagate(H, psi0, n_steps, dt, rescale, tol, precision, stream=stream))
    corr = torch.cat(corr_all, dim=1).contiguous()
    return dos(corr, dt, window, stream=stream)


def dos(corr, dt: float, window: str = "hann", stream=None):
    """(energies, dos) on the 2*n_steps grid E_j = j pi/(n_steps dt), j = -n_steps..n_steps-1."""
    import torch

    _require_cuda(corr, torch.complex128, "corr")
    if corr.dim() == 1:
        corr = corr.reshape(-1, 1)
    nt, S = corr.shape
    e = torch.empty(2 * nt, dtype=torch.float64, device=corr.device)
    d = torch.empty(2 * nt, dtype=torch.float64, device=corr.device)
    _check(lib().tbpm_dos(_ptr(corr), nt, S, float(dt), WIN[window], _ptr(e), _ptr(d), _stream(stream)))
    return e, d


def dos_backward(grad_dos, n_steps: int, n_states: int, dt: float, window: str = "hann", stream=None):
    import torch

    _require_cuda(grad_dos, torch.float64, "grad_dos")
    g = torch.empty((n_steps, n_states), dtype=torch.complex128, device=grad_dos.device)
    _check(lib().tbpm_dos_backward(_ptr(grad_dos), int(n_steps), int(n_states), float(dt), WIN[window], _ptr(g),
                                   _stream(stream)))
    return g


def backward(H: Hamiltonian, psi0, n_steps: int, dt: float, rescale: float, grad_corr, ckpt_every: int, ckpt,
             tol: float = 1e-12, stream=None):
    """(grad_val complex128 [nnz], grad_onsite float64 [n_orb]) of L through C (see include/tbpm.h)."""
    import torch

    _require_cuda(psi0, torch.complex128, "psi0")
    _require_cuda(grad_corr, torch.complex128, "grad_corr")
    n, S = psi0.shape
    inf = H.info()
    gv = torch.empty(max(inf["nnz"], 1), dtype=torch.complex128, device=psi0.device)
    go = torch.empty(n, dtype=torch.float64, device=psi0.device)
    _check(lib().tbpm_backward(H.handle, _ptr(psi0), S, int(n_steps), float(dt), float(rescale), float(tol),
                               _ptr(grad_corr), int(ckpt_every), _ptr(ckpt), _ptr(gv), _ptr(go), _stream(stream)))
    return gv[: inf["nnz"]], go


class Batch:
    """Several Hamiltonians propagated together (one launch per Chebyshev pass)."""

    def __init__(self, hams: Sequence[Hamiltonian]):
        self.hams = list(hams)
        arr = (ctypes.c_void_p * len(self.hams))(*[h.handle.value for h in self.hams])
        b = ctypes.c_void_p()
        _check(lib().tbpm_batch_create(arr, len(self.hams), ctypes.byref(b)))
        self._b = b

    def propagate(self, psi0s, n_steps: int, dts, rescales=None, tol: float = 1e-12, precision: str = "fp64",
                  return_norm: bool = False, graph: bool = True, sync: bool = True, stream=None):
        import torch

        n = len(self.hams)
        if len(psi0s) != n:
            raise ValueError("one psi0 per Hamiltonian")
        S = psi0s[0].shape[1]
        for p in psi0s:
            _require_cuda(p, torch.complex128, "psi0")
            if p.shape[1] != S:
                raise ValueError("all members need the same number of states")
        corrs = [torch.empty((n_steps, S), dtype=torch.complex128, device=psi0s[0].device) for _ in range(n)]
        norms = [torch.empty((n_steps, S), dtype=torch.float64, device=psi0s[0].device) for _ in range(n)] \
            if return_norm else None
        P = ctypes.c_void_p * n
        p_arr = P(*[_ptr(p) for p in psi0s])
        c_arr = P(*[_ptr(c) for c in corrs])
        n_arr = P(*[_ptr(x) for x in norms]) if norms else None
        dt_arr = np.ascontiguousarray(dts, dtype=np.float64)
        f_arr = np.zeros(n) if rescales is None else np.ascontiguousarray(rescales, dtype=np.float64)
        flags = (0 if graph else FLAG_NO_GRAPH) | (0 if sync else FLAG_ASYNC)
        _check(lib().tbpm_propagate_batched(self._b, p_arr, S, int(n_steps), dt_arr.ctypes.data, f_arr.ctypes.data,
                                            float(tol), _prec(precision), c_arr,
                                            n_arr if n_arr is not None else None, flags, _stream(stream)))
        return (corrs, norms) if return_norm else corrs

    def launch_config(self, precision: str = "fp64") -> dict:
        c = LaunchConfig()
        _check(lib().tbpm_batch_get_launch_config(self._b, _prec(precision), ctypes.byref(c)))
        return c.as_dict()

    def set_launch_config(self, wg_chunks=2, xcd_remap=1, nontemporal=1, unroll=1, staged=0, vec=None,
                          precision=None, fused=0):
        for p in ((FP64, FP32_MIXED) if precision is None else (_prec(precision),)):
            c = LaunchConfig(wg_chunks, xcd_remap, nontemporal, unroll, staged,
                             vec if vec is not None else (2 if p == FP32_MIXED else 1), fused)
            _check(lib().tbpm_batch_set_launch_config(self._b, p, ctypes.byref(c)))

    def autotune(self, n_states: int, precision: str = "fp64", stream=None):
        c = LaunchConfig()
        ms = ctypes.c_double()
        _check(lib().tbpm_batch_autotune(self._b, int(n_states), _prec(precision), ctypes.byref(c),
                                         ctypes.byref(ms), _stream(stream)))
        return c.as_dict(), ms.value

    def close(self):
        if getattr(self, "_b", None):
            lib().tbpm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_copy(src, dst, stream=None):
    """Plain device copy of src into dst (bandwidth calibration)."""
    nbytes = src.numel() * src.element_size()
    _check(lib().tbpm_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)))


def bench_pass(H: Hamiltonian, n_states: int, precision: str, n_launch: int, stream=None):
    """Enqueue n_launch launches of the interior Clenshaw pass (timing only)."""
    _check(lib().tbpm_bench_pass(H.handle, int(n_states), _prec(precision), int(n_launch), _stream(stream)))


def autotune_cached(H: Hamiltonian, n_states: int, precision: str, path: str | None = None, stream=None):
    """Autotune H for (n_states, precision), reusing a result stored in the JSON
    file ``path`` under the key (device, n_orb, nnz, max row, n_states,
    precision); the library's autotuner runs only on a cache miss."""
    import json

    import torch

    inf = H.info()
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    device = f"{getattr(props, 'gcnArchName', '')}:{props.multi_processor_count}"
    key = "|".join(str(x) for x in (device, inf["n_orb"], inf["nnz"], inf["max_row"], n_states, precision))
    cache = {}
    if path and os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    if key in cache:
        cfg = cache[key]["config"]
        H.set_launch_config(cfg["wg_chunks"], cfg["xcd_remap"], cfg["nontemporal"], cfg["unroll"],
                            cfg.get("staged", 0), cfg.get("vec"), precision=precision, fused=cfg.get("fused", 0))
        return cfg, cache[key]["ms_per_step"], True
    cfg, ms = H.autotune(n_states, precision, stream=stream)
    if path:
        cache[key] = {"config": cfg, "ms_per_step": ms}
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, path)
    return cfg, ms, False


def default_dt(rescale: float) -> float:
    """The paper's time step dt = pi / f (usage section, TBPM example)."""
    return math.pi / rescale
