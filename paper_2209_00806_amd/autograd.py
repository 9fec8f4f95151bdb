"""Differentiable TBPM DOS: torch.autograd.Function over the library's
forward (tbpm_propagate + tbpm_dos) and adjoint (tbpm_dos_backward +
tbpm_backward) entry points.

Gradients follow PyTorch's convention for complex tensors: the gradient G
of a real loss with respect to a complex tensor H satisfies
dL = Re sum conj(G) dH.  Rescale f and dt are held fixed.
"""
from __future__ import annotations

import torch

from . import tbpm


class TBPMDos(torch.autograd.Function):
    """D(E_j) for the Hamiltonian with stored off-diagonal values ``val``
    (complex128 [nnz], merged CSR order of ``H``) and on-site energies
    ``onsite`` (float64 [n_orb]).  Returns (energies, dos); only dos is
    differentiable."""

    @staticmethod
    def forward(ctx, val, onsite, H, psi0, n_steps, dt, rescale, ckpt_every, tol, window):
        H.set_values(val.detach().contiguous(), onsite.detach().contiguous())
        corr, ckpt = tbpm.propagate(H, psi0, n_steps, dt, rescale, tol=tol, ckpt_every=ckpt_every)
        E, D = tbpm.dos(corr, dt, window=window)
        ctx.H = H
        ctx.meta = (n_steps, dt, rescale, ckpt_every, tol, window)
        ctx.save_for_backward(val.detach(), onsite.detach(), psi0, ckpt)
        ctx.mark_non_differentiable(E)
        return E, D

    @staticmethod
    def backward(ctx, gE, gD):
        val, onsite, psi0, ckpt = ctx.saved_tensors
        n_steps, dt, rescale, ckpt_every, tol, window = ctx.meta
        H = ctx.H
        # the handle may have been given other values since the forward pass
        H.set_values(val.contiguous(), onsite.contiguous())
        S = psi0.shape[1]
        gcorr = tbpm.dos_backward(gD.contiguous().to(torch.float64), n_steps, S, dt, window=window)
        gval, gons = tbpm.backward(H, psi0, n_steps, dt, rescale, gcorr, ckpt_every, ckpt, tol=tol)
        return gval, gons, None, None, None, None, None, None, None, None


def tbpm_dos(H: "tbpm.Hamiltonian", val, onsite, psi0, n_steps: int, dt: float, rescale: float,
             ckpt_every: int = 64, tol: float = 1e-12, window: str = "hann"):
    """Differentiable (energies, dos) of H with values (val, onsite).  The
    rescale factor f must be given (> 0) and bound the spectrum for every
    value the optimiser visits: the values reach the library as device
    tensors, whose Gershgorin bound it never sees."""
    if not rescale > 0:
        raise ValueError("rescale must be positive: the values are set from device tensors, whose bound is unknown")
    return TBPMDos.apply(val, onsite, H, psi0, n_steps, dt, rescale, ckpt_every, tol, window)


def bond_values(n_nnz: int, slot_ij, slot_ji, bond_t):
    """CSR values of a real symmetric bond parameterisation: bond b sets the
    stored entries slot_ij[b] and slot_ji[b] to bond_t[b] (entries hit by
    several bonds get the sum).  Differentiable in bond_t."""
    t = bond_t.to(torch.complex128)
    val = torch.zeros(n_nnz, dtype=torch.complex128, device=bond_t.device)
    val = val.index_add(0, slot_ij, t)
    return val.index_add(0, slot_ji, t)
