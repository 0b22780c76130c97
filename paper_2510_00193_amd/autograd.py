"""torch.autograd surface of the coefficient adjoint.

MTPFunction makes a configuration's energy and forces differentiable functions of the
coefficients (linear xi, radial c, species shift s), so that a fitting loop can call
torch.autograd on any loss built from (E, F).  The backward pass is the library's
hand-written vector-Jacobian product (mtp_param_grad): the moments and their adjoints are
recomputed from the positions rather than stored between the two passes.  MTPBatchFunction is
the same over a Batch of configurations (mtp_batch_run forward, mtp_batch_vjp backward).

Derivatives with respect to positions, species or the cell are not provided (forces already
are the first derivative; their derivative would be the Hessian), and neither is a second
derivative with respect to the coefficients: both raise.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from .api import Batch, NeighborList, Potential


def _coef(t, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.detach().contiguous()


def _shapes(pot):
    return {"linear": (pot.n_alpha,), "radial": (pot.n_species, pot.n_species, pot.n_mu, pot.n_cheb),
            "shift": (pot.n_species,)}


class MTPFunction(torch.autograd.Function):
    """(E, F) = MTPFunction.apply(pot, pos, species, cell, linear, radial, shift, nlist=None).

    pot: a float64 Potential (its coefficients are overwritten in place by linear, radial and
    shift on every forward and backward); pos [N, 3] float64 and species [N] int32 on the GPU;
    cell a host 3x3 array; linear [n_alpha], radial [n_sp, n_sp, n_mu, n_cheb], shift [n_sp]
    float64 CUDA tensors; nlist an optional NeighborList.  Returns E (0-d) and F [N, 3].
    backward(ebar, fbar) returns the gradients of linear, radial and shift.
    """

    @staticmethod
    def forward(ctx, pot: Potential, pos, species, cell, linear, radial, shift, nlist: NeighborList = None):
        if any(ctx.needs_input_grad[1:4]):
            raise NotImplementedError("MTPFunction differentiates with respect to the coefficients only")
        sh = _shapes(pot)
        xi = _coef(linear, sh["linear"], "linear")
        c = _coef(radial, sh["radial"], "radial")
        s = _coef(shift, sh["shift"], "shift")
        pot.set_params(radial=c, linear=xi, shift=s)
        out = pot.compute(pos, species, cell, nlist=nlist, forces=True, virial=False)
        ctx.pot, ctx.cell, ctx.nlist = pot, cell, nlist
        ctx.save_for_backward(pos, species, xi, c, s)
        return out["energy"].clone(), out["forces"]

    @staticmethod
    @once_differentiable
    def backward(ctx, ebar, fbar):
        pos, species, xi, c, s = ctx.saved_tensors
        pot = ctx.pot
        # one host read of the energy cotangent (the C entry point takes it by value)
        e = 0.0 if ebar is None else float(ebar)
        if fbar is None:
            fbar = torch.zeros_like(pos)
        pot.set_params(radial=c, linear=xi, shift=s)
        dl, dr, ds = pot.param_grad(pos, species, ctx.cell, e, fbar.contiguous(), nlist=ctx.nlist)
        need = ctx.needs_input_grad
        return (None, None, None, None, dl if need[4] else None, dr if need[5] else None,
                ds if need[6] else None, None)


class MTPBatchFunction(torch.autograd.Function):
    """(E [n_cfg], F [N, 3]) = MTPBatchFunction.apply(batch, linear, radial, shift).

    The coefficients are written into the batch's potential in place on every forward and
    backward; backward(ebar [n_cfg], fbar [N, 3]) returns their gradients through
    mtp_batch_vjp (all configurations in one launch per kernel type).
    """

    @staticmethod
    def forward(ctx, batch: Batch, linear, radial, shift):
        pot = batch._pot
        sh = _shapes(pot)
        xi = _coef(linear, sh["linear"], "linear")
        c = _coef(radial, sh["radial"], "radial")
        s = _coef(shift, sh["shift"], "shift")
        pot.set_params(radial=c, linear=xi, shift=s)
        out = batch.run(batch.outputs(loss=False))
        ctx.batch = batch
        ctx.save_for_backward(xi, c, s)
        return out["energy"], out["forces"]

    @staticmethod
    @once_differentiable
    def backward(ctx, ebar, fbar):
        xi, c, s = ctx.saved_tensors
        b = ctx.batch
        dev = b.pos.device
        if ebar is None:
            ebar = torch.zeros(b.n_cfg, dtype=torch.float64, device=dev)
        if fbar is None:
            fbar = torch.zeros((b.n_atoms, 3), dtype=torch.float64, device=dev)
        b._pot.set_params(radial=c, linear=xi, shift=s)
        dl, dr, ds = b.vjp(ebar.contiguous(), fbar.contiguous())
        need = ctx.needs_input_grad
        return None, dl if need[1] else None, dr if need[2] else None, ds if need[3] else None


def energy_forces(pot, pos, species, cell, linear, radial, shift, nlist=None):
    """Differentiable (E, F) of one configuration (see MTPFunction)."""
    return MTPFunction.apply(pot, pos, species, cell, linear, radial, shift, nlist)


def batch_energy_forces(batch, linear, radial, shift):
    """Differentiable (E [n_cfg], F [N, 3]) of a batch (see MTPBatchFunction)."""
    return MTPBatchFunction.apply(batch, linear, radial, shift)
