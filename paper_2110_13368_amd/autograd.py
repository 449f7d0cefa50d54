"""torch.autograd view of n LOD steps with cell sources.

The forward pass runs the HIP step; the backward pass calls the library's
adjoint (checkpointed replay, reverse sources, reverse z/y/x solves).  The
differentiable inputs are the field and the parameters the step depends on:
D and lambda per substrate (diffusion and decay of the diffusion-decay
equation) and each cell's secretion rate S and uptake rate U (the cell source
term of the same equation).  Positions, volumes, saturation densities,
boundaries and the time step are fixed by the context.
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import Context


def _host(a) -> np.ndarray:
    """float64 host copy of a numpy array or torch tensor."""
    if isinstance(a, torch.Tensor):
        return a.detach().cpu().double().numpy()
    return np.asarray(a, np.float64)


def flat_params(ctx: Context):
    """Current D, lambda (float64, one per volume) and S, U (float64, per
    simulation its cells as last uploaded x n_sub, concatenated) of a context."""
    D = np.concatenate([p[0].ravel() for p in ctx.params])
    lam = np.concatenate([p[1].ravel() for p in ctx.params])
    cells = [c for c in ctx.cells if c is not None and c.n > 0]
    S = np.concatenate([_host(c.S).ravel() for c in cells] + [np.zeros(0)])
    U = np.concatenate([_host(c.U).ravel() for c in cells] + [np.zeros(0)])
    return tuple(torch.from_numpy(a.copy()) for a in (D, lam, S, U))


def _load(ctx: Context, D, lam, S, U) -> None:
    """Make the context's parameters equal D, lam, S, U (host float64).  The
    cells keep the positions, volumes and targets of their last upload."""
    state = getattr(ctx, "_autograd_params", None)
    if state is None:
        state = ctx._autograd_params = tuple(t.numpy().copy() for t in flat_params(ctx))
    D = D.detach().cpu().double().numpy()
    lam = lam.detach().cpu().double().numpy()
    S = S.detach().cpu().double().numpy()
    U = U.detach().cpu().double().numpy()
    if S.size != state[2].size or U.size != state[3].size or D.size != state[0].size:
        raise ValueError("parameter sizes do not match the context's current cells "
                         "(call flat_params again after moving or re-uploading cells)")
    v = c = 0
    for k, s in enumerate(ctx.sims):
        nv, nc = s.n_sub, ctx.n_cells(k) * s.n_sub
        if not (np.array_equal(D[v:v + nv], state[0][v:v + nv]) and np.array_equal(lam[v:v + nv], state[1][v:v + nv])):
            ctx.update_substrates(k, D[v:v + nv], lam[v:v + nv])
        if nc and not (np.array_equal(S[c:c + nc], state[2][c:c + nc]) and np.array_equal(U[c:c + nc], state[3][c:c + nc])):
            cl = ctx.cells[k]
            Sk, Uk = S[c:c + nc].reshape(-1, s.n_sub), U[c:c + nc].reshape(-1, s.n_sub)
            if isinstance(cl.V, torch.Tensor):  # a device upload: keep its positions on the device
                dev = cl.V.device
                ctx.upload_cells_device(k, cl.pos, cl.V, torch.from_numpy(Sk).to(dev),
                                        torch.from_numpy(Uk).to(dev), cl.rho_star)
            else:
                ctx.upload_cells(k, type(cl)(cl.pos, cl.V, Sk, Uk, cl.rho_star))
        v += nv
        c += nc
    ctx._autograd_params = (D.copy(), lam.copy(), S.copy(), U.copy())


class LODStepFn(torch.autograd.Function):
    """rho_n = (n LOD steps)(rho_0; D, lambda, S, U) for every simulation of a
    Context.  rho_0 and rho_n are float32 tensors in the context's field
    layout (``Context.to_field_layout`` / ``from_field_layout``); D, lambda,
    S, U are float64 as returned by ``flat_params``.  The backward pass keeps
    a checkpoint every ckpt_every steps and replays each segment."""

    @staticmethod
    def forward(fctx, rho0, D, lam, S, U, ctx: Context, n_steps: int, ckpt_every: int):
        if rho0.dtype != ctx.dtype or rho0.numel() != ctx.field_elems:
            raise ValueError("rho0 must be the context's whole field, in its precision")
        _load(ctx, D, lam, S, U)
        torch.cuda.synchronize(ctx.device)
        ctx.field.copy_(rho0.detach().reshape(-1))
        torch.cuda.synchronize(ctx.device)
        ctx.step(n_steps)
        ctx.sync()
        out = ctx.field.clone()
        torch.cuda.synchronize(ctx.device)
        fctx.save_for_backward(rho0, D, lam, S, U)
        fctx.sim, fctx.n_steps, fctx.ckpt_every = ctx, int(n_steps), int(ckpt_every)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        rho0, D, lam, S, U = fctx.saved_tensors
        ctx = fctx.sim
        _load(ctx, D, lam, S, U)
        torch.cuda.synchronize(ctx.device)
        ctx.field.copy_(rho0.detach().reshape(-1))
        torch.cuda.synchronize(ctx.device)
        g0, dD, dl, dS, dU = ctx.adjoint_flat(fctx.n_steps, fctx.ckpt_every, grad_out)
        return (g0.reshape(rho0.shape), dD.to(D.device), dl.to(lam.device), dS.to(S.device), dU.to(U.device),
                None, None, None)


def lod_steps(ctx: Context, rho0, n_steps: int, D, lam, S, U, ckpt_every: int = 20):
    return LODStepFn.apply(rho0, D, lam, S, U, ctx, n_steps, ckpt_every)
