"""Differentiable rollouts of the compact-kernel MPM step on the GPU.

`rollout` runs n steps of the differentiable step (include/ckmpm_adjoint.h) as one
torch.autograd.Function: the forward pass keeps the state at every k-th step; the
backward pass walks the segments in reverse, recomputes each segment's states from
its checkpoint with the forward kernels, and applies the step's reverse-mode
kernels one step at a time.  Every step runs in the HIP library; this module only
marshals tensors and orders the calls.
"""
from __future__ import annotations

import torch

from . import ckmpm


class AdContext:
    """RAII holder for an mpm_ad_ctx: grid geometry and walls of `cfg`, one
    fixed-corotated material (its modulus is replaced per particle by exp(logE))."""

    def __init__(self, cfg: ckmpm.mpm_config, mat: ckmpm.mpm_material):
        s, h = ckmpm.mpm_ad_create(cfg, mat)
        ckmpm.check(s, "mpm_ad_create")
        self.h = h

    def close(self):
        if self.h is not None and self.h.value:
            ckmpm.mpm_ad_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ad_config(sc, direct_budget_mib: int = 256) -> ckmpm.mpm_config:
    """mpm_config for the differentiable step on scene sc: a pool slot for every
    4x4x4-node block of the lattice (no per-call marking) when that costs at most
    `direct_budget_mib` MiB of device memory (7 KiB per block), else the block-sparse
    pool sized as for the main step."""
    nb = 1
    for a in range(3):
        nb *= sc.n_cells[a] // 4 + 1
    if nb * 7168 <= direct_budget_mib * 2 ** 20:
        return ckmpm.scene_config(sc, max_blocks=nb)
    return ckmpm.scene_config(sc)


def _step(ad: AdContext, state: torch.Tensor, logE: torch.Tensor, dt: float, stream) -> torch.Tensor:
    out = torch.empty_like(state)
    n = state.shape[1]
    ckmpm.check(ckmpm.mpm_ad_forward(ad.h, n, n, state.data_ptr(), logE.data_ptr(), out.data_ptr(), dt, stream),
                "mpm_ad_forward")
    return out


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, state0, logE, ad, nsteps, dt, every):
        stream = torch.cuda.current_stream()
        state0 = state0.detach().contiguous()
        logE = logE.detach().contiguous()
        checkpoints = [state0]
        st = state0
        for k in range(nsteps):
            st = _step(ad, st, logE, dt, stream)
            if (k + 1) % every == 0 and k + 1 < nsteps:
                checkpoints.append(st)
        ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream), "rollout forward")
        ctx.ad, ctx.nsteps, ctx.dt, ctx.every = ad, nsteps, dt, every
        ctx.save_for_backward(logE, *checkpoints)
        return st

    @staticmethod
    def backward(ctx, grad_out):
        stream = torch.cuda.current_stream()
        logE, *checkpoints = ctx.saved_tensors
        ad, nsteps, dt, every = ctx.ad, ctx.nsteps, ctx.dt, ctx.every
        n = logE.shape[0]
        cot = grad_out.contiguous().clone()
        logE_cot = torch.zeros_like(logE)
        for seg in range(len(checkpoints) - 1, -1, -1):
            first = seg * every
            length = min(every, nsteps - first)
            states = [checkpoints[seg]]
            for _ in range(length - 1):
                states.append(_step(ad, states[-1], logE, dt, stream))
            for j in range(length - 1, -1, -1):
                cot_in = torch.empty_like(cot)
                ckmpm.check(ckmpm.mpm_ad_backward(ad.h, n, n, states[j].data_ptr(), logE.data_ptr(), cot.data_ptr(),
                                                  cot_in.data_ptr(), logE_cot.data_ptr(), dt, stream),
                            "mpm_ad_backward")
                cot = cot_in
        ckmpm.check(ckmpm.mpm_ad_sync(ad.h, stream), "rollout backward")
        return cot, logE_cot, None, None, None, None


def rollout(ad: AdContext, state0: torch.Tensor, logE: torch.Tensor, nsteps: int, dt: float,
            checkpoint_every: int = 8) -> torch.Tensor:
    """State after `nsteps` steps from `state0` ((27, n) FP32 planes x, v, B, H, r on the
    GPU) with per-particle log modulus `logE` ((n,) FP32); differentiable with respect
    to both.  Memory: ceil(nsteps / checkpoint_every) saved states plus one segment."""
    if nsteps <= 0:
        return state0
    every = max(1, int(checkpoint_every))
    assert state0.dim() == 2 and state0.shape[0] == ckmpm.MPM_STATE_PLANES and state0.dtype == torch.float32
    assert logE.shape == (state0.shape[1],) and logE.dtype == torch.float32
    return _Rollout.apply(state0, logE, ad, int(nsteps), float(dt), every)


def planes(x: torch.Tensor, v: torch.Tensor, B: torch.Tensor, H: torch.Tensor) -> torch.Tensor:
    """(27, n) state from x, v (n, 3), B, H (n, 3, 3) (differentiable concatenation;
    the position remainder planes are zero)."""
    n = x.shape[0]
    r = torch.zeros((3, n), dtype=x.dtype, device=x.device)
    return torch.cat([x.t(), v.t(), B.reshape(n, 9).t(), H.reshape(n, 9).t(), r], dim=0).contiguous()
