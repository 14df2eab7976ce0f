"""Probe-energy objective as a differentiable PyTorch function.

J(eps_r, sigma) = dt * sum_{n<N} Hz_p(n+1/2)^2 of the coupled run (Sec. II-A
eqs. (3), (5) on the coarse grid, eq. (23) for every embedded model), with
the reduced models held fixed.  The forward pass runs the HIP library's
fdtd_rom_adjoint when a gradient is needed (one forward with checkpoints,
then the reverse sweep with per-segment recomputation) and a plain
fdtd_rom_run otherwise; backward only scales the stored gradients.  Cells
inside a reduced region or on its one-cell ring get zero gradient."""
from __future__ import annotations

import dataclasses

import numpy as np

from .sim import Simulation


def _problem_with(prob, eps_r, sigma):
    return dataclasses.replace(prob, eps_r=np.ascontiguousarray(eps_r, dtype=np.float64),
                               sigma=np.ascontiguousarray(sigma, dtype=np.float64))


def _function():
    import torch

    class ProbeEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, eps_r, sigma, prob, rom_mats, dtype, nsteps, probe, ckpt_every, device):
            p = _problem_with(prob, eps_r.detach().to("cpu", torch.float64).numpy(),
                              sigma.detach().to("cpu", torch.float64).numpy())
            nsteps = p.nsteps if nsteps is None else nsteps
            with Simulation(p, rom_mats, dtype=dtype, device=device) as sim:
                if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
                    J, ge, gs = sim.adjoint(nsteps, probe=probe, ckpt_every=ckpt_every)
                    ctx.save_for_backward(torch.from_numpy(ge).to(eps_r.device, eps_r.dtype),
                                          torch.from_numpy(gs).to(sigma.device, sigma.dtype))
                else:
                    sim.run(nsteps)
                    J = sim.objective(probe, 0, nsteps)
            return torch.tensor(J, dtype=torch.float64, device=eps_r.device)

        @staticmethod
        def backward(ctx, gJ):
            ge, gs = ctx.saved_tensors
            g = gJ.to(ge.dtype)
            return g * ge, g * gs, None, None, None, None, None, None, None

    return ProbeEnergy


_FN = None


def probe_energy(eps_r, sigma, prob, rom_mats, dtype=None, nsteps=None, probe=0, ckpt_every=0,
                 device="cuda:0"):
    """Differentiable J for per-cell maps eps_r, sigma (torch tensors [ny, nx])."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(eps_r, sigma, prob, rom_mats, dtype, nsteps, probe, ckpt_every, device)
