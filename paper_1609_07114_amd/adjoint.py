"""Probe-energy objective as a differentiable PyTorch function.

J(eps_r, sigma) = dt * sum_{n<N} Hz_p(n+1/2)^2 of the coupled run (Sec. II-A
eqs. (3), (5) on the coarse grid, eq. (23) for every embedded model), with
the reduced models held fixed.  The forward pass runs the HIP library's
fdtd_rom_adjoint when a gradient is needed (one forward with checkpoints,
then the reverse sweep with per-segment recomputation) and a plain
fdtd_rom_run otherwise; backward only scales the stored gradients.  Cells
inside a reduced region or on its one-cell ring get zero gradient.

probe_energy_models differentiates through the models as well: J of the
coarse maps and of every region's fine maps, the models rebuilt by the
library's builder at each call (gradients: fdtd_rom_adjoint_models and
fdtd_rom_build_vjp, the projection basis held at the one built)."""
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


def _model_function():
    import torch

    class ProbeEnergyModels(torch.autograd.Function):
        """J of the coupled run as a function of the coarse maps and of every
        region's fine maps: the models are built by the library from the
        fine maps at each call; the gradient holds the projection basis at
        the one built (fdtd_rom_adjoint_models, fdtd_rom_build_vjp)."""

        @staticmethod
        def forward(ctx, eps_r, sigma, prob, dtype, nsteps, probe, ckpt_every, device, *fine):
            from . import romgen
            cpu = lambda t: t.detach().to("cpu", torch.float64).numpy()
            nr = len(prob.roms)
            specs = [dataclasses.replace(s, eps_r=np.ascontiguousarray(cpu(fine[k])),
                                         sigma=np.ascontiguousarray(cpu(fine[nr + k])))
                     for k, s in enumerate(prob.roms)]
            p = dataclasses.replace(_problem_with(prob, cpu(eps_r), cpu(sigma)), roms=specs)
            nsteps = p.nsteps if nsteps is None else nsteps
            grad = any(ctx.needs_input_grad)
            mats = romgen.build_roms(p, keep=grad)   # builder states for the gradient, no rebuild
            with Simulation(p, mats, dtype=dtype, device=device) as sim:
                if grad:
                    J, ge, gs, models = sim.adjoint_models(nsteps, probe=probe, ckpt_every=ckpt_every)
                    fe, fs = [], []
                    for k, (a, b) in enumerate(romgen.build_vjps(p, models, roms=mats)):
                        fe.append(torch.from_numpy(a).to(fine[k].device, fine[k].dtype))
                        fs.append(torch.from_numpy(b).to(fine[nr + k].device, fine[nr + k].dtype))
                    ctx.save_for_backward(torch.from_numpy(ge).to(eps_r.device, eps_r.dtype),
                                          torch.from_numpy(gs).to(sigma.device, sigma.dtype), *fe, *fs)
                else:
                    sim.run(nsteps)
                    J = sim.objective(probe, 0, nsteps)
            return torch.tensor(J, dtype=torch.float64, device=eps_r.device)

        @staticmethod
        def backward(ctx, gJ):
            saved = ctx.saved_tensors
            g = gJ.to(saved[0].dtype)
            return (g * saved[0], g * saved[1], None, None, None, None, None, None) + tuple(g * t for t in saved[2:])

    return ProbeEnergyModels


_FN = None
_FN_MODELS = None


def probe_energy_models(eps_r, sigma, fine_eps_r, fine_sigma, prob, dtype=None, nsteps=None, probe=0,
                        ckpt_every=0, device="cuda:0"):
    """Differentiable J for the coarse maps eps_r, sigma ([ny, nx] tensors)
    and every region's fine maps (lists of [r*nj, r*ni] tensors, in the
    order of prob.roms): models rebuilt from the fine maps by the library at
    each call, gradients through eq. (23), the ring cells' half cells and
    the builder (basis held)."""
    global _FN_MODELS
    if _FN_MODELS is None:
        _FN_MODELS = _model_function()
    return _FN_MODELS.apply(eps_r, sigma, prob, dtype, nsteps, probe, ckpt_every, device,
                            *fine_eps_r, *fine_sigma)


def probe_energy(eps_r, sigma, prob, rom_mats, dtype=None, nsteps=None, probe=0, ckpt_every=0,
                 device="cuda:0"):
    """Differentiable J for per-cell maps eps_r, sigma (torch tensors [ny, nx])."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(eps_r, sigma, prob, rom_mats, dtype, nsteps, probe, ckpt_every, device)
