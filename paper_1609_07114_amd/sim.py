"""Simulation handle: device workspace from PyTorch, stream from PyTorch,
every computation in the HIP library (capi)."""
from __future__ import annotations

import numpy as np

from . import capi


class Simulation:
    def __init__(self, prob, rom_mats, max_steps=None, dtype=None, x0=None, device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required (torch.cuda.is_available() is False)")
        self.torch = torch
        self.prob = prob
        self.ps = capi.ProblemStruct.from_workload(prob, rom_mats, max_steps=max_steps,
                                                   dtype=dtype, x0=x0)
        self.nbytes = capi.fdtd_rom_workspace_size(self.ps)
        self.device = torch.device(device)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = capi.fdtd_rom_create(self.ps, self.ws.data_ptr(), self.nbytes,
                                      self.stream.cuda_stream)
        self.nprobes = len(prob.probes)
        self.q = [m["Rt"].shape[0] for m in rom_mats]

    def run(self, nsteps):
        capi.fdtd_rom_run(self.h, nsteps)

    def step(self):
        capi.fdtd_rom_step(self.h)

    def prepare_run(self, nsteps):
        """Set-up (tile roles, graph capture) of the next run(nsteps), no step."""
        capi.fdtd_rom_prepare_run(self.h, nsteps)

    def set_check_interval(self, every):
        capi.fdtd_rom_set_check_interval(self.h, every)

    def check_interval(self):
        return capi.fdtd_rom_get_check_interval(self.h)

    @property
    def steps_done(self):
        return capi.fdtd_rom_steps_done(self.h)

    def probes(self, first=0, count=None):
        if count is None:
            count = self.steps_done - first
        return capi.fdtd_rom_read_probes(self.h, first, count, self.nprobes)

    def objective(self, probe=0, first=0, count=None):
        """J = dt * sum over recorded rows of Hz_probe^2 (the adjoint's objective)."""
        if count is None:
            count = self.steps_done - first
        return capi.fdtd_rom_probe_objective(self.h, probe, first, count)

    def field(self, comp):
        return capi.fdtd_rom_read_field(self.h, comp, self.prob.nx, self.prob.ny)

    def rom_state(self, k):
        return capi.fdtd_rom_read_rom_state(self.h, k, self.q[k])

    def energy(self):
        """Discrete energy of the current state (Theorem 2 storage function)."""
        return capi.fdtd_rom_energy(self.h)

    def get_state(self):
        """Device tensor (uint8) holding the current state."""
        n = capi.fdtd_rom_state_size(self.h)
        buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        capi.fdtd_rom_get_state(self.h, buf.data_ptr())
        return buf

    def set_state(self, buf):
        if buf.device != self.device or buf.dtype != self.torch.uint8:
            raise ValueError("state must be a uint8 tensor on the simulation's device")
        if buf.numel() < capi.fdtd_rom_state_size(self.h):
            raise ValueError("state tensor too small")
        capi.fdtd_rom_set_state(self.h, buf.data_ptr())

    def coupled_update(self, k):
        return capi.fdtd_rom_coupled_update(self.ps, k)

    def set_tiling(self, seg):
        capi.fdtd_rom_set_tiling(self.h, seg)

    def get_tiling(self):
        return capi.fdtd_rom_get_tiling(self.h)

    def set_shared_gemm(self, enable):
        capi.fdtd_rom_set_shared_gemm(self.h, enable)

    def set_material_mode(self, mode):
        capi.fdtd_rom_set_material_mode(self.h, mode)

    def material_mode(self):
        return capi.fdtd_rom_get_material_mode(self.h)

    def set_graph(self, batch):
        capi.fdtd_rom_set_graph(self.h, batch)

    def set_time_blocking(self, on):
        capi.fdtd_rom_set_time_blocking(self.h, on)

    def time_blocking(self):
        return capi.fdtd_rom_get_time_blocking(self.h)

    def set_pair_split(self, percent):
        capi.fdtd_rom_set_pair_split(self.h, percent)

    def pair_split(self):
        return capi.fdtd_rom_get_pair_split(self.h)

    def adjoint(self, nsteps=None, probe=0, ckpt_every=0):
        """Forward run from the initial state plus the reverse sweep:
        (J, dJ/deps_r, dJ/dsigma) for J = dt * sum_n Hz_probe(n+1/2)^2."""
        nsteps = self.prob.nsteps if nsteps is None else nsteps
        nb = capi.fdtd_rom_adjoint_workspace_size(self.h, nsteps, ckpt_every)
        aws = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
        try:
            return capi.fdtd_rom_adjoint(self.h, nsteps, ckpt_every, probe, aws.data_ptr(), nb,
                                         self.prob.nx, self.prob.ny)
        finally:
            self.stream.synchronize()
            del aws

    def adjoint_models(self, nsteps=None, probe=0, ckpt_every=0):
        """The reverse sweep with the gradients through the reduced models:
        (J, dJ/deps_r, dJ/dsigma, [dict(Rt, Ft, Lt) of dJ/d(matrix)] per
        region); the coarse maps include the ring cells' eq. (13) share."""
        nsteps = self.prob.nsteps if nsteps is None else nsteps
        nb = capi.fdtd_rom_adjoint_models_workspace_size(self.h, nsteps, ckpt_every)
        aws = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
        shapes = [(s.q, s.n_ports) for s in self.prob.roms]
        try:
            return capi.fdtd_rom_adjoint_models(self.h, nsteps, ckpt_every, probe, aws.data_ptr(), nb,
                                                self.prob.nx, self.prob.ny, shapes)
        finally:
            self.stream.synchronize()
            del aws

    def profile(self, enable=True):
        capi.fdtd_rom_profile_enable(self.h, enable)

    def profile_read(self):
        return capi.fdtd_rom_profile_read(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            self.stream.synchronize()
            capi.fdtd_rom_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
