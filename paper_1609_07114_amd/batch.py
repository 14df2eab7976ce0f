"""Batch handle: B independent problems in one device workspace (PyTorch
tensor), advanced together by the HIP library (capi.fdtd_rom_batch_*)."""
from __future__ import annotations

from . import capi


class Batch:
    def __init__(self, probs, rom_mats, max_steps=None, dtype=None, device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required (torch.cuda.is_available() is False)")
        if len(probs) != len(rom_mats):
            raise ValueError("one list of reduced models per problem")
        self.torch = torch
        self.probs = list(probs)
        self.structs = [capi.ProblemStruct.from_workload(p, m, max_steps=max_steps, dtype=dtype)
                        for p, m in zip(probs, rom_mats)]
        self.nbytes = capi.fdtd_rom_batch_workspace_size(self.structs)
        self.device = torch.device(device)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = capi.fdtd_rom_batch_create(self.structs, self.ws.data_ptr(), self.nbytes,
                                            self.stream.cuda_stream)
        self.tiling = [16] * len(self.probs)

    def __len__(self):
        return len(self.probs)

    def run(self, nsteps):
        capi.fdtd_rom_batch_run(self.h, nsteps)

    @property
    def steps_done(self):
        return capi.fdtd_rom_batch_steps_done(self.h)

    def probes(self, b, first=0, count=None):
        if count is None:
            count = self.steps_done - first
        return capi.fdtd_rom_batch_read_probes(self.h, b, first, count, len(self.probs[b].probes))

    def field(self, b, comp):
        p = self.probs[b]
        return capi.fdtd_rom_batch_read_field(self.h, b, comp, p.nx, p.ny)

    def set_tiling(self, b, seg):
        """Rows per stencil wave of instance b (all instances for b = -1)."""
        capi.fdtd_rom_batch_set_tiling(self.h, b, seg)
        if b < 0:
            self.tiling = [seg] * len(self.probs)
        else:
            self.tiling[b] = seg

    def set_graph(self, steps):
        capi.fdtd_rom_batch_set_graph(self.h, steps)

    def set_pair_split(self, b, percent):
        """Far tiles' share (percent) in a pair's second launch, instance b
        (all instances for b = -1; -1 percent restores the default)."""
        capi.fdtd_rom_batch_set_pair_split(self.h, b, percent)

    def set_time_blocking(self, on):
        capi.fdtd_rom_batch_set_time_blocking(self.h, on)

    def time_blocking(self):
        return capi.fdtd_rom_batch_get_time_blocking(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            self.stream.synchronize()
            capi.fdtd_rom_batch_destroy(self.h)
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
