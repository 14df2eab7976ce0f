"""Reduced models for every refined region of a problem, built by the
library's host FP64 builder (fdtd_rom_build), regions in parallel threads
(the ctypes call releases the GIL).  Regions sharing a group >= 0 are built
once."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

from . import capi


def build_roms(prob, theta=0.99, clip=True, workers=None, basis="sprim", keep=False):
    """Every region's model (regions of one group share one build), in
    parallel threads.  keep: SPRIM builds also keep the builder's state
    (model dict key 'state') for build_vjp without a rebuild."""
    jobs = []
    slot = {}
    order = []
    for k, spec in enumerate(prob.roms):
        key = ("g", spec.group) if spec.group >= 0 else ("r", k)
        if key not in slot:
            slot[key] = len(jobs)
            jobs.append(spec)
        order.append(slot[key])

    def one(spec):
        if keep and basis == "sprim":
            return capi.fdtd_rom_build_keep(spec.ni, spec.nj, spec.r, prob.dx, prob.dy, prob.dt,
                                            spec.eps_r, spec.sigma, spec.q, spec.f_max, theta, clip,
                                            getattr(spec, "pec", None))
        return capi.fdtd_rom_build(spec.ni, spec.nj, spec.r, prob.dx, prob.dy, prob.dt,
                                   spec.eps_r, spec.sigma, spec.q, spec.f_max, theta, clip, basis,
                                   getattr(spec, "pec", None))
    workers = workers or min(len(jobs), max(1, min(16, os.cpu_count() or 1))) or 1
    if len(jobs) <= 1:
        built = [one(s) for s in jobs]
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            built = list(ex.map(one, jobs))
    return [built[i] for i in order]


def build_roms_many(probs, theta=0.99, clip=True, workers=None):
    """build_roms for a list of problems, every region of every problem in
    one thread pool."""
    jobs = []
    for b, prob in enumerate(probs):
        for spec in prob.roms:
            jobs.append((prob, spec))

    def one(job):
        prob, spec = job
        return capi.fdtd_rom_build(spec.ni, spec.nj, spec.r, prob.dx, prob.dy, prob.dt,
                                   spec.eps_r, spec.sigma, spec.q, spec.f_max, theta, clip,
                                   "sprim", getattr(spec, "pec", None))
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        built = list(ex.map(one, jobs))
    out, k = [], 0
    for prob in probs:
        out.append(built[k:k + len(prob.roms)])
        k += len(prob.roms)
    return out


def build_vjp(prob, k, grad_Rt, grad_Ft, theta=0.99, clip=True, basis="sprim", state=None):
    """Gradient of J with respect to region k's fine-cell eps_r and sigma
    ([r*nj, r*ni] each) from dJ/dR~ and dJ/dF~ of the model build_roms makes
    for it (the library's builder, its projection basis held).  state: the
    builder state build_roms(keep=True) kept for this region's model (no
    rebuild); else the model is rebuilt from prob."""
    if state is not None:
        return capi.fdtd_rom_model_state_vjp(state, grad_Rt, grad_Ft)
    spec = prob.roms[k]
    return capi.fdtd_rom_build_vjp(spec.ni, spec.nj, spec.r, prob.dx, prob.dy, prob.dt, spec.eps_r,
                                   spec.sigma, spec.q, spec.f_max, grad_Rt, grad_Ft, theta, clip, basis,
                                   getattr(spec, "pec", None))


def build_vjps(prob, model_grads, theta=0.99, clip=True, basis="sprim", workers=None, roms=None):
    """build_vjp for every region (model_grads: per region a dict with Rt
    and Ft gradients, as Simulation.adjoint_models returns), regions in
    parallel threads.  roms: the models of build_roms(keep=True), whose kept
    states spare the rebuilds; without them each call rebuilds its model."""
    n = len(prob.roms)
    st = lambda k: roms[k].get("state") if roms is not None else None
    one = lambda k: build_vjp(prob, k, model_grads[k]["Rt"], model_grads[k]["Ft"], theta, clip, basis, st(k))
    workers = workers or min(n, max(1, min(16, os.cpu_count() or 1))) or 1
    if n <= 1:
        return [one(k) for k in range(n)]
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, range(n)))
