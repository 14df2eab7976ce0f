"""Whole coupled run: coarse Yee grid plus embedded reduced models
(paper Sec. IV last paragraph: conventional FDTD updates on the coarse grid,
eq. (23) for every reduced model), with the storage function of Sec. V and
the Appendix for the stability checks.

One step n -> n+1 (leap-frog, x^n = [E^n; H^{n-1/2}], eq. (7)):
  1. Hz^{n+1/2} on coarse cells outside every reduced region, then additive
     Hz source increments of step n;
  2. E^{n+1} on coarse edges that are neither on a PEC wall nor on/inside a
     reduced region, then additive E source increments of step n;
  3. every reduced model: gather the coarse Hz^{n+1/2} just outside its ports,
     advance (literal eq. (19) solve, or the closed form of eq. (23)) and write
     y^{n+1} into the interface edges;
  4. record probes (Hz^{n+1/2}, E^{n+1}).

Storage function (derived from eq. (6) with B = L S, eqs. (24)-(25)):
  energy^n = x_c^T R_c x_c + sum_r x~_r^T R~_r x~_r,
where R_c is the coarse grid's R of the same form as the fine model (edge
areas halved on interface edges, coupling only to coarse cells outside the
regions).  Source-free, energy^{n+1} - energy^n equals minus the dissipation
1/2 (x^{n+1}+x^n)^T (F+F^T) (x^{n+1}+x^n) exactly, because the coarse-side
supply (-Sc) and the model-side supply (+Sc) cancel at every interface
(Appendix, eq. (A7)).
"""
from __future__ import annotations

import numpy as np

from .constants import EPS0, MU0
from . import cpml, yee
from .coupling import RomCoupling
from .yee import EX, EY, HZ


class CoupledRun:
    def __init__(self, prob, roms, mode="literal", fp32=False, init=None, solver="lu"):
        """``roms``: list of dict(Rt, Ft, Lt) aligned with prob.roms.
        mode 'literal' solves eq. (19); 'closed' applies eq. (23).  With
        fp32=True the stencil coefficients and eq. (23)'s update matrix on
        [x~^n; h] are rounded to float32 first (what an FP32 run computes
        with) and the run proceeds in FP64 arithmetic."""
        self.prob = prob
        self.mode = mode
        nx, ny = prob.nx, prob.ny
        self.f = yee.CoarseFields(nx, ny)
        blocks = [(s.i0, s.j0, s.ni, s.nj) for s in prob.roms]
        self.cell, self.exm, self.eym = yee.masks(nx, ny, blocks, getattr(prob, "pec", None))
        (self.ca_x, self.cb_x, self.ca_y, self.cb_y, self.chdy,
         self.chdx) = yee.edge_coefficients(prob.eps_r, prob.sigma, prob.dt,
                                            prob.dx, prob.dy, fp32=fp32)
        self.cpl = []
        for spec, m in zip(prob.roms, roms):
            c = RomCoupling(m["Rt"], m["Ft"], m["Lt"], spec.i0, spec.j0, spec.ni,
                            spec.nj, prob.eps_r, prob.sigma, prob.dx, prob.dy,
                            prob.dt)
            A, B, C = c.closed_form(solver)
            c.Ac, c.Bc, c.Cc = A, B, C
            # an FP32 run rounds eq. (23)'s update matrix on [x~^n; h]
            c.G32 = (np.asarray(c.update_matrix(solver), np.float32).astype(np.float64)
                     if fp32 else None)
            self.cpl.append(c)
        self.x = [np.zeros(c.q) for c in self.cpl]
        pml = getattr(prob, "pml", None)
        self.pml = cpml.Cpml(prob, fp32) if (pml is not None and pml.any) else None
        if init is not None:
            self.f.hz[...] = init["hz"] * self.cell
            self.f.ex[...] = init["ex"] * self.exm
            self.f.ey[...] = init["ey"] * self.eym
            for k, c in enumerate(self.cpl):
                self.x[k] = init["x"][k].copy()
                c.scatter(self.f.ex, self.f.ey, c.Lt.T @ self.x[k])
        self.z = [c.z_from(c.read_y(self.f.ex, self.f.ey), x) for c, x in zip(self.cpl, self.x)]
        self.n = 0

    def step(self):
        p, f, n = self.prob, self.f, self.n
        if self.pml is None:
            yee.update_h(f, self.chdy, self.chdx, self.cell)
        else:
            self.pml.update_h(f, self.chdy, self.chdx, self.cell)
        yee.apply_sources(f, p.sources, (HZ,), n)
        if self.pml is None:
            yee.update_e(f, self.ca_x, self.cb_x, self.ca_y, self.cb_y, self.exm, self.eym)
        else:
            self.pml.update_e(f, self.ca_x, self.cb_x, self.ca_y, self.cb_y, self.exm, self.eym)
        yee.apply_sources(f, p.sources, (EX, EY), n)
        for k, c in enumerate(self.cpl):
            h = c.gather(f.hz)
            if self.mode == "literal":
                self.z[k] = c.step_literal(self.z[k], h)
                iy, iu, ix = c.sl
                self.x[k] = self.z[k][ix].copy()
                y = self.z[k][iy]
            elif c.G32 is not None:
                out = c.G32 @ np.concatenate([self.x[k], h])
                self.x[k] = out[:c.q]
                y = out[c.q:]
            else:
                self.x[k] = c.Ac @ self.x[k] + c.Bc @ h
                y = c.Cc @ self.x[k]
            c.scatter(f.ex, f.ey, y)
        self.n += 1

    def probes(self):
        out = np.empty(len(self.prob.probes))
        for k, pr in enumerate(self.prob.probes):
            out[k] = self.f.field(pr.comp)[pr.j, pr.i]
        return out

    # storage function ------------------------------------------------------
    def _edge_weights(self):
        """(eps-area/dt, sigma-area) per coarse E edge entering R_c / F_c."""
        p = self.prob
        nx, ny, dx, dy, dt = p.nx, p.ny, p.dx, p.dy, p.dt
        er, sg = p.eps_r, p.sigma
        wex = np.zeros((ny + 1, nx))
        sex = np.zeros((ny + 1, nx))
        wey = np.zeros((ny, nx + 1))
        sey = np.zeros((ny, nx + 1))
        A = dx * dy
        wex[1:ny, :] = A * EPS0 * 0.5 * (er[1:, :] + er[:-1, :]) / dt
        sex[1:ny, :] = A * 0.5 * (sg[1:, :] + sg[:-1, :])
        wey[:, 1:nx] = A * EPS0 * 0.5 * (er[:, 1:] + er[:, :-1]) / dt
        sey[:, 1:nx] = A * 0.5 * (sg[:, 1:] + sg[:, :-1])
        wex *= self.exm
        sex *= self.exm
        wey *= self.eym
        sey *= self.eym
        for c in self.cpl:
            for k, (comp, ei, ej, oi, oj, dl, dlh) in enumerate(c.ports):
                w = dl * dlh * EPS0 * er[oj, oi] / dt
                s = dl * dlh * sg[oj, oi]
                if comp == EX:
                    wex[ej, ei] = w
                    sex[ej, ei] = s
                else:
                    wey[ej, ei] = w
                    sey[ej, ei] = s
        return wex, sex, wey, sey

    def energy(self):
        p = self.prob
        if not hasattr(self, "_w"):
            self._w = self._edge_weights()
        wex, _, wey, _ = self._w
        f = self.f
        hz = f.hz * self.cell
        e = np.sum(wex * f.ex ** 2) + np.sum(wey * f.ey ** 2)
        e += np.sum(MU0 * p.dx * p.dy / p.dt * hz ** 2)
        # - E^T K H, K restricted to coarse cells outside the regions
        act_x = wex > 0
        act_y = wey > 0
        e -= np.sum(np.where(act_x, f.ex, 0.0) * self._kh_x(hz)) + \
            np.sum(np.where(act_y, f.ey, 0.0) * self._kh_y(hz))
        for c, x in zip(self.cpl, self.x):
            e += x @ (c.Rt @ x)
        return float(e)

    def _kh_x(self, hz):
        p = self.prob
        out = np.zeros((p.ny + 1, p.nx))
        out[:-1, :] += p.dx * hz   # edge (i, j) with cell (i, j) above it
        out[1:, :] -= p.dx * hz    # edge (i, j+1) with cell (i, j) below it
        return out

    def _kh_y(self, hz):
        p = self.prob
        out = np.zeros((p.ny, p.nx + 1))
        out[:, :-1] -= p.dy * hz   # edge (i, j) with cell (i, j) to its right
        out[:, 1:] += p.dy * hz    # edge (i+1, j) with cell (i, j) to its left
        return out

    def dissipation(self, prev_ex, prev_ey, prev_x):
        """1/2 (x^{n+1}+x^n)^T (F+F^T) (x^{n+1}+x^n) between a saved state and now."""
        if not hasattr(self, "_w"):
            self._w = self._edge_weights()
        _, sex, _, sey = self._w
        d = 0.5 * np.sum(sex * (self.f.ex + prev_ex) ** 2)
        d += 0.5 * np.sum(sey * (self.f.ey + prev_ey) ** 2)
        for c, x, x0 in zip(self.cpl, self.x, prev_x):
            s = x + x0
            d += 0.5 * s @ ((c.Ft + c.Ft.T) @ s)
        return float(d)


def run(prob, roms, nsteps=None, mode="literal", fp32=False, init=None,
        record_energy=False):
    """Probe series [nsteps, nprobes] (and the energy before each step)."""
    sim = CoupledRun(prob, roms, mode=mode, fp32=fp32, init=init)
    nsteps = prob.nsteps if nsteps is None else nsteps
    out = np.empty((nsteps, len(prob.probes)))
    energy = np.empty(nsteps + 1) if record_energy else None
    for n in range(nsteps):
        if record_energy:
            energy[n] = sim.energy()
        sim.step()
        out[n] = sim.probes()
    if record_energy:
        energy[nsteps] = sim.energy()
        return out, energy
    return out


def build_roms(prob, basis="sprim", clip=True, theta=0.99):
    """Oracle reduced models for every region of ``prob`` (shared models
    for regions with equal group >= 0 are built once)."""
    from .rom import build_rom
    out = []
    cache = {}
    for spec in prob.roms:
        key = spec.group if spec.group >= 0 else None
        if key is not None and key in cache:
            out.append(cache[key])
            continue
        m = build_rom(spec.eps_r, spec.sigma, spec.r, prob.dx, prob.dy, prob.dt,
                      spec.q, spec.f_max, basis=basis, clip=clip, theta=theta,
                      pec=getattr(spec, "pec", None))
        m = dict(Rt=m["Rt"], Ft=m["Ft"], Lt=m["Lt"], q1=m["q1"], q2=m["q2"],
                 clipped=m["clipped"], smax_before=m["smax_before"],
                 smax_after=m["smax_after"])
        if key is not None:
            cache[key] = m
        out.append(m)
    return out
