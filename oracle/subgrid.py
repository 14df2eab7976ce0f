"""Direct subgridding with the paper's interface rule, coded from the Yee
integral form without any descriptor system, projection or coupling matrix.

Each refined region carries explicit fine fields (cells dx/r, dy/r, eq. (2)).
Its boundary E equals the coarse interface E (eq. (15)); the coarse hanging
variable is the mean of the fine ones (eq. (16)).  Adding eq. (13) to the r
fine boundary rows of eq. (4) eliminates the hanging variables, which leaves
one update per coarse interface edge over its merged dual cell (coarse half
cell outside, r fine half cells inside), e.g. on a South edge:
  [dx dy/2 (e_c/dt + s_c/2) + sum_f dxh dyh/2 (e_f/dt + s_f/2)] y^{n+1}
     = [same with -] y^n + dxh * sum_f Hfine(f, 0) - dx * Hcoarse_below.
The embedded-model path with an identity basis must reproduce this run to
round-off (for r = 1 it is plain Yee on the whole grid).

Parity: this module *is* a pin for the coupling code; it is itself checked
by reducing to plain Yee when r = 1 and by its energy balance.
"""
from __future__ import annotations

import numpy as np

from .constants import EPS0, MU0
from . import yee
from .yee import EX, EY, HZ


class _Region:
    def __init__(self, spec, prob):
        self.s = spec
        r = spec.r
        self.Nx, self.Ny = r * spec.ni, r * spec.nj
        self.dxh, self.dyh = prob.dx / r, prob.dy / r
        self.hz = np.zeros((self.Ny, self.Nx))
        self.ex = np.zeros((self.Ny + 1, self.Nx))
        self.ey = np.zeros((self.Ny, self.Nx + 1))
        e, s = spec.eps_r, spec.sigma
        dt = prob.dt
        # interior fine edge coefficients (eq. (3))
        ee = EPS0 * 0.5 * (e[1:, :] + e[:-1, :]); ss = 0.5 * (s[1:, :] + s[:-1, :])
        self.ca_x = (ee / dt - ss / 2) / (ee / dt + ss / 2)
        self.cb_x = 1.0 / (ee / dt + ss / 2) / self.dyh
        ee = EPS0 * 0.5 * (e[:, 1:] + e[:, :-1]); ss = 0.5 * (s[:, 1:] + s[:, :-1])
        self.ca_y = (ee / dt - ss / 2) / (ee / dt + ss / 2)
        self.cb_y = 1.0 / (ee / dt + ss / 2) / self.dxh


def run(prob, nsteps=None):
    nsteps = prob.nsteps if nsteps is None else nsteps
    nx, ny, dx, dy, dt = prob.nx, prob.ny, prob.dx, prob.dy, prob.dt
    f = yee.CoarseFields(nx, ny)
    blocks = [(s.i0, s.j0, s.ni, s.nj) for s in prob.roms]
    cell, exm, eym = yee.masks(nx, ny, blocks)
    ca_x, cb_x, ca_y, cb_y, chdy, chdx = yee.edge_coefficients(
        prob.eps_r, prob.sigma, dt, dx, dy)
    regs = [_Region(s, prob) for s in prob.roms]
    out = np.empty((nsteps, len(prob.probes)))
    er, sg = prob.eps_r, prob.sigma
    for n in range(nsteps):
        yee.update_h(f, chdy, chdx, cell)
        for g in regs:
            g.hz += dt / MU0 * ((g.ex[1:, :] - g.ex[:-1, :]) / g.dyh
                                - (g.ey[:, 1:] - g.ey[:, :-1]) / g.dxh)
        yee.apply_sources(f, prob.sources, (HZ,), n)
        yee.update_e(f, ca_x, cb_x, ca_y, cb_y, exm, eym)
        yee.apply_sources(f, prob.sources, (EX, EY), n)
        for g in regs:
            s = g.s
            r = s.r
            fe, fs = s.eps_r, s.sigma
            # fine interior edges
            g.ex[1:-1, :] = g.ca_x * g.ex[1:-1, :] + g.cb_x * (g.hz[1:, :] - g.hz[:-1, :])
            g.ey[:, 1:-1] = g.ca_y * g.ey[:, 1:-1] - g.cb_y * (g.hz[:, 1:] - g.hz[:, :-1])
            # merged interface edges
            for c in range(s.ni):
                fi = slice(c * r, (c + 1) * r)
                for side in ("S", "N"):
                    if side == "S":
                        ej, oj, frow = s.j0, s.j0 - 1, 0
                    else:
                        ej, oj, frow = s.j0 + s.nj, s.j0 + s.nj, g.Ny - 1
                    ei = s.i0 + c
                    wp = dx * dy / 2 * (EPS0 * er[oj, ei] / dt + sg[oj, ei] / 2)
                    wm = dx * dy / 2 * (EPS0 * er[oj, ei] / dt - sg[oj, ei] / 2)
                    wp += np.sum(g.dxh * g.dyh / 2 * (EPS0 * fe[frow, fi] / dt + fs[frow, fi] / 2))
                    wm += np.sum(g.dxh * g.dyh / 2 * (EPS0 * fe[frow, fi] / dt - fs[frow, fi] / 2))
                    hf = g.dxh * np.sum(g.hz[frow, fi])
                    hc = dx * f.hz[oj, ei]
                    rhs = wm * f.ex[ej, ei] + (hf - hc if side == "S" else hc - hf)
                    f.ex[ej, ei] = rhs / wp
            for c in range(s.nj):
                fj = slice(c * r, (c + 1) * r)
                for side in ("W", "E"):
                    if side == "W":
                        ei, oi, fcol = s.i0, s.i0 - 1, 0
                    else:
                        ei, oi, fcol = s.i0 + s.ni, s.i0 + s.ni, g.Nx - 1
                    ej = s.j0 + c
                    wp = dy * dx / 2 * (EPS0 * er[ej, oi] / dt + sg[ej, oi] / 2)
                    wm = dy * dx / 2 * (EPS0 * er[ej, oi] / dt - sg[ej, oi] / 2)
                    wp += np.sum(g.dyh * g.dxh / 2 * (EPS0 * fe[fj, fcol] / dt + fs[fj, fcol] / 2))
                    wm += np.sum(g.dyh * g.dxh / 2 * (EPS0 * fe[fj, fcol] / dt - fs[fj, fcol] / 2))
                    hf = g.dyh * np.sum(g.hz[fj, fcol])
                    hc = dy * f.hz[ej, oi]
                    # -dHz/dx over the merged cell: -(H_right - H_left)
                    rhs = wm * f.ey[ej, ei] + (hc - hf if side == "W" else hf - hc)
                    f.ey[ej, ei] = rhs / wp
            # fine boundary E = coarse interface E (eq. (15))
            for c in range(s.ni):
                g.ex[0, c * r:(c + 1) * r] = f.ex[s.j0, s.i0 + c]
                g.ex[g.Ny, c * r:(c + 1) * r] = f.ex[s.j0 + s.nj, s.i0 + c]
            for c in range(s.nj):
                g.ey[c * r:(c + 1) * r, 0] = f.ey[s.j0 + c, s.i0]
                g.ey[c * r:(c + 1) * r, g.Nx] = f.ey[s.j0 + c, s.i0 + s.ni]
        for k, pr in enumerate(prob.probes):
            out[n, k] = f.field(pr.comp)[pr.j, pr.i]
    return out
