"""Convolutional PML (CPML) layers on the coarse grid - test infrastructure.

Not in the paper: its waveguide and reflection experiments (Sec. VI-B,
VI-C) terminate the guide with perfectly matched layers without giving
equations.  The layers here are the stretched-coordinate PML in recursive
convolution form (Roden and Gedney, "Convolution PML (CPML)", Microwave
Opt. Technol. Lett. 27, 2000), written on the TEz Yee grid of eqs. (3), (5):

  d/dx -> (1/kappa_x) d/dx + psi_x,  psi_x^{new} = b_x psi_x + a_x (d/dx)^{new}
  b = exp(-(sigma/kappa + alpha) dt/eps0),
  a = sigma (b - 1) / (sigma kappa + kappa^2 alpha)   (0 where sigma = 0),

with the auxiliary psi stored multiplied by the cell size, so that with the
raw differences dF of the Yee update
  psi~' = b psi~ + a dF,   curl term = (1/kappa) dF + psi~'.
Grading inside a layer of D cells, rho = depth/D in (0, 1]:
  sigma = sigma_max rho^m, kappa = 1 + (kappa_max - 1) rho^m,
  alpha = alpha_max (1 - rho),  sigma_max = scale * 0.8 (m + 1) / (eta0 d).
E samples sit at k d, Hz samples at (k + 1/2) d.  Outside the layers
kappa = 1, a = 0, b = 1 and psi stays zero: the update is eqs. (3), (5).

Parity: pinned by exact reduction to the plain update when sigma = 0 and
kappa = 1, by the reflection of a pulse against a domain large enough to
show none, and by the decay of the stored energy after the pulse has left.
"""
from __future__ import annotations

import numpy as np

from .constants import C0, EPS0, MU0

ETA0 = MU0 * C0


def axis_profiles(n, d, dt, n_lo, n_hi, m, sigma_scale, kappa_max, alpha_max, fp32=False):
    """(ik_e, b_e, a_e) at E samples k d (k = 0..n) and (ik_h, b_h, a_h) at Hz
    samples (k + 1/2) d (k = 0..n-1) along one axis of n cells."""
    length = n * d
    d_lo = n_lo * d
    d_hi = n_hi * d
    sigma_max = sigma_scale * 0.8 * (m + 1.0) / (ETA0 * d)

    def coeffs(x):
        rho = np.zeros_like(x)
        if n_lo > 0:
            lo = x < d_lo
            rho[lo] = (d_lo - x[lo]) / d_lo
        if n_hi > 0:
            hi = x > length - d_hi
            rho[hi] = (x[hi] - (length - d_hi)) / d_hi
        inside = rho > 0
        sigma = np.where(inside, sigma_max * rho ** m, 0.0)
        kappa = np.where(inside, 1.0 + (kappa_max - 1.0) * rho ** m, 1.0)
        alpha = np.where(inside, alpha_max * (1.0 - rho), 0.0)
        b = np.exp(-(sigma / kappa + alpha) * dt / EPS0)
        denom = sigma * kappa + kappa ** 2 * alpha
        a = np.where(sigma > 0, sigma * (b - 1.0) / np.where(denom > 0, denom, 1.0), 0.0)
        ik = 1.0 / kappa
        if fp32:
            ik, b, a = (np.asarray(v, np.float32).astype(np.float64) for v in (ik, b, a))
        return ik, b, a

    xe = np.arange(n + 1) * d
    xh = (np.arange(n) + 0.5) * d
    return coeffs(xe) + coeffs(xh)


class Cpml:
    """Profiles and auxiliary state of the four possible layers."""

    def __init__(self, prob, fp32=False):
        p = prob.pml
        (self.ikx_e, self.bx_e, self.ax_e, self.ikx_h, self.bx_h, self.ax_h) = axis_profiles(
            prob.nx, prob.dx, prob.dt, p.n_xlo, p.n_xhi, p.m, p.sigma_scale, p.kappa_max,
            p.alpha_max, fp32)
        (self.iky_e, self.by_e, self.ay_e, self.iky_h, self.by_h, self.ay_h) = axis_profiles(
            prob.ny, prob.dy, prob.dt, p.n_ylo, p.n_yhi, p.m, p.sigma_scale, p.kappa_max,
            p.alpha_max, fp32)
        ny, nx = prob.ny, prob.nx
        self.psi_hx = np.zeros((ny, nx))       # d/dx of Ey at Hz
        self.psi_hy = np.zeros((ny, nx))       # d/dy of Ex at Hz
        self.psi_ex = np.zeros((ny + 1, nx))   # d/dy of Hz at Ex
        self.psi_ey = np.zeros((ny, nx + 1))   # d/dx of Hz at Ey

    def update_h(self, f, chdy, chdx, cell_mask):
        """Hz^{n-1/2} -> Hz^{n+1/2} (eq. (5) with stretched derivatives)."""
        dex = f.ex[1:, :] - f.ex[:-1, :]
        dey = f.ey[:, 1:] - f.ey[:, :-1]
        self.psi_hy = self.by_h[:, None] * self.psi_hy + self.ay_h[:, None] * dex
        self.psi_hx = self.bx_h[None, :] * self.psi_hx + self.ax_h[None, :] * dey
        curl = (chdy * (self.iky_h[:, None] * dex + self.psi_hy)
                - chdx * (self.ikx_h[None, :] * dey + self.psi_hx))
        f.hz += np.where(cell_mask, curl, 0.0)

    def update_e(self, f, ca_x, cb_x, ca_y, cb_y, ex_mask, ey_mask):
        """E^n -> E^{n+1} on active edges (eq. (3) with stretched derivatives)."""
        ny, nx = f.ny, f.nx
        dhx = np.zeros((ny + 1, nx))
        dhx[1:ny, :] = f.hz[1:, :] - f.hz[:-1, :]
        dhy = np.zeros((ny, nx + 1))
        dhy[:, 1:nx] = f.hz[:, 1:] - f.hz[:, :-1]
        self.psi_ex = np.where(ex_mask, self.by_e[:, None] * self.psi_ex + self.ay_e[:, None] * dhx,
                               self.psi_ex)
        self.psi_ey = np.where(ey_mask, self.bx_e[None, :] * self.psi_ey + self.ax_e[None, :] * dhy,
                               self.psi_ey)
        new_ex = ca_x * f.ex + cb_x * (self.iky_e[:, None] * dhx + self.psi_ex)
        new_ey = ca_y * f.ey - cb_y * (self.ikx_e[None, :] * dhy + self.psi_ey)
        f.ex[...] = np.where(ex_mask, new_ex, f.ex)
        f.ey[...] = np.where(ey_mask, new_ey, f.ey)
