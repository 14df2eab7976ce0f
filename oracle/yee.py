"""Coarse TEz Yee grid (paper Sec. I eq. (1), Sec. II-A eqs. (3) and (5)).

Field layout (natural, wall edges included):
  Hz[j, i]  j < ny,  i < nx     cell centres
  Ex[j, i]  j <= ny, i < nx     horizontal edges y = j*dy
  Ey[j, i]  j < ny,  i <= nx    vertical edges x = i*dx
PEC walls: Ex[0,:], Ex[ny,:], Ey[:,0], Ey[:,nx] stay zero.

Update, divided through by the cell areas of eqs. (3) and (5):
  Hz^{n+1/2} = Hz^{n-1/2} + dt/mu0 * [(Ex(j+1)-Ex(j))/dy - (Ey(i+1)-Ey(i))/dx]
  Ex^{n+1}   = Ca*Ex^n + Cb/dy * (Hz(j) - Hz(j-1))
  Ey^{n+1}   = Ca*Ey^n - Cb/dx * (Hz(i) - Hz(i-1))
with Ca = (eps/dt - sigma/2)/(eps/dt + sigma/2), Cb = 1/(eps/dt + sigma/2),
eps and sigma the averages over the two cells sharing the edge (eq. (3)).

Two coefficient models:
  * FP64: the formula above in double precision.
  * FP32 run: the coefficients an FP32 run uses are defined as float32
    quantities: per cell a = f32(eps0*eps_r/dt), b = f32(sigma/2); per edge
    s = f32(a1+a2), t = f32(b1+b2), rcp = f32(1/f32(s+t)),
    Ca = f32(f32(s-t)*rcp), Cb/dy = f32(f32(2/dy)*rcp).  Algebraically equal
    to the FP64 formula; the oracle evaluates an FP32 run in FP64 arithmetic
    with exactly these rounded coefficients.

Parity: pinned by the discrete-dispersion eigenvalues of a small cavity,
the CFL boundary of eq. (1), PEC resonances and the exact energy balance.
"""
from __future__ import annotations

import numpy as np

from .constants import EPS0, MU0

HZ, EX, EY = 0, 1, 2


def _f32(x):
    return np.asarray(x, dtype=np.float32)


def edge_coefficients(eps_r, sigma, dt, dx, dy, fp32=False):
    """Return (ca_x, cbdy_x, ca_y, cbdx_y, chdy, chdx) as float64 arrays.

    ca_x, cbdy_x: [ny+1, nx] (rows 0 and ny unused); ca_y, cbdx_y:
    [ny, nx+1] (columns 0 and nx unused).  chdy = dt/(mu0*dy) multiplies the
    Ex difference in the Hz update, chdx = dt/(mu0*dx) the Ey difference."""
    eps_r = np.asarray(eps_r, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    ny, nx = eps_r.shape
    ca_x = np.zeros((ny + 1, nx))
    cb_x = np.zeros((ny + 1, nx))
    ca_y = np.zeros((ny, nx + 1))
    cb_y = np.zeros((ny, nx + 1))
    if not fp32:
        # eq. (3): edge eps, sigma = mean of the two adjacent cells
        ex_eps = EPS0 * 0.5 * (eps_r[1:, :] + eps_r[:-1, :])
        ex_sig = 0.5 * (sigma[1:, :] + sigma[:-1, :])
        ey_eps = EPS0 * 0.5 * (eps_r[:, 1:] + eps_r[:, :-1])
        ey_sig = 0.5 * (sigma[:, 1:] + sigma[:, :-1])
        for (eps, sig, ca, cb, d, sl) in (
                (ex_eps, ex_sig, ca_x, cb_x, dy, (slice(1, ny), slice(None))),
                (ey_eps, ey_sig, ca_y, cb_y, dx, (slice(None), slice(1, nx)))):
            num = eps / dt - sig / 2.0
            den = eps / dt + sig / 2.0
            ca[sl] = num / den
            cb[sl] = 1.0 / den / d
        chdy = dt / (MU0 * dy)
        chdx = dt / (MU0 * dx)
        return ca_x, cb_x, ca_y, cb_y, chdy, chdx
    # FP32 coefficient model (see module docstring)
    a = _f32(EPS0 * eps_r / dt)
    b = _f32(sigma / 2.0)
    two_dy = np.float32(2.0 / dy)
    two_dx = np.float32(2.0 / dx)
    one = np.float32(1.0)
    for (a1, a2, b1, b2, ca, cb, k, sl) in (
            (a[:-1, :], a[1:, :], b[:-1, :], b[1:, :], ca_x, cb_x, two_dy,
             (slice(1, ny), slice(None))),
            (a[:, :-1], a[:, 1:], b[:, :-1], b[:, 1:], ca_y, cb_y, two_dx,
             (slice(None), slice(1, nx)))):
        s = a1 + a2
        t = b1 + b2
        rcp = one / (s + t)
        ca[sl] = ((s - t) * rcp).astype(np.float64)
        cb[sl] = (k * rcp).astype(np.float64)
    chdy = float(np.float32(dt / (MU0 * dy)))
    chdx = float(np.float32(dt / (MU0 * dx)))
    return ca_x, cb_x, ca_y, cb_y, chdy, chdx


def masks(nx, ny, blocks, pec=None):
    """Active cells / edges of the coarse grid.

    ``blocks``: iterable of (i0, j0, ni, nj) reduced regions; ``pec``:
    [ny, nx] bool of perfectly conducting cells, or None.  A cell is active
    outside every block and every PEC cell (a PEC cell's Hz stays zero).  An
    edge is active when it is not on a PEC wall, not on a side of a PEC cell
    (zero tangential E) and neither inside nor on the boundary of a block
    (boundary edges are the interface E, written by the reduced-model
    update)."""
    cell = np.ones((ny, nx), dtype=bool)
    ex = np.zeros((ny + 1, nx), dtype=bool)
    ey = np.zeros((ny, nx + 1), dtype=bool)
    ex[1:ny, :] = True
    ey[:, 1:nx] = True
    for (i0, j0, ni, nj) in blocks:
        cell[j0:j0 + nj, i0:i0 + ni] = False
        ex[j0:j0 + nj + 1, i0:i0 + ni] = False
        ey[j0:j0 + nj, i0:i0 + ni + 1] = False
    if pec is not None:
        pec = np.asarray(pec, dtype=bool)
        cell &= ~pec
        ex[:-1, :] &= ~pec
        ex[1:, :] &= ~pec
        ey[:, :-1] &= ~pec
        ey[:, 1:] &= ~pec
    return cell, ex, ey


class CoarseFields:
    def __init__(self, nx, ny):
        self.nx, self.ny = nx, ny
        self.hz = np.zeros((ny, nx))
        self.ex = np.zeros((ny + 1, nx))
        self.ey = np.zeros((ny, nx + 1))

    def field(self, comp):
        return (self.hz, self.ex, self.ey)[comp]

    def copy(self):
        c = CoarseFields(self.nx, self.ny)
        c.hz[...] = self.hz
        c.ex[...] = self.ex
        c.ey[...] = self.ey
        return c


def update_h(f: CoarseFields, chdy, chdx, cell_mask):
    """Hz^{n-1/2} -> Hz^{n+1/2} on active cells (eq. (5))."""
    curl = chdy * (f.ex[1:, :] - f.ex[:-1, :]) - chdx * (f.ey[:, 1:] - f.ey[:, :-1])
    f.hz += np.where(cell_mask, curl, 0.0)


def update_e(f: CoarseFields, ca_x, cb_x, ca_y, cb_y, ex_mask, ey_mask):
    """E^n -> E^{n+1} on active edges (eq. (3)), using Hz^{n+1/2}."""
    ny, nx = f.ny, f.nx
    new_ex = f.ex.copy()
    new_ex[1:ny, :] = ca_x[1:ny, :] * f.ex[1:ny, :] + cb_x[1:ny, :] * (f.hz[1:, :] - f.hz[:-1, :])
    f.ex[...] = np.where(ex_mask, new_ex, f.ex)
    new_ey = f.ey.copy()
    new_ey[:, 1:nx] = ca_y[:, 1:nx] * f.ey[:, 1:nx] - cb_y[:, 1:nx] * (f.hz[:, 1:] - f.hz[:, :-1])
    f.ey[...] = np.where(ey_mask, new_ey, f.ey)


def apply_sources(f: CoarseFields, sources, comp_set, n):
    for s in sources:
        if s.comp in comp_set:
            f.field(s.comp)[s.j0:s.j1, s.i0:s.i1] += s.incr[n]


def cfl_dt(dx, dy, c):
    """Right-hand side of eq. (1)."""
    return 1.0 / (c * np.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2))
