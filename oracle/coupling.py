"""Coupling of a reduced model to the coarse grid (paper Sec. IV, eqs. (13)-(23)).

Coarse interface E with a hanging variable (eq. (13), matrix form eq. (14)):
  Dl Dl' (De/dt + Ds/2) y^{n+1} = Dl Dl' (De/dt - Ds/2) y^n + Dl G^T H^{n+1/2} - Dl G^T U^{n+1/2}
where, per interface edge, Dl is the coarse edge length, Dl' the half-edge
crossing the interface, De, Ds the material of the coarse half cell outside
the region, H the coarse Hz just outside and U the hanging variable.  From
eq. (13) and its N/W/E analogues, Dl G^T = Sc = diag(-dx, +dx, +dy, -dy) for
ports ordered S, N, W, E.

With the reduced model built on coarse ports (interpolation rule (15)-(16)
applied before reduction, so T = I and r -> 1 in eqs. (17)-(22)), the
literal system of eq. (19) in z = [y; U; x~] reads
  A1 = [[C+, Sc, 0], [I, 0, -L~^T], [0, -L~ Sc, R~ + F~]]
  A2 = [[C-, 0, 0], [0, 0, 0], [0, 0, R~ - F~]]
  A1 z^{n+1} = A2 z^n + [Sc H^{n+1/2}; 0; 0]                   (eq. (19))
with C+- = Dl Dl' (De/dt +- Ds/2).  Eliminating y and U (y = L~^T x~ at
every step) gives the closed form of eq. (23):
  x~^{n+1} = A~ x~^n + B~' H^{n+1/2},  y^{n+1} = C~ x~^{n+1}
           = C~ A~ x~^n + C~ B~' H^{n+1/2},
  A~ = (R~+F~+L~ C+ L~^T)^{-1} (R~-F~+L~ C- L~^T),
  B~' = (R~+F~+L~ C+ L~^T)^{-1} L~ Sc,  C~ = L~^T.

Parity: the literal and closed forms are checked against each other, and
with an identity basis against plain Yee (r = 1) and direct merged-edge
subgridding (r > 1), which are coded independently of this module.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .constants import EPS0
from .yee import EX, EY


def coarse_ports(i0, j0, ni, nj, dx, dy):
    """Per port (order S, N, W, E; index increasing along each side):
    (comp, edge_i, edge_j, out_i, out_j, Dl, Dl_half)."""
    ports = []
    for c in range(ni):
        ports.append((EX, i0 + c, j0, i0 + c, j0 - 1, dx, dy / 2))
    for c in range(ni):
        ports.append((EX, i0 + c, j0 + nj, i0 + c, j0 + nj, dx, dy / 2))
    for c in range(nj):
        ports.append((EY, i0, j0 + c, i0 - 1, j0 + c, dy, dx / 2))
    for c in range(nj):
        ports.append((EY, i0 + ni, j0 + c, i0 + ni, j0 + c, dy, dx / 2))
    return ports


def port_scale(ni, nj, dx, dy):
    return np.concatenate([np.full(ni, -dx), np.full(ni, +dx),
                           np.full(nj, +dy), np.full(nj, -dy)])


class RomCoupling:
    """One embedded reduced model: literal eq. (19) solve and the closed form."""

    def __init__(self, Rt, Ft, Lt, i0, j0, ni, nj, eps_r, sigma, dx, dy, dt):
        self.Rt, self.Ft, self.Lt = Rt, Ft, Lt
        self.i0, self.j0, self.ni, self.nj = i0, j0, ni, nj
        self.ports = coarse_ports(i0, j0, ni, nj, dx, dy)
        self.np_ = len(self.ports)
        self.q = Rt.shape[0]
        self.Sc = port_scale(ni, nj, dx, dy)
        cp = np.zeros(self.np_)
        cm = np.zeros(self.np_)
        for k, (_, _, _, oi, oj, dl, dlh) in enumerate(self.ports):
            e = EPS0 * eps_r[oj, oi]
            s = sigma[oj, oi]
            cp[k] = dl * dlh * (e / dt + s / 2.0)
            cm[k] = dl * dlh * (e / dt - s / 2.0)
        self.Cp, self.Cm = cp, cm
        npp, q = self.np_, self.q
        n = 2 * npp + q
        A1 = np.zeros((n, n))
        A2 = np.zeros((n, n))
        iy = slice(0, npp)
        iu = slice(npp, 2 * npp)
        ix = slice(2 * npp, n)
        A1[iy, iy] = np.diag(cp)
        A1[iy, iu] = np.diag(self.Sc)
        A1[iu, iy] = np.eye(npp)
        A1[iu, ix] = -Lt.T
        A1[ix, iu] = -Lt * self.Sc[None, :]
        A1[ix, ix] = Rt + Ft
        A2[iy, iy] = np.diag(cm)
        A2[ix, ix] = Rt - Ft
        self.A1, self.A2 = A1, A2
        self.lu = sla.lu_factor(A1)
        self.sl = (iy, iu, ix)

    # literal form ---------------------------------------------------------
    def step_literal(self, z, hnear):
        iy, iu, ix = self.sl
        rhs = self.A2 @ z
        rhs[iy] += self.Sc * hnear
        return sla.lu_solve(self.lu, rhs)

    def z_from(self, y, x):
        z = np.zeros(2 * self.np_ + self.q)
        iy, iu, ix = self.sl
        z[iy] = y
        z[ix] = x
        return z

    # closed form ----------------------------------------------------------
    def closed_form(self, solver="lu"):
        """Eq. (23) eliminated: A~ = M^{-1} N, B~' = M^{-1} L~ Sc, C~ = L~^T
        with M = R~ + F~ + L~ C+ L~^T, N = R~ - F~ + L~ C- L~^T.  ``solver``
        'lu' (partial pivoting) or 'qr' (Householder): two backward-stable
        routes to the same matrices, whose difference measures how well
        FP64 determines them for an ill-conditioned M."""
        Lt = self.Lt
        M = self.Rt + self.Ft + (Lt * self.Cp[None, :]) @ Lt.T
        N = self.Rt - self.Ft + (Lt * self.Cm[None, :]) @ Lt.T
        LS = Lt * self.Sc[None, :]
        if solver == "lu":
            A = np.linalg.solve(M, N)
            B = np.linalg.solve(M, LS)
        elif solver == "qr":
            Qm, Rm = np.linalg.qr(M)
            A = sla.solve_triangular(Rm, Qm.T @ N)
            B = sla.solve_triangular(Rm, Qm.T @ LS)
        else:
            raise ValueError(solver)
        C = Lt.T.copy()
        return A, B, C

    def update_matrix(self, solver="lu"):
        """Eq. (23) as one map on [x~^n; h^{n+1/2}] -> [x~^{n+1}; y^{n+1}]:
        G = [[A~, B~'], [C~ A~, C~ B~']] (y^{n+1} taken directly from the
        step-n quantities, as eq. (23) gives it)."""
        A, B, C = self.closed_form(solver)
        return np.block([[A, B], [C @ A, C @ B]])

    def gather(self, hz):
        return np.array([hz[oj, oi] for (_, _, _, oi, oj, _, _) in self.ports])

    def scatter(self, ex, ey, y):
        for k, (comp, ei, ej, _, _, _, _) in enumerate(self.ports):
            (ex if comp == EX else ey)[ej, ei] = y[k]

    def read_y(self, ex, ey):
        return np.array([(ex if comp == EX else ey)[ej, ei]
                         for (comp, ei, ej, _, _, _, _) in self.ports])
