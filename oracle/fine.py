"""Fine-region FDTD model as a discrete-time descriptor system
(paper Sec. II, eqs. (2)-(8); passivity structure eqs. (24)-(25)).

A refined region of ni x nj coarse cells, refinement r, has Nx = r*ni by
Ny = r*nj fine cells of size dxh = dx/r, dyh = dy/r (eq. (2)).  State
(eq. (7)): x = [Ex (Nx x (Ny+1)); Ey ((Nx+1) x Ny); Hz (Nx x Ny)], all
boundary E included, E at step n, Hz at n-1/2.  Inputs u are the hanging
magnetic fields on the South, North, West and East boundaries, outputs y
the collocated boundary E (eq. (8)), ordered S, N, W, E with the index
increasing along each side.

Written as (R + F) x^{n+1} = (R - F) x^n + B u^{n+1/2}, y = L^T x (eq. (6))
with
  R = [[De/dt, -K/2], [-K^T/2, Dm/dt]],   F = [[Ds/2, -K/2], [K^T/2, 0]],
so that (R+F) = [[De/dt + Ds/2, -K], [0, Dm/dt]] and
(R-F) = [[De/dt - Ds/2, 0], [-K^T, Dm/dt]] reproduce eqs. (3)-(5) row by row:
  * De, Ds: diagonal, edge area (dxh*dyh, halved on boundary edges, eq. (4))
    times the edge-averaged eps, sigma (eq. (3));
  * Dm = mu0*dxh*dyh (eq. (5));
  * K (E x H): Ex(i,j) has +dxh at Hz(i,j) and -dxh at Hz(i,j-1); Ey(i,j)
    has -dyh at Hz(i,j) and +dyh at Hz(i-1,j); neighbours outside the region
    are the hanging variables and go to B;
  * B = L S with S = diag(-dxh I, +dxh I, +dyh I, -dyh I) (eq. (25)).
The paper defers these expressions to its ref. [bekmambetova2016]; they are
derived here from eqs. (3)-(5) and checked against eq. (25), eq. (24b) and
the paper's state counts 7,600 / 2,760 / 7,008.

Coarse-port restriction (reading of eqs. (15)-(16) applied before reduction):
the r fine boundary E samples lying on one coarse interface edge are equal
to that coarse E (eq. (15)); P slaves them to one coordinate.  The restricted
model R' = P^T R P, F' = P^T F P has input U = (1/r) T^T u (eq. (16)) and
B' = P^T B T = Lc Sc with Sc = diag(-dx, +dx, +dy, -dy).

PEC cells (the thin metal irises of Sec. VI-B): every edge of a PEC fine
cell carries zero tangential E and the cell's Hz stays zero, so those
samples are not unknowns.  P leaves them out (they are pinned to zero);
a coarse port whose r fine edges are all pinned has no coordinate and its
column of Lc is zero.  A port with only some of its fine edges pinned
would contradict eq. (15) and is rejected.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .constants import EPS0, MU0


class FineIndex:
    """Index bookkeeping of the full fine state."""

    def __init__(self, Nx, Ny):
        self.Nx, self.Ny = Nx, Ny
        self.n_ex = Nx * (Ny + 1)
        self.n_ey = (Nx + 1) * Ny
        self.n_e = self.n_ex + self.n_ey
        self.n_h = Nx * Ny
        self.n = self.n_e + self.n_h

    def ex(self, i, j):
        return j * self.Nx + i

    def ey(self, i, j):
        return self.n_ex + j * (self.Nx + 1) + i

    def hz(self, i, j):
        return self.n_e + j * self.Nx + i

    def ports(self):
        """Fine boundary E indices in port order S, N, W, E."""
        Nx, Ny = self.Nx, self.Ny
        s = [self.ex(i, 0) for i in range(Nx)]
        n = [self.ex(i, Ny) for i in range(Nx)]
        w = [self.ey(0, j) for j in range(Ny)]
        e = [self.ey(Nx, j) for j in range(Ny)]
        return s, n, w, e


def state_count(Nx, Ny):
    return FineIndex(Nx, Ny).n


def assemble(eps_r, sigma, dxh, dyh, dt):
    """Full fine model.  Returns dict with R, F, B, L (sparse), S (dense
    diag), the diagonal blocks De, Ds, Dm, K and the index object."""
    eps_r = np.asarray(eps_r, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    Ny, Nx = eps_r.shape
    ix = FineIndex(Nx, Ny)
    De = np.zeros(ix.n_e)
    Ds = np.zeros(ix.n_e)
    Krow, Kcol, Kval = [], [], []
    area = dxh * dyh
    # Ex(i, j): horizontal edge between Hz(i, j-1) (below) and Hz(i, j) (above)
    for j in range(Ny + 1):
        for i in range(Nx):
            e = ix.ex(i, j)
            cells = []
            if j - 1 >= 0:
                cells.append((i, j - 1))
            if j < Ny:
                cells.append((i, j))
            # boundary edge: half cell of the one adjacent fine cell (eq. (4))
            for (ci, cj) in cells:
                De[e] += 0.5 * area * EPS0 * eps_r[cj, ci]
                Ds[e] += 0.5 * area * sigma[cj, ci]
            if j < Ny:
                Krow.append(e); Kcol.append(ix.hz(i, j) - ix.n_e); Kval.append(+dxh)
            if j - 1 >= 0:
                Krow.append(e); Kcol.append(ix.hz(i, j - 1) - ix.n_e); Kval.append(-dxh)
    # Ey(i, j): vertical edge between Hz(i-1, j) (left) and Hz(i, j) (right)
    for j in range(Ny):
        for i in range(Nx + 1):
            e = ix.ey(i, j)
            cells = []
            if i - 1 >= 0:
                cells.append((i - 1, j))
            if i < Nx:
                cells.append((i, j))
            for (ci, cj) in cells:
                De[e] += 0.5 * area * EPS0 * eps_r[cj, ci]
                Ds[e] += 0.5 * area * sigma[cj, ci]
            if i < Nx:
                Krow.append(e); Kcol.append(ix.hz(i, j) - ix.n_e); Kval.append(-dyh)
            if i - 1 >= 0:
                Krow.append(e); Kcol.append(ix.hz(i - 1, j) - ix.n_e); Kval.append(+dyh)
    K = sp.csr_matrix((Kval, (Krow, Kcol)), shape=(ix.n_e, ix.n_h))
    Dm = np.full(ix.n_h, MU0 * area)
    R = sp.bmat([[sp.diags(De / dt), -0.5 * K], [-0.5 * K.T, sp.diags(Dm / dt)]], format="csr")
    F = sp.bmat([[sp.diags(Ds / 2.0), -0.5 * K], [0.5 * K.T, None]], format="csr")
    s, n, w, e = ix.ports()
    port_idx = s + n + w + e
    npf = len(port_idx)
    L = sp.csr_matrix((np.ones(npf), (port_idx, np.arange(npf))), shape=(ix.n, npf))
    S = np.concatenate([np.full(Nx, -dxh), np.full(Nx, +dxh),
                        np.full(Ny, +dyh), np.full(Ny, -dyh)])
    B = L @ sp.diags(S)
    return dict(R=R.tocsr(), F=F.tocsr(), B=B.tocsr(), L=L, S=S, De=De, Ds=Ds,
                Dm=Dm, K=K, index=ix, dxh=dxh, dyh=dyh)


def pinned_edges(pec, Nx, Ny):
    """Fine edges on a PEC cell (zero tangential E): (pin_ex [Ny+1, Nx],
    pin_ey [Ny, Nx+1]).  ``pec``: [Ny, Nx] bool or None."""
    pin_ex = np.zeros((Ny + 1, Nx), dtype=bool)
    pin_ey = np.zeros((Ny, Nx + 1), dtype=bool)
    if pec is not None:
        pec = np.asarray(pec, dtype=bool)
        pin_ex[:-1, :] |= pec      # south edge of each PEC cell
        pin_ex[1:, :] |= pec       # north edge
        pin_ey[:, :-1] |= pec      # west edge
        pin_ey[:, 1:] |= pec       # east edge
    return pin_ex, pin_ey


def restriction(ix: FineIndex, r: int, pec=None):
    """P (full -> restricted) and T (fine ports <- coarse ports).

    Restricted state: [interior Ex (j=1..Ny-1, i); interior Ey (j; i=1..Nx-1);
    coarse ports S (ni), N (ni), W (nj), E (nj); Hz (all)], leaving out the
    samples pinned by PEC cells (``pec`` [Ny, Nx] bool) and the ports whose
    fine edges are all pinned."""
    Nx, Ny = ix.Nx, ix.Ny
    ni, nj = Nx // r, Ny // r
    pin_ex, pin_ey = pinned_edges(pec, Nx, Ny)
    pec_c = np.zeros((Ny, Nx), dtype=bool) if pec is None else np.asarray(pec, dtype=bool)
    rows, cols = [], []
    col = 0
    for j in range(1, Ny):
        for i in range(Nx):
            if not pin_ex[j, i]:
                rows.append(ix.ex(i, j)); cols.append(col); col += 1
    for j in range(Ny):
        for i in range(1, Nx):
            if not pin_ey[j, i]:
                rows.append(ix.ey(i, j)); cols.append(col); col += 1
    n_int = col
    # coarse ports, S (ni), N (ni), W (nj), E (nj): the fine boundary edges
    # of each, all pinned (no coordinate) or none
    sides = ([[(pin_ex, 0, i) for i in range(c * r, (c + 1) * r)] for c in range(ni)]
             + [[(pin_ex, Ny, i) for i in range(c * r, (c + 1) * r)] for c in range(ni)]
             + [[(pin_ey, j, 0) for j in range(c * r, (c + 1) * r)] for c in range(nj)]
             + [[(pin_ey, j, Nx) for j in range(c * r, (c + 1) * r)] for c in range(nj)])
    n_pc = 2 * (ni + nj)
    port_col = []
    for k, edges in enumerate(sides):
        pins = [bool(m[a, b]) for (m, a, b) in edges]
        if any(pins) and not all(pins):
            raise ValueError(f"coarse port {k}: only some of its fine edges lie on PEC cells")
        if all(pins):
            port_col.append(-1)
        else:
            port_col.append(col)
            col += 1
    for k, edges in enumerate(sides):
        if port_col[k] < 0:
            continue
        for (m, a, b) in edges:
            rows.append(ix.ex(b, a) if m is pin_ex else ix.ey(b, a))
            cols.append(port_col[k])
    n_e_r = col
    for j in range(Ny):
        for i in range(Nx):
            if not pec_c[j, i]:
                rows.append(ix.hz(i, j)); cols.append(col); col += 1
    n_h_r = col - n_e_r
    n_r = col
    P = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(ix.n, n_r))
    # T: fine port p (S,N,W,E order) -> coarse port
    trow, tcol = [], []
    for i in range(Nx):
        trow.append(i); tcol.append(i // r)
    for i in range(Nx):
        trow.append(Nx + i); tcol.append(ni + i // r)
    for j in range(Ny):
        trow.append(2 * Nx + j); tcol.append(2 * ni + j // r)
    for j in range(Ny):
        trow.append(2 * Nx + Ny + j); tcol.append(2 * ni + nj + j // r)
    T = sp.csr_matrix((np.ones(len(trow)), (trow, tcol)), shape=(2 * (Nx + Ny), n_pc))
    live = [k for k in range(n_pc) if port_col[k] >= 0]
    Lc = sp.csr_matrix((np.ones(len(live)), ([port_col[k] for k in live], live)),
                       shape=(n_r, n_pc))
    return dict(P=P, T=T, Lc=Lc, n_e=n_e_r, n_h=n_h_r, n=n_r, n_ports=n_pc,
                dead_ports=[k for k in range(n_pc) if port_col[k] < 0])


def coarse_port_scale(ni, nj, dx, dy):
    """Sc = diag(-dx I_ni, +dx I_ni, +dy I_nj, -dy I_nj): the coarse analog of eq. (25)."""
    return np.concatenate([np.full(ni, -dx), np.full(ni, +dx),
                           np.full(nj, +dy), np.full(nj, -dy)])


def restricted_model(eps_r, sigma, r, dx, dy, dt, pec=None):
    """Fine model restricted to coarse ports (and without the samples PEC
    cells pin): R', F', Lc, B' = Lc Sc."""
    Ny, Nx = np.asarray(eps_r).shape
    full = assemble(eps_r, sigma, dx / r, dy / r, dt)
    rs = restriction(full["index"], r, pec)
    P = rs["P"]
    Rr = (P.T @ full["R"] @ P).tocsr()
    Fr = (P.T @ full["F"] @ P).tocsr()
    Sc = coarse_port_scale(Nx // r, Ny // r, dx, dy)
    Br = (rs["Lc"] @ sp.diags(Sc)).tocsr()
    return dict(R=Rr, F=Fr, L=rs["Lc"], B=Br, S=Sc, n_e=rs["n_e"], n_h=rs["n_h"],
                n=rs["n"], n_ports=rs["n_ports"], full=full, restriction=rs)
