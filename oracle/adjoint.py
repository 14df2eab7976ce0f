"""Discrete adjoint of the coupled run: gradient of
    J = dt * sum_{n=0}^{N-1} (Hz_p^{n+1/2})^2
with respect to the per-cell relative permittivity and conductivity of the
coarse grid (paper Sec. II-A eq. (3) coefficients; eq. (23) coupling held
fixed: the reduced models are inputs).

The forward step (oracle.sim) is linear in the state s^n = (E^n, Hz^{n-1/2},
x~^n) for fixed coefficients:
  1. Hz' = M (Hz + curlE(E)) + src            (eq. (5), M = active-cell mask)
  2. E'  = Ca E + Cb curlH(Hz') + src          on active edges (eq. (3))
  3. [x~'; y'] = G [x~; gather(Hz')],  E'[interface] = y'   (eq. (23))
  4. J += dt (Hz'_p)^2
The reverse sweep applies the transpose of 3, 2, 1 in that order with
lambda^N = 0, and accumulates dJ/dCa_e = sum lambda_E'_e E_e and
dJ/dCb_e = sum lambda_E'_e dH_e over active edges.  With a = eps/dt,
b = sigma/2 on an edge (eps, sigma the mean of its two cells),
Ca = (a-b)/(a+b) and Cb/d = 1/((a+b) d):
  dCa/da = 2b/(a+b)^2, dCa/db = -2a/(a+b)^2, d(Cb/d)/da = d(Cb/d)/db = -1/((a+b)^2 d),
  da/deps_r(cell) = eps0/(2 dt), db/dsigma(cell) = 1/4 for each of the edge's cells.
Cells inside reduced regions and their one-cell rings (whose half cells
enter C+- of eq. (13)) get zero gradient: the models are held fixed.

With absorbing layers (oracle.cpml) the state also holds the auxiliary
fields psi, and steps 1-2 become (per cell / active edge, b, a, 1/kappa the
layer profiles):
  psi_hy' = b psi_hy + a dEx,  psi_hx' = b psi_hx + a dEy,
  Hz' = Hz + M (chdy (dEx/kappa + psi_hy') - chdx (dEy/kappa + psi_hx')),
  psi_ex' = b psi_ex + a dHz,  Ex' = Ca Ex + Cb (dHz/kappa + psi_ex')  (Ey: - Cb),
so in reverse each psi' collects its own adjoint plus the +-chdy mu /
+-Cb lambda_E term, hands b times that to the old psi and a times it to the
difference it filters; dJ/dCb then weighs the stretched difference
dHz/kappa + psi'.  Outside the layers (a = 0, b = 1/kappa = 1) this is the
plain transpose above.

Parity: pinned by central finite differences of the oracle's own forward
run and by the transpose identity <lambda, delta s> of one step (with and
without layers).
"""
from __future__ import annotations

import numpy as np

from .constants import EPS0
from . import sim as osim
from . import yee


def _edge_ab(prob):
    """a = eps/dt, b = sigma/2 on interior edges (FP64)."""
    er, sg, dt = prob.eps_r, prob.sigma, prob.dt
    ax = EPS0 * 0.5 * (er[1:, :] + er[:-1, :]) / dt
    bx = 0.25 * (sg[1:, :] + sg[:-1, :])
    ay = EPS0 * 0.5 * (er[:, 1:] + er[:, :-1]) / dt
    by = 0.25 * (sg[:, 1:] + sg[:, :-1])
    return ax, bx, ay, by


def gradient_mask(prob):
    """True for cells whose gradient is reported (outside every region and
    its one-cell ring, and not a PEC cell, whose material takes no part)."""
    m = np.ones((prob.ny, prob.nx), dtype=bool)
    for s in prob.roms:
        m[max(s.j0 - 1, 0):s.j0 + s.nj + 1, max(s.i0 - 1, 0):s.i0 + s.ni + 1] = False
    pec = getattr(prob, "pec", None)
    if pec is not None:
        m &= ~np.asarray(pec, dtype=bool)
    return m


def forward_states(prob, roms, nsteps=None, probe=0, fp32=False):
    """Forward run keeping (E^n, Hz^{n-1/2}) for n = 0..N and the objective.
    fp32: the eq. (3) coefficients and eq. (23) update matrix rounded to FP32
    as an FP32 run holds them (arithmetic stays FP64)."""
    run = osim.CoupledRun(prob, roms, mode="closed", fp32=fp32)
    nsteps = prob.nsteps if nsteps is None else nsteps

    def snap():
        s = (run.f.ex.copy(), run.f.ey.copy(), run.f.hz.copy())
        if run.pml is not None:
            s += (run.pml.psi_ex.copy(), run.pml.psi_ey.copy())
        return s
    states = [snap()]
    run.x_hist = [[x.copy() for x in run.x]]   # reduced states x~^n, n = 0..N
    J = 0.0
    pr = prob.probes[probe]
    for n in range(nsteps):
        run.step()
        states.append(snap())
        run.x_hist.append([x.copy() for x in run.x])
        J += prob.dt * run.f.hz[pr.j, pr.i] ** 2
    return run, states, J


def transpose_step(run, Gs, lam, lam_out=None):
    """lambda^n = M^T lambda^{n+1} for one forward step M of ``run``
    (steps 3, 2, 1 of the module docstring transposed, in that order).
    lam = (lam_ex, lam_ey, lam_hz, lam_x) is the adjoint of the state after
    the step (any objective term already added to lam_hz), followed with
    absorbing layers by (lam_psi_hx, lam_psi_hy, lam_psi_ex, lam_psi_ey).
    Returns the adjoint of the state before the step (same layout) and
    (lex, ley), the adjoint of the new E on the edges eq. (3) updates (the
    coefficient gradients' weights).  ``lam_out`` (a list, optional)
    receives per model the adjoint of the step's eq. (23) outputs
    [x~^{n+1}; y^{n+1}]."""
    pml = run.pml
    lam_ex, lam_ey, lam_hz, lam_x = lam[:4]
    cell, exm, eym = run.cell, run.exm, run.eym
    ca_x, cb_x, ca_y, cb_y, chdy, chdx = run.ca_x, run.cb_x, run.ca_y, run.cb_y, run.chdy, run.chdx
    ny, nx = cell.shape
    lam_h = lam_hz.copy()
    lam_ex_in = lam_ex.copy()
    lam_ey_in = lam_ey.copy()
    # 3. coupling: [x'; y'] = G [x; gather(Hz')], y' into interface edges
    new_lam_x = []
    for c, G, lx in zip(run.cpl, Gs, lam_x):
        ly = c.read_y(lam_ex_in, lam_ey_in)
        if lam_out is not None:
            lam_out.append(np.concatenate([lx, ly]))
        back = G.T @ np.concatenate([lx, ly])
        new_lam_x.append(back[:c.q].copy())
        for k, (_, _, _, oi, oj, _, _) in enumerate(c.ports):
            lam_h[oj, oi] += back[c.q + k]
        c.scatter(lam_ex_in, lam_ey_in, np.zeros(c.np_))   # consumed
    # 2. E' = Ca E + Cb curlH(Hz') on active edges; vx, vy: the adjoints of
    # the Hz differences dHz = Hz(j)-Hz(j-1) (Ex), Hz(i)-Hz(i-1) (Ey)
    lex = np.where(exm, lam_ex_in, 0.0)
    ley = np.where(eym, lam_ey_in, 0.0)
    if pml is None:
        vx = lex * cb_x
        vy = -ley * cb_y
    else:
        l_phx, l_phy, l_pex, l_pey = lam[4:]
        tx = l_pex + cb_x * lex            # adjoint of psi_ex' (its own + through Ex')
        ty = l_pey - cb_y * ley
        vx = np.where(exm, cb_x * pml.iky_e[:, None] * lex + pml.ay_e[:, None] * tx, 0.0)
        vy = np.where(eym, -cb_y * pml.ikx_e[None, :] * ley + pml.ax_e[None, :] * ty, 0.0)
        new_pex = np.where(exm, pml.by_e[:, None] * tx, l_pex)
        new_pey = np.where(eym, pml.bx_e[None, :] * ty, l_pey)
    lam_h += vx[:-1, :] - vx[1:, :]       # edge (i,j) above cell (i,j-1): +, edge (i,j+1): -
    lam_h += vy[:, :-1] - vy[:, 1:]
    # 1. Hz' = M (Hz + chdy dEx - chdx dEy), dEx = Ex(j+1)-Ex(j), dEy = Ey(i+1)-Ey(i)
    mu = lam_h * cell
    if pml is None:
        ldex = chdy * mu
        ldey = -chdx * mu
    else:
        thy = l_phy + chdy * mu            # adjoint of psi_hy' (its own + through Hz')
        thx = l_phx - chdx * mu
        ldex = chdy * pml.iky_h[:, None] * mu + pml.ay_h[:, None] * thy
        ldey = -chdx * pml.ikx_h[None, :] * mu + pml.ax_h[None, :] * thx
        new_phy = pml.by_h[:, None] * thy
        new_phx = pml.bx_h[None, :] * thx
    new_ex = lex * ca_x
    new_ey = ley * ca_y
    new_ex[1:, :] += ldex
    new_ex[:-1, :] -= ldex
    new_ey[:, 1:] += ldey
    new_ey[:, :-1] -= ldey
    # walls carry no adjoint (E fixed at zero there)
    new_ex[0, :] = 0.0
    new_ex[ny, :] = 0.0
    new_ey[:, 0] = 0.0
    new_ey[:, nx] = 0.0
    out = (new_ex, new_ey, mu, new_lam_x)
    if pml is not None:
        out += (new_phx, new_phy, new_pex, new_pey)
    return out, (lex, ley)


def _sweep(prob, roms, nsteps, probe, fp32, models):
    """Forward run and reverse sweep.  Returns (run, J, [g_ca_x, g_cb_x,
    g_ca_y, g_cb_y], dG): the gradients of J with respect to the eq. (3)
    coefficients of every E edge, and with ``models`` per model the
    gradient with respect to its eq. (23) update matrix G,
    dJ/dG = sum_n lam_out^{n+1} [x~^n; h^{n+1/2}]^T (else None)."""
    run, states, J = forward_states(prob, roms, nsteps, probe, fp32)
    pml = run.pml
    nx, ny = prob.nx, prob.ny
    cell = run.cell
    pr = prob.probes[probe]
    if pr.comp != yee.HZ:
        raise ValueError("objective probe must be an Hz probe")
    Gs = [c.G32 if fp32 else c.update_matrix() for c in run.cpl]
    dG = [np.zeros_like(G) for G in Gs] if models else None
    lam = (np.zeros((ny + 1, nx)), np.zeros((ny, nx + 1)), np.zeros((ny, nx)),
           [np.zeros(c.q) for c in run.cpl])
    if pml is not None:
        lam += (np.zeros((ny, nx)), np.zeros((ny, nx)), np.zeros((ny + 1, nx)), np.zeros((ny, nx + 1)))
    g_cax = np.zeros((ny + 1, nx))
    g_cbx = np.zeros((ny + 1, nx))
    g_cay = np.zeros((ny, nx + 1))
    g_cby = np.zeros((ny, nx + 1))
    for n in range(nsteps - 1, -1, -1):
        ex0, ey0 = states[n][:2]         # E^n
        hz1 = states[n + 1][2]           # Hz^{n+1/2}
        hz1 = hz1 * cell
        # objective: J += dt (Hz'_p)^2
        lam_hz = lam[2].copy()
        lam_hz[pr.j, pr.i] += 2.0 * prob.dt * hz1[pr.j, pr.i]
        lam_out = [] if models else None
        lam, (lex, ley) = transpose_step(run, Gs, (lam[0], lam[1], lam_hz) + tuple(lam[3:]), lam_out)
        if models:
            for k, c in enumerate(run.cpl):
                z = np.concatenate([run.x_hist[n][k], c.gather(hz1)])
                dG[k] += np.outer(lam_out[k], z)
        dhx = np.zeros((ny + 1, nx))
        dhx[1:ny, :] = hz1[1:, :] - hz1[:-1, :]
        dhy = np.zeros((ny, nx + 1))
        dhy[:, 1:nx] = hz1[:, 1:] - hz1[:, :-1]
        if pml is not None:              # the stretched differences dHz/kappa + psi'
            dhx = pml.iky_e[:, None] * dhx + states[n + 1][3]
            dhy = pml.ikx_e[None, :] * dhy + states[n + 1][4]
        g_cax += lex * ex0
        g_cbx += lex * dhx
        g_cay += ley * ey0
        g_cby -= ley * dhy
    return run, J, (g_cax, g_cbx, g_cay, g_cby), dG


def _cell_gradient(prob, g_edges):
    """Chain rule from the eq. (3) coefficients of the updated edges to the
    per-cell eps_r and sigma (unmasked)."""
    g_cax, g_cbx, g_cay, g_cby = g_edges
    nx, ny = prob.nx, prob.ny
    ax, bx, ay, by = _edge_ab(prob)
    d = {}
    for (gca, gcb, a, b, dd, sl) in ((g_cax, g_cbx, ax, bx, prob.dy, (slice(1, ny), slice(None))),
                                     (g_cay, g_cby, ay, by, prob.dx, (slice(None), slice(1, nx)))):
        s2 = (a + b) ** 2
        dca_da = 2 * b / s2
        dca_db = -2 * a / s2
        dcb_dab = -1.0 / (s2 * dd)
        ga = gca[sl] * dca_da + gcb[sl] * dcb_dab     # dJ/da on each edge
        gb = gca[sl] * dca_db + gcb[sl] * dcb_dab     # dJ/db
        d[id(gca)] = (ga, gb)
    gex_a, gex_b = d[id(g_cax)]   # [ny-1, nx], edge between cells (i,j-1),(i,j)
    gey_a, gey_b = d[id(g_cay)]   # [ny, nx-1], edge between cells (i-1,j),(i,j)
    geps = np.zeros((ny, nx))
    gsig = np.zeros((ny, nx))
    fa = EPS0 / (2.0 * prob.dt)
    fb = 0.25
    geps[:-1, :] += fa * gex_a
    geps[1:, :] += fa * gex_a
    geps[:, :-1] += fa * gey_a
    geps[:, 1:] += fa * gey_a
    gsig[:-1, :] += fb * gex_b
    gsig[1:, :] += fb * gex_b
    gsig[:, :-1] += fb * gey_b
    gsig[:, 1:] += fb * gey_b
    return geps, gsig


def adjoint_gradient(prob, roms, nsteps=None, probe=0, fp32=False):
    """Return (J, dJ/deps_r [ny,nx], dJ/dsigma [ny,nx]).  fp32: transpose of
    the forward with FP32-rounded coefficients (see forward_states)."""
    nsteps = prob.nsteps if nsteps is None else nsteps
    _, J, g_edges, _ = _sweep(prob, roms, nsteps, probe, fp32, models=False)
    geps, gsig = _cell_gradient(prob, g_edges)
    m = gradient_mask(prob)
    return J, np.where(m, geps, 0.0), np.where(m, gsig, 0.0)


def objective(prob, roms, nsteps=None, probe=0):
    return forward_states(prob, roms, nsteps, probe)[2]
