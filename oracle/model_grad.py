"""Gradients through the reduced models (test infrastructure only).

The objective is the adjoint's J = dt * sum_n (Hz_p^{n+1/2})^2.  Besides the
coarse material outside the regions (``adjoint``), J depends on

  * each region's eq. (23) update matrix G = [[A~, B~'], [C~A~, C~B~']]:
      dJ/dG = sum_n lam_out^{n+1} [x~^n; h^{n+1/2}]^T,
    lam_out the adjoint of the step's eq. (23) outputs [x~^{n+1}; y^{n+1}];
  * through the closed form of eq. (23) (Sec. IV-C), with
      M = R~ + F~ + L~ C+ L~^T,  N = R~ - F~ + L~ C- L~^T,
      A~ = M^{-1} N,  B~' = M^{-1} L~ Sc,  C~ = L~^T,
    on the reduced matrices R~, F~, L~ of eqs. (11)-(12) and on C+- of
    eq. (13), whose half cells are the coarse cells just outside each port
    (the region's one-cell ring): C+- = Dl Dl' (eps0 eps_r/dt +- sigma/2);
  * through the congruence of eqs. (11)-(12) on the fine model's edge
    permittivities and conductivities (eqs. (3)-(4): each fine edge takes
    half the cell area of each adjacent fine cell), and through the eq. (27)
    clip when it is active.

The projection basis V = blkdiag(V1, V2) is held at its built value: the
gradient is that of the parametric reduced model R~(p) = V^T R(p) V with a
fixed V, the usual reading when one basis serves nearby designs.  The
result depends on V only through its column spaces: replacing V1, V2 by
V1 Q1, V2 Q2 (Q orthogonal) turns R~, F~, L~ and the clipped K~ into
congruent copies and leaves every input-output quantity, J included,
unchanged.  With the identity basis (no reduction) there is no basis to
hold and this is the gradient of the whole pipeline.

Reverse-mode rules used (all plain matrix calculus):
  * X = M^{-1} Y:  Y_bar = M^{-T} X_bar,  M_bar = -M^{-T} X_bar X^T;
  * a symmetric matrix function F = Z f(diag mu) Z^T of S = Z diag(mu) Z^T
    (Daleckii-Krein): S_bar = Z (D o (Z^T sym(F_bar) Z)) Z^T with
    D_ij = (f(mu_i) - f(mu_j)) / (mu_i - mu_j), D_ii = f'(mu_i);
  * eq. (27)'s clip lowers the singular values of
    M = R11^{-1/2} K~ R22^{-1/2} (R11 = dt R~11, R22 = dt R~22, K~ = -2 R~12)
    to lim = theta 2/dt, i.e. M_c = M g(M^T M) with g(mu) = min(1, lim/sqrt(mu)),
    and K~_c = R11^{1/2} M_c R22^{1/2}; R~22 and K~ do not depend on the
    material when V is held, so only R11's path is differentiated.

Parity: pinned by central finite differences of the oracle's forward run
(with respect to R~, F~, L~, to ring cells, and to fine cells through
``rom.build_rom`` with the basis held), by the identity basis (the whole
pipeline differentiated), and by the basis invariance above.
"""
from __future__ import annotations

import numpy as np

from .constants import EPS0
from . import adjoint as oadj


def update_matrix_vjp(c, gG):
    """Gradients of J with respect to R~, F~, L~ and C+-, C- per port of one
    coupled model ``c`` (oracle.coupling.RomCoupling), given dJ/dG."""
    q = c.q
    A, B, C = c.closed_form()
    Lt = c.Lt
    M = c.Rt + c.Ft + (Lt * c.Cp[None, :]) @ Lt.T
    gA = gG[:q, :q] + C.T @ gG[q:, :q]
    gB = gG[:q, q:] + C.T @ gG[q:, q:]
    gC = gG[q:, :q] @ A.T + gG[q:, q:] @ B.T
    WA = np.linalg.solve(M.T, gA)       # N_bar
    WB = np.linalg.solve(M.T, gB)       # (L~ Sc)_bar
    gM = -(WA @ A.T + WB @ B.T)
    gN = WA
    gRt = gM + gN
    gFt = gM - gN
    gLt = ((gM + gM.T) @ Lt) * c.Cp[None, :] + ((gN + gN.T) @ Lt) * c.Cm[None, :] \
        + WB * c.Sc[None, :] + gC.T
    gCp = np.einsum("ak,ab,bk->k", Lt, gM, Lt)
    gCm = np.einsum("ak,ab,bk->k", Lt, gN, Lt)
    return gRt, gFt, gLt, gCp, gCm


def interior_mask(prob):
    """True for cells whose material J can depend on: outside every region
    (rings included) and not PEC."""
    m = np.ones((prob.ny, prob.nx), dtype=bool)
    for s in prob.roms:
        m[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = False
    pec = getattr(prob, "pec", None)
    if pec is not None:
        m &= ~np.asarray(pec, dtype=bool)
    return m


def model_gradient(prob, roms, nsteps=None, probe=0, fp32=False):
    """J and its gradients: the coarse maps dJ/deps_r, dJ/dsigma (ring cells
    included, through C+-; zero inside regions and on PEC cells) and per
    region dict(G, Rt, Ft, Lt) of dJ/d(matrix).  fp32: the run with FP32
    coefficients and update matrices (the matrix gradients are then taken
    through the FP64 closed form at the same models)."""
    nsteps = prob.nsteps if nsteps is None else nsteps
    run, J, g_edges, dG = oadj._sweep(prob, roms, nsteps, probe, fp32, models=True)
    geps, gsig = oadj._cell_gradient(prob, g_edges)
    out = []
    for c, gG in zip(run.cpl, dG):
        gRt, gFt, gLt, gCp, gCm = update_matrix_vjp(c, gG)
        for k, (_, _, _, oi, oj, dl, dlh) in enumerate(c.ports):
            geps[oj, oi] += dl * dlh * EPS0 / prob.dt * (gCp[k] + gCm[k])
            gsig[oj, oi] += dl * dlh * 0.5 * (gCp[k] - gCm[k])
        out.append(dict(G=gG, Rt=gRt, Ft=gFt, Lt=gLt))
    m = interior_mask(prob)
    return dict(J=J, eps_r=np.where(m, geps, 0.0), sigma=np.where(m, gsig, 0.0), models=out)


def _sym(X):
    return 0.5 * (X + X.T)


def _dk_vjp(Z, D, Fbar):
    """Daleckii-Krein pull-back: S_bar = Z (D o (Z^T sym(F_bar) Z)) Z^T."""
    return Z @ (D * (Z.T @ _sym(Fbar) @ Z)) @ Z.T


def clip_vjp(R11, R22, K, lim, gKc):
    """dJ/dR11 of K~_c = R11^{1/2} M g(M^T M) R22^{1/2},
    M = R11^{-1/2} K R22^{-1/2}, given dJ/dK~_c (R22, K held)."""
    nu, Y = np.linalg.eigh(R11)
    w, Zr = np.linalg.eigh(R22)
    rn = np.sqrt(nu)
    P = (Y * rn) @ Y.T
    Q = (Y / rn) @ Y.T
    R22h = (Zr * np.sqrt(w)) @ Zr.T
    R22ih = (Zr / np.sqrt(w)) @ Zr.T
    M = Q @ K @ R22ih
    mu, U = np.linalg.eigh(M.T @ M)
    mu = np.maximum(mu, 0.0)
    sq = np.sqrt(mu)
    big = sq > lim
    g = np.where(big, lim / np.where(big, sq, 1.0), 1.0)
    Gm = (U * g) @ U.T
    Phi = M @ Gm
    # difference quotients of g on the spectrum of M^T M
    n = mu.size
    Dg = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if big[i] and big[j]:
                Dg[i, j] = -lim / (sq[i] * sq[j] * (sq[i] + sq[j]))
            elif big[i] != big[j] and mu[i] != mu[j]:
                Dg[i, j] = (g[i] - g[j]) / (mu[i] - mu[j])
    # d sqrt and d 1/sqrt on the spectrum of R11
    Dp = 1.0 / (rn[:, None] + rn[None, :])
    Dq = -1.0 / (rn[:, None] * rn[None, :] * (rn[:, None] + rn[None, :]))
    gP = gKc @ R22h @ Phi.T
    gPhi = P @ gKc @ R22h
    gM = gPhi @ Gm
    gS = _dk_vjp(U, Dg, M.T @ gPhi)
    gM = gM + M @ (gS + gS.T)
    gQ = gM @ R22ih @ K.T
    return _dk_vjp(Y, Dp, gP) + _dk_vjp(Y, Dq, gQ)


def build_vjp(rom, gRt, gFt):
    """dJ/deps_r and dJ/dsigma of the region's fine cells [r*nj, r*ni] from
    dJ/dR~ and dJ/dF~ of a model made by ``rom.build_rom`` (its basis held;
    L~ = V^T Lc does not depend on the material)."""
    q1 = rom["q1"]
    dt = rom["dt"]
    Rt = rom["Rt"]
    gRt = np.asarray(gRt, np.float64)
    gFt = np.asarray(gFt, np.float64)
    gR11 = gRt[:q1, :q1].copy()
    if rom["clipped"]:
        gK = -0.5 * gRt[:q1, q1:] - 0.5 * gRt[q1:, :q1].T - 0.5 * gFt[:q1, q1:] + 0.5 * gFt[q1:, :q1].T
        lim = rom["theta"] * 2.0 / dt
        gR11 += dt * clip_vjp(dt * Rt[:q1, :q1], dt * Rt[q1:, q1:], rom["K0"], lim, gK)
    gF11 = gFt[:q1, :q1]
    model = rom["model"]
    full = model["full"]
    ix = full["index"]
    P = model["restriction"]["P"]
    W1 = P[:ix.n_e, :model["n_e"]] @ rom["V1"]      # full fine E edges x q1
    dDe = np.sum((W1 @ gR11) * W1, axis=1) / dt      # dJ/d(De) per fine edge
    dDs = np.sum((W1 @ gF11) * W1, axis=1) * 0.5     # dJ/d(Ds)
    Nx, Ny = ix.Nx, ix.Ny
    area = full["dxh"] * full["dyh"]
    ge = np.zeros((Ny, Nx))
    gs = np.zeros((Ny, Nx))
    w = 0.5 * area
    for j in range(Ny + 1):
        for i in range(Nx):
            e = ix.ex(i, j)
            for cj in (j - 1, j):
                if 0 <= cj < Ny:
                    ge[cj, i] += w * EPS0 * dDe[e]
                    gs[cj, i] += w * dDs[e]
    for j in range(Ny):
        for i in range(Nx + 1):
            e = ix.ey(i, j)
            for ci in (i - 1, i):
                if 0 <= ci < Nx:
                    ge[j, ci] += w * EPS0 * dDe[e]
                    gs[j, ci] += w * dDs[e]
    return ge, gs
