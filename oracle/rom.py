"""Model order reduction of a fine region (paper Sec. III, eqs. (9)-(12)),
passivity conditions (Sec. V, eqs. (24)-(26), Theorem 1) and the
CFL-extending perturbation (Sec. V-E, eq. (27)).

Steps, in the paper's order:
  1. fine descriptor system, restricted to coarse ports (``fine``);
  2. SPRIM-style projection V = blkdiag(V1, V2) (eq. (9)): block Arnoldi on
     (p0 R + F)^{-1} R started from (p0 R + F)^{-1} B, with the real
     expansion point p0 = pi * f_max * dt (the bilinear variable
     p = (z-1)/(z+1) reaches about pi*f*dt at the band edge); the Arnoldi
     vectors are split into their E rows and H rows, each orthonormalised
     separately (SPRIM keeps the E/H block structure).  The E basis takes
     q1 = ceil(q/2) columns and the H basis q2 = floor(q/2); whole blocks are
     taken in Krylov order and a partial block contributes its leading left
     singular vectors;
  3. congruence R~ = V^T R V, F~ = V^T F V, L~ = V^T L, B~ = L~ Sc (eqs. (11)-(12));
  4. if max singular value of R11^{-1/2} K~ R22^{-1/2} exceeds theta*2/dt,
     clip it to theta*2/dt and rebuild K~ (eq. (27)); K~ is replaced wherever
     it appears (in R~ and in F~), which leaves F~ + F~^T and B~ unchanged.
     theta = 0.99 (strict inequality keeps R~ > 0).

Parity: the content of a reduced model depends on SPRIM details the paper
does not give (expansion point, block handling); runs are therefore
compared on identical reduced-model inputs.  The builder itself is pinned
by Theorem 1's invariants (R~ = R~^T > 0, F~ + F~^T >= 0, B~ = L~ Sc), by
moment matching at p0 when the whole first block is kept, by the identity
basis reproducing the unreduced region, and by the clip's effect on the
spectral radius of the coupled scheme.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fine


def _gs_in_order(vectors, q, tol=1e-10):
    """Euclidean Gram-Schmidt (two passes) over columns in the given order,
    skipping columns whose residual falls below tol times their norm; stops
    at q columns."""
    out = []
    for k in range(vectors.shape[1]):
        if len(out) >= q:
            break
        v = vectors[:, k].copy()
        nv = np.linalg.norm(v)
        if nv == 0.0:
            continue
        for _ in range(2):
            for u in out:
                v -= (u @ v) * u
        nr = np.linalg.norm(v)
        if nr <= tol * nv:
            continue
        out.append(v / nr)
    return np.array(out).T if out else np.zeros((vectors.shape[0], 0))


def krylov_directions(apply_solve, R, X0, mass, ncols, tol=1e-12):
    """Ordered directions of the block Krylov space of (p0R+F)^{-1}R started
    at X0 = (p0R+F)^{-1}B.  Each block is made orthogonal to all earlier
    directions in the mass inner product <a,b> = a^T diag(mass) b (two
    passes); within a block, directions are ordered by decreasing mass norm
    (eigenvectors of the block's mass Gram matrix) and normalised.  Directions
    with norm below tol times the first block's largest are deflated."""
    dirs = np.zeros((X0.shape[0], 0))
    Xk = X0
    ref = None
    while dirs.shape[1] < ncols:
        Y = Xk
        for _ in range(2):
            if dirs.shape[1]:
                Y = Y - dirs @ (dirs.T @ (mass[:, None] * Y))
        G = Y.T @ (mass[:, None] * Y)
        lam, Z = np.linalg.eigh(0.5 * (G + G.T))
        order = np.argsort(lam)[::-1]
        lam, Z = lam[order], Z[:, order]
        if ref is None:
            ref = lam[0]
        keep = lam > (tol ** 2) * ref
        if not np.any(keep):
            break
        W = (Y @ Z[:, keep]) / np.sqrt(lam[keep])[None, :]
        dirs = np.hstack([dirs, W])
        Xk = apply_solve(R @ W)
    return dirs


def sprim_basis(model, q, p0):
    """V1 (E rows, q1 = ceil(q/2) columns) and V2 (H rows, q2 = floor(q/2)).

    SPRIM splits every Krylov direction into its E and H rows and
    orthonormalises each set (eq. (9)).  When q is below twice the Krylov
    columns generated, both sets are cut from the *same* ordered directions,
    so that each retained E direction keeps its H partner (cutting the E and
    H rows independently pairs unrelated directions and leaves K~ ~ 0)."""
    R, F, B = model["R"], model["F"], model["B"]
    n_e = model["n_e"]
    q1 = (q + 1) // 2
    q2 = q // 2
    mass = R.diagonal().copy()          # diag(De/dt, Dm/dt) > 0
    lu = spla.splu((p0 * R + F).tocsc())
    X0 = lu.solve(B.toarray())
    need = max(q1, q2)
    dirs = krylov_directions(lu.solve, R, X0, mass, need)
    # extra directions let the E/H sets skip dependent columns
    if dirs.shape[1] < need + 8:
        dirs = krylov_directions(lu.solve, R, X0, mass, need + 8)
    V1 = _gs_in_order(dirs[:n_e], q1)
    V2 = _gs_in_order(dirs[n_e:], q2)
    return V1, V2


def congruence(model, V1, V2):
    """Eqs. (11)-(12): R~ = V^T R V, F~ = V^T F V, L~ = V^T L with the block
    diagonal V = diag(V1, V2) (dense; R, F, L sparse)."""
    n1, q1 = V1.shape
    n2, q2 = V2.shape
    V = np.zeros((n1 + n2, q1 + q2))
    V[:n1, :q1] = V1
    V[n1:, q1:] = V2
    Rt = V.T @ (model["R"] @ V)
    Rt = 0.5 * (Rt + Rt.T)
    Ft = V.T @ (model["F"] @ V)
    Lt = V.T @ model["L"].toarray()
    return Rt, Ft, Lt


def _sym_pow(A, p):
    w, Q = np.linalg.eigh(0.5 * (A + A.T))
    return (Q * w ** p) @ Q.T


def cfl_singular_values(Rt, q1, dt):
    """Singular values s_k of R11^{-1/2} K~ R22^{-1/2} (eq. (27))."""
    R11 = dt * Rt[:q1, :q1]
    R22 = dt * Rt[q1:, q1:]
    K = -2.0 * Rt[:q1, q1:]
    M = _sym_pow(R11, -0.5) @ K @ _sym_pow(R22, -0.5)
    return np.linalg.svd(M, compute_uv=False)


def cfl_clip(Rt, Ft, q1, dt, theta=0.99):
    """Enforce s_k <= theta*2/dt by clipping singular values (eq. (27))."""
    R11 = dt * Rt[:q1, :q1]
    R22 = dt * Rt[q1:, q1:]
    K = -2.0 * Rt[:q1, q1:]
    R11h = _sym_pow(R11, 0.5)
    R22h = _sym_pow(R22, 0.5)
    M = _sym_pow(R11, -0.5) @ K @ _sym_pow(R22, -0.5)
    U, s, Wt = np.linalg.svd(M, full_matrices=False)
    smax_before = float(s.max()) if s.size else 0.0
    lim = theta * 2.0 / dt
    if smax_before <= lim:
        return Rt, Ft, smax_before, smax_before, False
    s2 = np.minimum(s, lim)
    Kc = R11h @ (U * s2) @ Wt @ R22h
    Rt = Rt.copy()
    Ft = Ft.copy()
    Rt[:q1, q1:] = -0.5 * Kc
    Rt[q1:, :q1] = -0.5 * Kc.T
    Ft[:q1, q1:] = -0.5 * Kc
    Ft[q1:, :q1] = +0.5 * Kc.T
    return Rt, Ft, smax_before, float(s2.max()), True


def build_rom(eps_r, sigma, r, dx, dy, dt, q, f_max, basis="sprim", clip=True,
              theta=0.99, pec=None):
    """Reduced model of one refined region.

    Returns dict(Rt, Ft, Lt, q1, q2, Sc, smax_before, smax_after, clipped, p0,
    V1, V2, K0 (K~ before the clip), model).
    ``basis='identity'`` skips reduction (V = I, q = restricted state size);
    ``basis=(V1, V2)`` projects on the given basis (a basis built earlier,
    held fixed while the material changes).
    ``pec``: fine cells that are perfect conductors (their samples are
    left out of the model, see ``fine``)."""
    model = fine.restricted_model(eps_r, sigma, r, dx, dy, dt, pec)
    if isinstance(basis, tuple):
        V1, V2 = basis
        p0 = float("nan")
    elif basis == "identity":
        n_e, n_h = model["n_e"], model["n_h"]
        V1 = np.eye(n_e)
        V2 = np.eye(n_h)
        p0 = float("nan")
    else:
        p0 = math.pi * f_max * dt
        if not (0.0 < p0 < 1.0):
            raise ValueError(f"expansion point p0={p0} outside (0, 1)")
        V1, V2 = sprim_basis(model, q, p0)
    q1 = V1.shape[1]
    q2 = V2.shape[1]
    Rt, Ft, Lt = congruence(model, V1, V2)
    K0 = -2.0 * Rt[:q1, q1:]
    smax0 = smax1 = float("nan")
    clipped = False
    if clip:
        Rt, Ft, smax0, smax1, clipped = cfl_clip(Rt, Ft, q1, dt, theta)
    return dict(Rt=Rt, Ft=Ft, Lt=Lt, q1=q1, q2=q2, Sc=model["S"], p0=p0,
                smax_before=smax0, smax_after=smax1, clipped=clipped,
                V1=V1, V2=V2, K0=K0, model=model, theta=theta, dt=dt)


def transfer(Rt, Ft, Lt, Sc, p):
    """H(p) = L^T (p R + F)^{-1} L Sc: the reduced model's response in the
    bilinear variable p = (z-1)/(z+1), invariant under any invertible change
    of reduced coordinates."""
    A = p * Rt + Ft
    return Lt.T @ np.linalg.solve(A, Lt * Sc[None, :])


def transfer_full(model, p):
    A = (p * model["R"] + model["F"]).tocsc()
    X = spla.splu(A).solve(model["B"].toarray().astype(A.dtype))
    return model["L"].T @ X
