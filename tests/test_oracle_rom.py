"""Pins of the oracle's fine-region model, reduction and coupling.

* state counts printed in the paper (Sec. VI: 7,600 / 2,760 / 7,008);
* eq. (24)-(25) structure: R = R^T, F + F^T = diag(Ds, 0) >= 0, B = L S with
  S's signs; R > 0 exactly up to the CFL limit eq. (1) for vacuum;
* coarse-port restriction: B' = P^T B T = Lc Sc;
* Theorem 1 invariants for SPRIM and for random block-diagonal V;
* moment matching at p0 when whole Krylov blocks are kept;
* the clip of eq. (27): no-op below the limit, s_max <= 0.99*2/dt after,
  unclipped model above the fine CFL makes the coupled scheme unstable,
  clipped one keeps spectral radius <= 1 (Theorem 2);
* identity basis == plain Yee (r = 1) and == direct subgridding (r > 1);
* literal eq. (19) == closed form eq. (23);
* exact energy balance (storage function of Sec. V / Appendix).
"""
import copy
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import coupling, fine, rom, sim, subgrid, yee
from oracle.constants import C0, EPS0, MU0
from tests._util import rel_l2, zero_sources
from tests.test_oracle_yee import one_step_matrix


@pytest.mark.parametrize("n,count", [(50, 7600), (30, 2760), (48, 7008)])
def test_paper_state_counts(n, count):
    assert fine.state_count(n, n) == count


def _region(seed, ni=3, nj=2, r=3, lossy=True):
    rng = np.random.default_rng(seed)
    er = rng.uniform(1, 5, (r * nj, r * ni))
    sg = rng.uniform(0, 0.05, (r * nj, r * ni)) if lossy else np.zeros((r * nj, r * ni))
    return er, sg


def test_fine_structure_eq24_25():
    er, sg = _region(0)
    dx, dy, dt = 0.01, 0.012, 1e-12
    m = fine.assemble(er, sg, dx / 3, dy / 3, dt)
    R, F, B, L, S = m["R"], m["F"], m["B"], m["L"], m["S"]
    assert abs(R - R.T).max() == 0.0
    FF = (F + F.T).toarray()
    n_e = m["index"].n_e
    assert np.allclose(FF[:n_e, :n_e], np.diag(m["Ds"]), rtol=0, atol=1e-300)
    assert np.all(FF[n_e:, :] == 0) and np.all(FF[:, n_e:] == 0)
    assert np.all(m["Ds"] >= 0)
    # eq. (25): S = L^T B with signs (-dxh, +dxh, +dyh, -dyh)
    assert np.allclose((L.T @ B).toarray(), np.diag(S))
    Nx, Ny = 9, 6
    assert np.all(S[:Nx] == -dx / 3) and np.all(S[Nx:2 * Nx] == dx / 3)
    assert np.all(S[2 * Nx:2 * Nx + Ny] == dy / 3) and np.all(S[2 * Nx + Ny:] == -dy / 3)
    # (R+F) is upper block-triangular and (R-F) lower: the explicit leap-frog
    RpF = (R + F).toarray()
    RmF = (R - F).toarray()
    assert np.all(RpF[n_e:, :n_e] == 0) and np.all(RmF[:n_e, n_e:] == 0)


def test_fine_update_matches_eq4_south_row():
    """One row of (R+F)x' = (R-F)x + Bu written out: eq. (4) for a South
    boundary Ex with hanging variable."""
    er, sg = _region(1)
    dxh, dyh, dt = 0.004, 0.005, 5e-12
    m = fine.assemble(er, sg, dxh, dyh, dt)
    ix = m["index"]
    rng = np.random.default_rng(2)
    x = rng.standard_normal(ix.n)
    u = rng.standard_normal(m["B"].shape[1])
    xn = sp.linalg.spsolve((m["R"] + m["F"]).tocsc(), (m["R"] - m["F"]) @ x + m["B"] @ u)
    i = 4
    e = ix.ex(i, 0)
    eps = EPS0 * er[0, i]
    lhs = dxh * dyh / 2 * (eps / dt + sg[0, i] / 2) * xn[e]
    rhs = dxh * dyh / 2 * (eps / dt - sg[0, i] / 2) * x[e] + dxh * xn[ix.hz(i, 0)] - dxh * u[i]
    assert lhs == pytest.approx(rhs, rel=1e-10)
    # eq. (5) for one Hz
    h = ix.hz(2, 3)
    lhs = dxh * dyh * MU0 / dt * (xn[h] - x[h])
    rhs = (-dxh * x[ix.ex(2, 3)] + dxh * x[ix.ex(2, 4)] + dyh * x[ix.ey(2, 3)]
           - dyh * x[ix.ey(3, 3)])
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_fine_cfl_equals_eq1_vacuum():
    """R > 0 (eq. (24a)) holds exactly up to the CFL limit of eq. (1) for a
    vacuum region with hanging variables."""
    Nx, Ny = 6, 5
    er = np.ones((Ny, Nx))
    sg = np.zeros((Ny, Nx))
    dxh, dyh = 0.002, 0.0025
    lim = yee.cfl_dt(dxh, dyh, C0)
    m = fine.assemble(er, sg, dxh, dyh, lim)
    n_e = m["index"].n_e
    De, Dm, K = m["De"], m["Dm"], m["K"].toarray()
    M = (K / np.sqrt(De)[:, None]) / np.sqrt(Dm)[None, :]
    smax = np.linalg.svd(M, compute_uv=False).max()
    assert smax * lim / 2 == pytest.approx(1.0, abs=1e-12)
    for f, pos in ((0.999, True), (1.001, False)):
        R = fine.assemble(er, sg, dxh, dyh, f * lim)["R"].toarray()
        mineig = np.linalg.eigvalsh(R / np.sqrt(np.outer(np.diag(R), np.diag(R)))).min()
        assert (mineig > 0) == pos


def test_restriction_input_map():
    er, sg = _region(3, ni=3, nj=2, r=3)
    dx, dy, dt = 0.01, 0.012, 1e-12
    rm = fine.restricted_model(er, sg, 3, dx, dy, dt)
    full = rm["full"]
    P, T = rm["restriction"]["P"], rm["restriction"]["T"]
    lhs = (P.T @ full["B"] @ T).toarray()
    rhs = (rm["L"] @ sp.diags(rm["S"])).toarray()
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-15)
    assert np.allclose(rm["S"], np.r_[[-dx] * 3, [dx] * 3, [dy] * 2, [-dy] * 2])


def test_theorem1_sprim_and_random_blockdiag():
    er, sg = _region(4, ni=3, nj=3, r=2)
    dx, dy = 0.01, 0.01
    dt = 0.99 * yee.cfl_dt(dx / 2, dy / 2, C0)
    m = rom.build_rom(er, sg, 2, dx, dy, dt, 10, 5e9)
    Rt, Ft, Lt, Sc = m["Rt"], m["Ft"], m["Lt"], m["Sc"]
    np.linalg.cholesky(Rt)
    assert np.linalg.eigvalsh(Ft + Ft.T).min() >= -1e-12 * np.abs(Ft).max()
    # B~ = V^T B = L~ Sc (eq. (26c))
    model = m["model"]
    V = sp.block_diag([sp.csr_matrix(m["V1"]), sp.csr_matrix(m["V2"])])
    assert np.allclose((V.T @ model["B"]).toarray(), Lt * Sc[None, :], rtol=0, atol=1e-14)
    # any full-rank block-diagonal V keeps passivity (Theorem 1)
    rng = np.random.default_rng(5)
    for _ in range(3):
        V1 = rng.standard_normal((model["n_e"], 7))
        V2 = rng.standard_normal((model["n_h"], 6))
        R2, F2, L2 = rom.congruence(model, V1, V2)
        np.linalg.cholesky(R2)
        assert np.linalg.eigvalsh(F2 + F2.T).min() >= -1e-12 * np.abs(F2).max()


def test_moment_matching_full_block():
    """With whole first blocks kept (q1, q2 >= ports) the model's response
    equals the unreduced region's at p0."""
    er, sg = _region(6, ni=2, nj=2, r=2)
    dx = dy = 0.01
    dt = 0.99 * yee.cfl_dt(dx / 2, dy / 2, C0)
    n_p = 8
    m = rom.build_rom(er, sg, 2, dx, dy, dt, 2 * n_p, 5e9)
    assert m["q1"] == n_p and m["q2"] == n_p
    H_full = rom.transfer_full(m["model"], m["p0"])
    H_rom = rom.transfer(m["Rt"], m["Ft"], m["Lt"], m["Sc"], m["p0"])
    assert np.max(np.abs(H_rom - H_full)) / np.max(np.abs(H_full)) < 1e-10
    # away from p0 they differ (the test is not vacuous)
    Hf2 = rom.transfer_full(m["model"], 0.9)
    Hr2 = rom.transfer(m["Rt"], m["Ft"], m["Lt"], m["Sc"], 0.9)
    assert np.max(np.abs(Hr2 - Hf2)) / np.max(np.abs(Hf2)) > 1e-8


def _small_coupled(dt_frac_coarse, r=2, lossy=True, seed=11):
    p = W.random_problem(seed, 10, 9, 10, nroms=1, block=(3, 3), r=r, q=0,
                         dt_frac_coarse=dt_frac_coarse, lossy=lossy)
    return zero_sources(p)


def test_cfl_clip_stabilises():
    """dt = 0.95 coarse CFL = 1.9x the fine CFL with r = 2: the unreduced
    region violates eq. (24a); unclipped the coupled scheme has poles
    outside the unit circle, after the clip of eq. (27) it has none."""
    p = _small_coupled(0.95, r=2, lossy=False)
    unc = sim.build_roms(p, basis="identity", clip=False)
    clp = sim.build_roms(p, basis="identity", clip=True)
    assert clp[0]["clipped"]
    assert clp[0]["smax_after"] <= 0.99 * 2 / p.dt * (1 + 1e-12)
    assert clp[0]["smax_before"] > 2 / p.dt
    rho_u = np.max(np.abs(np.linalg.eigvals(one_step_matrix(p, unc))))
    rho_c = np.max(np.abs(np.linalg.eigvals(one_step_matrix(p, clp))))
    assert rho_u > 1 + 1e-3
    assert rho_c < 1 + 1e-9


def test_clip_noop_below_fine_cfl():
    er, sg = _region(7, ni=2, nj=3, r=2)
    dx = dy = 0.01
    dt = 0.9 * yee.cfl_dt(dx / 2, dy / 2, C0)
    a = rom.build_rom(er, sg, 2, dx, dy, dt, 12, 5e9, clip=False)
    b = rom.build_rom(er, sg, 2, dx, dy, dt, 12, 5e9, clip=True)
    assert not b["clipped"]
    assert np.array_equal(a["Rt"], b["Rt"]) and np.array_equal(a["Ft"], b["Ft"])


def test_theorem2_spectral_radius_two_roms():
    p = W.random_problem(12, 16, 12, 10, nroms=2, block=(3, 3), r=2, q=10,
                         dt_frac_coarse=0.9)
    zero_sources(p)
    ms = sim.build_roms(p)
    rho = np.max(np.abs(np.linalg.eigvals(one_step_matrix(p, ms))))
    assert rho < 1 + 1e-9


def test_identity_basis_r1_is_plain_yee():
    p = W.random_problem(1, 20, 18, 150, nroms=1, block=(5, 4), r=1, q=0)
    ms = sim.build_roms(p, basis="identity", clip=False)
    a = sim.run(p, ms, mode="literal")
    pp = copy.deepcopy(p)
    s = p.roms[0]
    pp.eps_r[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.eps_r
    pp.sigma[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.sigma
    pp.roms = []
    b = sim.run(pp, [])
    assert rel_l2(a, b) < 1e-13


def test_identity_basis_r3_is_subgridding():
    p = W.random_problem(3, 24, 22, 200, nroms=2, block=(5, 4), r=3, q=0)
    ms = sim.build_roms(p, basis="identity", clip=False)
    a = sim.run(p, ms, mode="literal")
    b = sim.run(p, ms, mode="closed")
    c = subgrid.run(p)
    assert rel_l2(a, c) < 1e-13
    assert rel_l2(b, c) < 1e-13


def test_literal_equals_closed_form_c1():
    p = W.cavity_c1(nsteps=600)
    ms = sim.build_roms(p)
    a = sim.run(p, ms, mode="literal")
    b = sim.run(p, ms, mode="closed")
    assert rel_l2(b, a) < 1e-13


def test_closed_form_qr_route_equals_literal():
    """The QR route to eq. (23)'s closed form (used to measure how well FP64
    determines it) gives the literal eq. (19) run on a well-conditioned
    model, as the LU route does."""
    p = W.cavity_c1(nsteps=600)
    ms = sim.build_roms(p)
    a = sim.run(p, ms, mode="literal")
    r = sim.CoupledRun(p, ms, mode="closed", solver="qr")
    b = np.empty_like(a)
    for n in range(p.nsteps):
        r.step()
        b[n] = r.probes()
    assert rel_l2(b, a) < 1e-13


@pytest.mark.parametrize("lossy", [True, False])
def test_energy_balance_exact(lossy):
    p = W.random_problem(4, 24, 22, 60, nroms=2, block=(5, 4), r=2, q=12, lossy=lossy)
    zero_sources(p)
    ms = sim.build_roms(p)
    rng = np.random.default_rng(0)
    init = dict(hz=rng.standard_normal((22, 24)), ex=rng.standard_normal((23, 24)) * 300,
                ey=rng.standard_normal((22, 25)) * 300,
                x=[rng.standard_normal(m["Rt"].shape[0]) for m in ms])
    run = sim.CoupledRun(p, ms, mode="literal", init=init)
    e_first = run.energy()
    for n in range(60):
        e0 = run.energy()
        ex0, ey0, x0 = run.f.ex.copy(), run.f.ey.copy(), [x.copy() for x in run.x]
        run.step()
        e1 = run.energy()
        d = run.dissipation(ex0, ey0, x0)
        assert abs(e1 - e0 + d) <= 1e-13 * e_first
        assert d >= -1e-14 * e_first
        if not lossy:
            assert d <= 1e-14 * e_first
    assert run.energy() <= e_first * (1 + 1e-13)


def _pec_problem(r, q=0, seed=1, nsteps=150):
    p = W.pec_problem(seed, r=r, q=q, nsteps=nsteps)
    s = p.roms[0]
    cell, exm, eym = yee.masks(p.nx, p.ny, [(s.i0, s.j0, s.ni, s.nj)], p.pec)
    for src in p.sources:
        m = (cell, exm, eym)[src.comp]
        assert np.all(m[src.j0:src.j1, src.i0:src.i1])
    for pr in p.probes:
        assert (cell, exm, eym)[pr.comp][pr.j, pr.i]
    return p


def test_identity_basis_r1_with_pec_is_plain_yee_with_pec():
    """PEC cells inside a region (fine model without their samples, dead
    ports) and on its ring: with r = 1 and the identity basis the embedded
    run equals plain Yee on the whole grid with the same PEC cells (two
    independent codings of the pinned samples), to round-off."""
    p = _pec_problem(1)
    ms = sim.build_roms(p, basis="identity", clip=False)
    s = p.roms[0]
    m = fine.restricted_model(s.eps_r, s.sigma, 1, p.dx, p.dy, p.dt, s.pec)
    assert m["restriction"]["dead_ports"] == [2, 9, 17]
    assert np.all(ms[0]["Lt"][:, [2, 9, 17]] == 0)
    a = sim.run(p, ms, mode="literal")
    b_lit = sim.run(p, ms, mode="closed")
    pp = copy.deepcopy(p)
    pp.eps_r[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.eps_r
    pp.sigma[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.sigma
    pp.pec[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.pec
    pp.roms = []
    b = sim.run(pp, [])
    assert np.abs(b).max() > 0
    assert rel_l2(a, b) < 1e-13
    assert rel_l2(b_lit, b) < 1e-13


def test_partially_pinned_port_rejected():
    p = _pec_problem(2)
    s = p.roms[0]
    s.pec = np.zeros_like(s.pec)
    s.pec[0, 0] = True                         # one of S port 0's two fine edges
    with pytest.raises(ValueError):
        fine.restricted_model(s.eps_r, s.sigma, 2, p.dx, p.dy, p.dt, s.pec)


def test_pec_reduced_models_passive_and_energy_exact():
    """SPRIM models of a region with PEC cells (r = 2): Theorem 1 invariants,
    the coupled one-step map's spectral radius <= 1 (Theorem 2) and the
    exact energy balance of a lossy run."""
    p = _pec_problem(2, q=12, seed=5, nsteps=40)
    zero_sources(p)
    ms = sim.build_roms(p)
    m = ms[0]
    assert np.all(np.linalg.eigvalsh(m["Rt"]) > 0)
    assert np.min(np.linalg.eigvalsh(m["Ft"] + m["Ft"].T)) > -1e-12 * np.abs(m["Ft"]).max()
    assert np.all(m["Lt"][:, [2, 9, 17]] == 0)
    rho = np.max(np.abs(np.linalg.eigvals(one_step_matrix(p, ms))))
    assert rho < 1 + 1e-9
    rng = np.random.default_rng(2)
    init = dict(hz=rng.standard_normal((p.ny, p.nx)), ex=rng.standard_normal((p.ny + 1, p.nx)) * 300,
                ey=rng.standard_normal((p.ny, p.nx + 1)) * 300, x=[rng.standard_normal(m["Rt"].shape[0])])
    run = sim.CoupledRun(p, ms, mode="literal", init=init)
    e_first = run.energy()
    for n in range(40):
        e0 = run.energy()
        ex0, ey0, x0 = run.f.ex.copy(), run.f.ey.copy(), [x.copy() for x in run.x]
        run.step()
        d = run.dissipation(ex0, ey0, x0)
        assert abs(run.energy() - e0 + d) <= 1e-13 * e_first
        assert d >= -1e-14 * e_first
