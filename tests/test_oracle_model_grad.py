"""Pins of the oracle's gradients through the reduced models
(oracle.model_grad): central finite differences of the oracle's own
forward run with respect to a model's R~, F~, L~ (random directions), to
the ring cells whose half cells enter eq. (13), and to fine cells through
the model build with the basis held (SPRIM with and without the eq. (27)
clip); the identity basis, where nothing is held, with the clip active;
and the invariance of the fine gradient under a change of basis within the
same column spaces."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import model_grad as mg
from oracle import rom as orom
from oracle import sim as osim


def _problem(r=2, q=12, seed=31, nsteps=250):
    return W.random_problem(seed, 30, 26, nsteps, nroms=1, block=(5, 4), r=r, q=q,
                            dt_frac_coarse=0.9, f_bw=3e9)


@pytest.fixture(scope="module")
def case():
    p = _problem()
    roms = osim.build_roms(p)
    return p, roms, mg.model_gradient(p, roms)


def test_matrix_gradients_match_central_differences(case):
    p, roms, g = case
    rng = np.random.default_rng(1)
    m = roms[0]
    for key in ("Rt", "Ft", "Lt"):
        D = rng.standard_normal(m[key].shape)
        h = 1e-7 * np.linalg.norm(m[key]) / np.linalg.norm(D)
        mp, mm = dict(m), dict(m)
        mp[key] = m[key] + h * D
        mm[key] = m[key] - h * D
        fd = (oadj.objective(p, [mp]) - oadj.objective(p, [mm])) / (2 * h)
        an = float(np.sum(g["models"][0][key] * D))
        assert an == pytest.approx(fd, rel=1e-5), key


def test_update_matrix_gradient_is_sum_of_outer_products(case):
    """dJ/dG against central differences along a random direction of G
    itself (the run applies eq. (23) as one update matrix)."""
    p, roms, g = case
    run = osim.CoupledRun(p, roms, mode="closed")
    G = run.cpl[0].update_matrix()
    D = np.random.default_rng(2).standard_normal(G.shape)
    h = 1e-7 * np.linalg.norm(G) / np.linalg.norm(D)

    def J_of(Gx):
        r = osim.CoupledRun(p, roms, mode="closed")
        r.cpl[0].G32 = Gx       # the run applies this matrix as given
        pr = p.probes[0]
        J = 0.0
        for _ in range(p.nsteps):
            r.step()
            J += p.dt * r.f.hz[pr.j, pr.i] ** 2
        return J
    fd = (J_of(G + h * D) - J_of(G - h * D)) / (2 * h)
    assert float(np.sum(g["models"][0]["G"] * D)) == pytest.approx(fd, rel=1e-6)


def test_ring_cells_match_central_differences(case):
    p, roms, g = case
    s = p.roms[0]
    ring = [(s.i0 - 1, s.j0 + 1), (s.i0 + 2, s.j0 - 1), (s.i0 + s.ni, s.j0 + 2), (s.i0 + 1, s.j0 + s.nj)]
    for (i, j) in ring:
        for arr, h in (("eps_r", 1e-4), ("sigma", 1e-5)):
            pp, pm = copy.deepcopy(p), copy.deepcopy(p)
            getattr(pp, arr)[j, i] += h
            getattr(pm, arr)[j, i] -= h
            fd = (oadj.objective(pp, roms) - oadj.objective(pm, roms)) / (2 * h)
            assert g[arr][j, i] == pytest.approx(fd, rel=1e-6), (i, j, arr)
            assert g[arr][j, i] != 0.0


def test_outside_cells_equal_plain_adjoint_and_inside_zero(case):
    p, roms, g = case
    J, ge, gs = oadj.adjoint_gradient(p, roms)
    m = oadj.gradient_mask(p)
    assert g["J"] == J
    assert np.array_equal(g["eps_r"][m], ge[m]) and np.array_equal(g["sigma"][m], gs[m])
    s = p.roms[0]
    assert np.all(g["eps_r"][s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] == 0.0)


def _fine_fd_check(p, full, basis, cells, rel):
    s = p.roms[0]

    def model(er, sg):
        m = orom.build_rom(er, sg, s.r, p.dx, p.dy, p.dt, full["Rt"].shape[0], s.f_max, basis=basis)
        return [dict(Rt=m["Rt"], Ft=m["Ft"], Lt=m["Lt"])]
    g = mg.model_gradient(p, model(s.eps_r, s.sigma))
    ge, gs = mg.build_vjp(full, g["models"][0]["Rt"], g["models"][0]["Ft"])
    for (i, j) in cells:
        for arr, h, gg in (("eps_r", 1e-4 * s.eps_r[j, i], ge), ("sigma", 1e-4, gs)):
            a = getattr(s, arr)
            ap, am = a.copy(), a.copy()
            ap[j, i] += h
            am[j, i] -= h
            if arr == "eps_r":
                fd = (oadj.objective(p, model(ap, s.sigma)) - oadj.objective(p, model(am, s.sigma))) / (2 * h)
            else:
                fd = (oadj.objective(p, model(s.eps_r, ap)) - oadj.objective(p, model(s.eps_r, am))) / (2 * h)
            assert gg[j, i] == pytest.approx(fd, rel=rel, abs=1e-6 * np.abs(gg).max()), (i, j, arr)
    return ge, gs


def test_fine_cells_sprim_basis_held():
    p = _problem()
    s = p.roms[0]
    full = orom.build_rom(s.eps_r, s.sigma, s.r, p.dx, p.dy, p.dt, s.q, s.f_max)
    assert not full["clipped"]
    Ny, Nx = s.eps_r.shape
    _fine_fd_check(p, full, (full["V1"], full["V2"]), [(0, 0), (3, 2), (Nx - 1, Ny - 1), (0, 4)], 1e-5)


def test_fine_cells_sprim_clip_active_and_basis_invariance():
    """r = 3, q = 140: the reduced model keeps modes beyond the step's limit,
    so eq. (27) clips; the gradient goes through the clip."""
    p = _problem(r=3, q=140)
    s = p.roms[0]
    full = orom.build_rom(s.eps_r, s.sigma, s.r, p.dx, p.dy, p.dt, s.q, s.f_max)
    assert full["clipped"] and full["smax_before"] > full["smax_after"]
    Ny, Nx = s.eps_r.shape
    ge, gs = _fine_fd_check(p, full, (full["V1"], full["V2"]), [(0, 0), (4, 3), (Nx - 1, Ny - 1), (7, 0)],
                            1e-5)
    rng = np.random.default_rng(3)
    Q1 = np.linalg.qr(rng.standard_normal((full["q1"],) * 2))[0]
    Q2 = np.linalg.qr(rng.standard_normal((full["q2"],) * 2))[0]
    rot = orom.build_rom(s.eps_r, s.sigma, s.r, p.dx, p.dy, p.dt, s.q, s.f_max,
                         basis=(full["V1"] @ Q1, full["V2"] @ Q2))
    g2 = mg.model_gradient(p, [dict(Rt=rot["Rt"], Ft=rot["Ft"], Lt=rot["Lt"])])
    ge2, gs2 = mg.build_vjp(rot, g2["models"][0]["Rt"], g2["models"][0]["Ft"])
    assert np.linalg.norm(ge2 - ge) <= 1e-9 * np.linalg.norm(ge)
    assert np.linalg.norm(gs2 - gs) <= 1e-9 * np.linalg.norm(gs)


def test_fine_cells_identity_basis_whole_pipeline():
    """No basis to hold: the finite differences rebuild everything
    (restriction, congruence with V = I, the active clip)."""
    p = _problem()
    s = p.roms[0]
    full = orom.build_rom(s.eps_r, s.sigma, s.r, p.dx, p.dy, p.dt, 0, s.f_max, basis="identity")
    assert full["clipped"]
    Ny, Nx = s.eps_r.shape
    _fine_fd_check(p, full, "identity", [(0, 0), (3, 2), (Nx - 1, Ny - 1), (5, 0)], 1e-5)
