"""Pins of the oracle's discrete adjoint: central finite differences of the
oracle's own forward run (lossy and lossless, with embedded models), zero
gradient on masked cells, and the objective's definition."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import sim as osim


@pytest.fixture(scope="module")
def case():
    p = W.random_problem(31, 30, 26, 250, nroms=1, block=(5, 4), r=2, q=12,
                         dt_frac_coarse=0.9, f_bw=3e9)
    roms = osim.build_roms(p)
    J, ge, gs = oadj.adjoint_gradient(p, roms)
    return p, roms, J, ge, gs


def _fd(p, roms, arr, i, j, h):
    pp = copy.deepcopy(p)
    getattr(pp, arr)[j, i] += h
    pm = copy.deepcopy(p)
    getattr(pm, arr)[j, i] -= h
    return (oadj.objective(pp, roms) - oadj.objective(pm, roms)) / (2 * h)


def test_objective_is_time_integrated_probe_energy(case):
    p, roms, J, _, _ = case
    pr = osim.run(p, roms, mode="closed")[:, 0]
    assert J == pytest.approx(p.dt * np.sum(pr ** 2), rel=1e-12)


def test_adjoint_matches_central_differences(case):
    p, roms, J, ge, gs = case
    m = oadj.gradient_mask(p)
    rng = np.random.default_rng(0)
    cells = [(i, j) for j in range(1, p.ny - 1) for i in range(1, p.nx - 1) if m[j, i]]
    for k in rng.choice(len(cells), 5, replace=False):
        i, j = cells[k]
        fd_e = _fd(p, roms, "eps_r", i, j, 1e-4)
        fd_s = _fd(p, roms, "sigma", i, j, 1e-5)
        assert ge[j, i] == pytest.approx(fd_e, rel=2e-6, abs=1e-6 * np.abs(ge).max())
        assert gs[j, i] == pytest.approx(fd_s, rel=2e-6, abs=1e-6 * np.abs(gs).max())


def test_adjoint_lossless_two_models():
    p = W.random_problem(33, 34, 28, 200, nroms=2, block=(4, 4), r=2, q=10,
                         dt_frac_coarse=0.9, lossy=False, f_bw=3e9)
    roms = osim.build_roms(p)
    J, ge, gs = oadj.adjoint_gradient(p, roms)
    m = oadj.gradient_mask(p)
    assert np.all(ge[~m] == 0) and np.all(gs[~m] == 0)
    (i, j) = [(i, j) for j in range(2, p.ny - 2) for i in range(2, p.nx - 2) if m[j, i]][17]
    assert ge[j, i] == pytest.approx(_fd(p, roms, "eps_r", i, j, 1e-4), rel=2e-6,
                                     abs=1e-6 * np.abs(ge).max())
    assert gs[j, i] == pytest.approx(_fd(p, roms, "sigma", i, j, 1e-5), rel=2e-6,
                                     abs=1e-6 * np.abs(gs).max())


def test_fp32_coefficient_mode_tracks_fp64(case):
    """The FP32-coefficient variant (the transpose of the forward an FP32 run
    computes) stays within FP32 coefficient rounding of the FD-pinned FP64
    gradient."""
    p, roms, J, ge, gs = case
    J32, ge32, gs32 = oadj.adjoint_gradient(p, roms, fp32=True)
    assert J32 == pytest.approx(J, rel=1e-5)
    assert np.linalg.norm(ge32 - ge) <= 1e-4 * np.linalg.norm(ge)
    assert np.linalg.norm(gs32 - gs) <= 1e-4 * np.linalg.norm(gs)


def test_transpose_step_dot_product_identity():
    """<M ds, lam> = <ds, M^T lam> for one forward step of the oracle (no
    sources, two models, lossy): the reverse step is the exact transpose of
    the forward step on the state space (active and interface E, active Hz,
    reduced states)."""
    p = W.random_problem(34, 36, 30, 10, nroms=2, block=(5, 4), r=2, q=10,
                         dt_frac_coarse=0.9, f_bw=3e9)
    for s in p.sources:
        s.incr[:] = 0.0
    roms = osim.build_roms(p)
    run = osim.CoupledRun(p, roms, mode="closed")
    rng = np.random.default_rng(7)
    mx = run.exm.astype(float)
    my = run.eym.astype(float)
    for c in run.cpl:
        for (comp, ei, ej, _, _, _, _) in c.ports:
            (mx if comp == 1 else my)[ej, ei] = 1.0
    ds = (rng.standard_normal(mx.shape) * mx, rng.standard_normal(my.shape) * my,
          rng.standard_normal(run.cell.shape) * run.cell,
          [rng.standard_normal(c.q) for c in run.cpl])
    lam = (rng.standard_normal(mx.shape) * mx, rng.standard_normal(my.shape) * my,
           rng.standard_normal(run.cell.shape) * run.cell,
           [rng.standard_normal(c.q) for c in run.cpl])
    run.f.ex[...] = ds[0]
    run.f.ey[...] = ds[1]
    run.f.hz[...] = ds[2]
    run.x = [x.copy() for x in ds[3]]
    run.step()
    Mds = (run.f.ex, run.f.ey, run.f.hz * run.cell, run.x)

    def dot(a, b):
        return (np.sum(a[0] * b[0]) + np.sum(a[1] * b[1]) + np.sum(a[2] * b[2]) +
                sum(float(u @ v) for u, v in zip(a[3], b[3])))
    Gs = [c.update_matrix() for c in run.cpl]
    MTlam, _ = oadj.transpose_step(run, Gs, lam)
    lhs, rhs = dot(Mds, lam), dot(ds, MTlam)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0), (lhs, rhs)


def _layered(seed, nsteps=250, pml=None):
    p = W.random_problem(seed, 34, 30, nsteps, nroms=1, block=(4, 4), r=2, q=10,
                         dt_frac_coarse=0.9, f_bw=3e9)
    s = p.roms[0]
    p.pml = pml or W.Pml(n_xlo=min(5, s.i0 - 1), n_xhi=min(5, p.nx - s.i0 - s.ni - 1),
                         n_ylo=min(4, s.j0 - 1), n_yhi=min(4, p.ny - s.j0 - s.nj - 1),
                         kappa_max=3.0, alpha_max=0.03)
    assert p.pml.any
    return p


def test_transpose_step_with_layers():
    """The dot-product identity of one step with absorbing layers: the
    state now also holds the four auxiliary fields (random in the test)."""
    p = _layered(35, nsteps=10)
    for s in p.sources:
        s.incr[:] = 0.0
    roms = osim.build_roms(p)
    run = osim.CoupledRun(p, roms, mode="closed")
    rng = np.random.default_rng(8)
    mx = run.exm.astype(float)
    my = run.eym.astype(float)
    for c in run.cpl:
        for (comp, ei, ej, _, _, _, _) in c.ports:
            (mx if comp == 1 else my)[ej, ei] = 1.0
    shapes = [run.pml.psi_hx.shape, run.pml.psi_hy.shape, run.pml.psi_ex.shape, run.pml.psi_ey.shape]

    def draw():
        return ((rng.standard_normal(mx.shape) * mx, rng.standard_normal(my.shape) * my,
                 rng.standard_normal(run.cell.shape) * run.cell, [rng.standard_normal(c.q) for c in run.cpl])
                + tuple(rng.standard_normal(sh) for sh in shapes))
    ds, lam = draw(), draw()
    run.f.ex[...] = ds[0]
    run.f.ey[...] = ds[1]
    run.f.hz[...] = ds[2]
    run.x = [x.copy() for x in ds[3]]
    run.pml.psi_hx, run.pml.psi_hy, run.pml.psi_ex, run.pml.psi_ey = (a.copy() for a in ds[4:])
    run.step()
    Mds = (run.f.ex, run.f.ey, run.f.hz * run.cell, run.x,
           run.pml.psi_hx, run.pml.psi_hy, run.pml.psi_ex, run.pml.psi_ey)

    def dot(a, b):
        return (sum(np.sum(u * v) for k, (u, v) in enumerate(zip(a, b)) if k != 3) +
                sum(float(u @ v) for u, v in zip(a[3], b[3])))
    Gs = [c.update_matrix() for c in run.cpl]
    MTlam, _ = oadj.transpose_step(run, Gs, lam)
    lhs, rhs = dot(Mds, lam), dot(ds, MTlam)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0), (lhs, rhs)


def test_adjoint_with_layers_matches_central_differences():
    """Gradients through absorbing layers (kappa and alpha active) against
    central differences, at cells inside a layer and in the interior."""
    p = _layered(36)
    roms = osim.build_roms(p)
    J, ge, gs = oadj.adjoint_gradient(p, roms)
    m = oadj.gradient_mask(p)
    L = p.pml
    in_layer = [(i, j) for j in range(1, p.ny - 1) for i in range(1, p.nx - 1)
                if m[j, i] and (i < L.n_xlo or i >= p.nx - L.n_xhi or j < L.n_ylo or j >= p.ny - L.n_yhi)]
    interior = [(i, j) for j in range(1, p.ny - 1) for i in range(1, p.nx - 1)
                if m[j, i] and (i, j) not in in_layer]
    rng = np.random.default_rng(2)
    picks = [in_layer[k] for k in rng.choice(len(in_layer), 3, replace=False)] + \
            [interior[k] for k in rng.choice(len(interior), 2, replace=False)]
    for (i, j) in picks:
        fd_e = _fd(p, roms, "eps_r", i, j, 1e-4)
        fd_s = _fd(p, roms, "sigma", i, j, 1e-5)
        assert ge[j, i] == pytest.approx(fd_e, rel=2e-6, abs=1e-6 * np.abs(ge).max()), (i, j)
        assert gs[j, i] == pytest.approx(fd_s, rel=2e-6, abs=1e-6 * np.abs(gs).max()), (i, j)


def test_adjoint_with_pec_cells_matches_central_differences():
    """PEC cells on the coarse grid and inside the region (a plate touching
    a port): cells next to the metal against central differences of the
    forward, and zero gradient on the PEC cells themselves."""
    p = W.pec_problem(7, r=2, q=10, nsteps=200)
    roms = osim.build_roms(p)
    J, ge, gs = oadj.adjoint_gradient(p, roms)
    m = oadj.gradient_mask(p)
    assert not m[p.pec].any()
    assert np.all(ge[p.pec] == 0) and np.all(gs[p.pec] == 0)
    s = p.roms[0]
    # cells beside the coarse PEC plate (below the region's ring) and a far one
    ci = s.i0 + 2
    cells = [(ci - 1, s.j0 - 3), (ci + 1, s.j0 - 3)]
    cells = [(i, j) for (i, j) in cells if 0 <= j and m[j, i]]
    assert cells
    for (i, j) in cells:
        assert ge[j, i] == pytest.approx(_fd(p, roms, "eps_r", i, j, 1e-4), rel=2e-6,
                                         abs=1e-6 * np.abs(ge).max())
        assert gs[j, i] == pytest.approx(_fd(p, roms, "sigma", i, j, 1e-5), rel=2e-6,
                                         abs=1e-6 * np.abs(gs).max())
