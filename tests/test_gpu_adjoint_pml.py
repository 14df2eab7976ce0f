"""GPU reverse sweep through absorbing layers (fdtd_rom_adjoint through the
C ABI): against the oracle's transpose of the layered run, against central
finite differences of the GPU's own FP64 forward at cells inside the
layers, and across checkpoint intervals.  Bars as for the PEC-walled
sweep: FP64 <= 1e-12, FP32 <= 1e-5 relative L2 over the gradient maps.

The grids are wide and tall enough that waves of the reverse step fall
both inside the layers (layer form) and wholly outside them (plain form),
so the hand-over between the two forms is exercised.  The objective's
probe sits inside a layer near a source, so that cells inside the layers
carry a fair share of the gradient; FP64 is also held to its bar on the
layer cells alone."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import sim as osim
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _with_layers(p, want, probe, **grading):
    """Layers of up to `want` = (xlo, xhi, ylo, yhi) cells, thinned so that
    every region and its ring stay two cells clear of them; the objective's
    Hz probe moved to `probe` = (i, j)."""
    p = copy.deepcopy(p)
    p.probes[0] = W.Probe(W.HZ, *probe)
    lim = [want[0], want[1], want[2], want[3]]
    for s in p.roms:
        lim[0] = min(lim[0], s.i0 - 2)
        lim[1] = min(lim[1], p.nx - s.i0 - s.ni - 2)
        lim[2] = min(lim[2], s.j0 - 2)
        lim[3] = min(lim[3], p.ny - s.j0 - s.nj - 2)
    p.pml = W.Pml(*[max(0, v) for v in lim], **grading)
    assert p.pml.any
    return p


def _gpu_adj(prob, roms, dtype=None, ckpt=0):
    print(f"[gpu-adjoint-pml] {prob.nx}x{prob.ny} {dtype or prob.dtype} steps={prob.nsteps} "
          f"ckpt={ckpt} pml={prob.pml}", flush=True)
    with Simulation(prob, roms, max_steps=prob.nsteps, dtype=dtype) as s:
        return s.adjoint(prob.nsteps, ckpt_every=ckpt)


def _gpu_J(prob, roms):
    with Simulation(prob, roms, max_steps=prob.nsteps, dtype="f64") as s:
        s.run(prob.nsteps)
        pr = s.probes(0, prob.nsteps)[:, 0]
    return prob.dt * float(np.sum(pr * pr))


def _layer_cells(p):
    L = p.pml
    m = np.zeros((p.ny, p.nx), bool)
    m[:, :L.n_xlo] = True
    m[:, p.nx - L.n_xhi:] = True
    m[:L.n_ylo] = True
    m[p.ny - L.n_yhi:] = True
    return m


def _compare(p, g, o, tol):
    assert g[0] == pytest.approx(o[0], rel=tol)
    assert rel_l2(g[1], o[1]) <= tol, rel_l2(g[1], o[1])
    assert rel_l2(g[2], o[2]) <= tol, rel_l2(g[2], o[2])
    if tol < 1e-8:
        m = _layer_cells(p)
        assert rel_l2(g[1][m], o[1][m]) <= tol, rel_l2(g[1][m], o[1][m])
        assert rel_l2(g[2][m], o[2][m]) <= tol, rel_l2(g[2][m], o[2][m])


@pytest.fixture(scope="module")
def layered():
    p = W.random_problem(41, 150, 140, 300, nroms=2, block=(5, 4), r=2, q=10,
                         dt_frac_coarse=0.9, f_bw=3e9)
    p = _with_layers(p, (10, 10, 8, 8), (144, 118), kappa_max=3.0, alpha_max=0.03)
    return p, osim.build_roms(p)


@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", TOL32)])
def test_layered_adjoint_vs_oracle(layered, dtype, tol):
    p, roms = layered
    o = oadj.adjoint_gradient(p, roms, fp32=(dtype == "f32"))
    _compare(p, _gpu_adj(p, roms, dtype=dtype), o, tol)


def test_layers_at_the_ends_only_with_models():
    """A waveguide's terminations: layers at the two x ends only."""
    p = W.random_problem(42, 190, 40, 300, nroms=2, block=(5, 4), r=2, q=10,
                         dt_frac_coarse=0.9, f_bw=3e9)
    p = _with_layers(p, (12, 12, 0, 0), (8, 5), m=4.0, kappa_max=2.0, alpha_max=0.02)
    roms = osim.build_roms(p)
    _compare(p, _gpu_adj(p, roms, dtype="f64"), oadj.adjoint_gradient(p, roms), TOL64)


def test_layers_all_sides_no_models_ragged():
    """Uneven layer thicknesses, a width that is not a multiple of the
    reverse step's 61 owned columns, kappa and alpha at their strongest."""
    p = W.random_problem(43, 203, 77, 250, nroms=0, dt_frac_coarse=0.9, f_bw=3e9)
    p = _with_layers(p, (12, 15, 6, 9), (5, 72), m=4.0, kappa_max=5.0, alpha_max=0.05)
    _compare(p, _gpu_adj(p, [], dtype="f64"), oadj.adjoint_gradient(p, []), TOL64)


@pytest.mark.parametrize("ckpt", [1, 7])
def test_layered_checkpoint_interval_does_not_change_result(layered, ckpt):
    """The recompute restores the auxiliary fields with the fields, so the
    layered gradient is the same bit for bit at any checkpoint interval."""
    p, roms = layered
    ref = _gpu_adj(p, roms, dtype="f64")
    got = _gpu_adj(p, roms, dtype="f64", ckpt=ckpt)
    assert got[0] == ref[0]
    assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])


def test_layered_adjoint_vs_gpu_finite_differences():
    """Central differences of the GPU FP64 forward, at cells inside the
    x-low layer around the probe, one in the corner, and the interior."""
    p = W.random_problem(51, 70, 60, 250, nroms=1, block=(5, 4), r=2, q=10,
                         dt_frac_coarse=0.9, f_bw=3e9)
    p = _with_layers(p, (8, 8, 7, 7), (4, 30), kappa_max=3.0, alpha_max=0.03)
    roms = osim.build_roms(p)
    J, ge, gs = _gpu_adj(p, roms, dtype="f64")
    cells = [(3, 28), (6, 33), (2, 30), (7, 25), (5, 10)] + W.fd_cells(p, count=2, seed=9)
    for (i, j) in cells:
        for name, g, h in (("eps_r", ge, 1e-4 * p.eps_r[j, i]), ("sigma", gs, 1e-5)):
            pp = copy.deepcopy(p)
            getattr(pp, name)[j, i] += h
            pm = copy.deepcopy(p)
            getattr(pm, name)[j, i] -= h
            fd = (_gpu_J(pp, roms) - _gpu_J(pm, roms)) / (2 * h)
            assert g[j, i] == pytest.approx(fd, rel=2e-6, abs=1e-6 * np.abs(g).max()), (name, i, j)


@pytest.mark.parametrize("ckpt", [0, 7])
def test_layered_handle_after_adjoint_runs_on_like_a_plain_run(ckpt):
    """With layers the last segment's recompute also hands the handle the
    auxiliary fields: afterwards the handle's probes and fields, and the
    steps it then takes, equal a plain run's bit for bit."""
    n, more = 300, 30
    p = W.random_problem(41, 150, 140, n + more, nroms=2, block=(5, 4), r=2, q=10,
                         dt_frac_coarse=0.9, f_bw=3e9)
    p = _with_layers(p, (10, 10, 8, 8), (144, 118), kappa_max=3.0, alpha_max=0.03)
    roms = osim.build_roms(p)
    with Simulation(p, roms, max_steps=n + more, dtype="f64") as s:
        s.adjoint(n, ckpt_every=ckpt)
        s.run(more)
        a = (s.probes(0, n + more), [s.field(c) for c in range(3)])
    with Simulation(p, roms, max_steps=n + more, dtype="f64") as s:
        s.run(n + more)
        b = (s.probes(0, n + more), [s.field(c) for c in range(3)])
    assert np.array_equal(a[0], b[0])
    for c in range(3):
        assert np.array_equal(a[1][c], b[1][c]), c
