"""GPU reverse sweep (fdtd_rom_adjoint through the C ABI) against the CPU
FP64 oracle adjoint, against central finite differences of the GPU's own
FP64 forward, across checkpoint intervals, and through the PyTorch
autograd wrapper.  Bars: FP64 <= 1e-12 relative L2 over the gradient maps;
FP32 <= 1e-5 relative L2 against the oracle's transpose of the FP32
forward (the oracle evaluates it in FP64 arithmetic on the FP32-rounded
coefficients and update matrices, so the bar measures the sweep's own
arithmetic).  Against the FP64 run of the full C5 workload the FP32 maps
are held to 5e-5: that distance is set by rounding the eq. (3)
coefficients and eq. (23) matrices to FP32 (a different discrete problem),
not by the sweep's arithmetic."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import sim as osim
from paper_1609_07114_amd import capi, romgen
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _gpu_adj(prob, roms, nsteps=None, dtype=None, ckpt=0, probe=0):
    nsteps = prob.nsteps if nsteps is None else nsteps
    print(f"[gpu-adjoint] {prob.name} {dtype or prob.dtype} steps={nsteps} ckpt={ckpt}", flush=True)
    with Simulation(prob, roms, max_steps=nsteps, dtype=dtype) as s:
        return s.adjoint(nsteps, probe=probe, ckpt_every=ckpt)


def _gpu_J(prob, roms, nsteps, dtype="f64", probe=0):
    with Simulation(prob, roms, max_steps=nsteps, dtype=dtype) as s:
        s.run(nsteps)
        pr = s.probes(0, nsteps)[:, probe]
    return prob.dt * float(np.sum(pr * pr))


def _compare(g, o, tol):
    Jg, geg, gsg = g
    Jo, geo, gso = o
    print(f"[gpu-adjoint] J {abs(Jg - Jo) / abs(Jo):.2e} eps {rel_l2(geg, geo):.2e} sigma {rel_l2(gsg, gso):.2e}",
          flush=True)
    assert Jg == pytest.approx(Jo, rel=tol)
    assert rel_l2(geg, geo) <= tol, rel_l2(geg, geo)
    assert rel_l2(gsg, gso) <= tol, rel_l2(gsg, gso)


@pytest.fixture(scope="module")
def small():
    p = W.random_problem(31, 30, 26, 250, nroms=1, block=(5, 4), r=2, q=12,
                         dt_frac_coarse=0.9, f_bw=3e9)
    return p, osim.build_roms(p)


@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", TOL32)])
def test_adjoint_matches_oracle_one_model(small, dtype, tol):
    p, roms = small
    o = oadj.adjoint_gradient(p, roms, fp32=(dtype == "f32"))
    _compare(_gpu_adj(p, roms, dtype=dtype), o, tol)


@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", TOL32)])
def test_adjoint_matches_oracle_two_models_ragged(dtype, tol):
    """Two models, a grid whose width is not a multiple of 64, lossless."""
    p = W.random_problem(33, 70, 45, 300, nroms=2, block=(5, 4), r=2, q=10,
                         dt_frac_coarse=0.9, lossy=False, f_bw=3e9)
    roms = osim.build_roms(p)
    o = oadj.adjoint_gradient(p, roms, fp32=(dtype == "f32"))
    _compare(_gpu_adj(p, roms, dtype=dtype), o, tol)


def test_adjoint_no_models_wide_grid():
    p = W.random_problem(35, 130, 20, 200, nroms=0, dt_frac_coarse=0.9, f_bw=3e9)
    _compare(_gpu_adj(p, []), oadj.adjoint_gradient(p, []), TOL64)


@pytest.mark.parametrize("ckpt", [1, 7, 250])
def test_checkpoint_interval_does_not_change_result(small, ckpt):
    """Recomputed segments reproduce the forward states bit for bit, so every
    checkpoint interval (one step, ragged last segment, no recompute beyond
    the initial state) gives the same gradient."""
    p, roms = small
    ref = _gpu_adj(p, roms, dtype="f64", ckpt=0)
    got = _gpu_adj(p, roms, dtype="f64", ckpt=ckpt)
    assert got[0] == ref[0]
    assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_material_table_and_per_cell_arrays_agree(small, dtype):
    """The reverse step reads the material through the handle's 16-bit
    table when it has one, else the per-cell arrays: the same values, so
    the same gradient bit for bit."""
    p, roms = small
    out = []
    for mode in (1, 0):
        with Simulation(p, roms, max_steps=p.nsteps, dtype=dtype) as s:
            assert s.material_mode()[1] > 0
            s.set_material_mode(mode)
            out.append(s.adjoint(p.nsteps, ckpt_every=60))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def test_adjoint_shared_model_gemm_fp32():
    """FP32 run whose regions share one model (MFMA GEMM forward): the
    recomputed forward takes the same path, gradient against the oracle."""
    p = W.many_copies(n=400, nsteps=300, q=40, spacing=48, block=8)
    roms = osim.build_roms(p)
    o = oadj.adjoint_gradient(p, roms, probe=1, fp32=True)
    _compare(_gpu_adj(p, roms, dtype="f32", probe=1), o, TOL32)


def test_adjoint_rejects_bad_calls(small):
    p, roms = small
    with Simulation(p, roms, dtype="f64") as s:
        with pytest.raises(capi.FdtdError):
            s.adjoint(p.nsteps + 1)
        with pytest.raises(capi.FdtdError):
            s.adjoint(10, probe=len(p.probes))
        s.run(1)
        with pytest.raises(capi.FdtdError):
            s.adjoint(10)


def test_adjoint_vs_gpu_finite_differences(small):
    """Central differences of the GPU FP64 forward objective."""
    p, roms = small
    J, ge, gs = _gpu_adj(p, roms, dtype="f64")
    for (i, j) in W.fd_cells(p, count=4, seed=3):
        for name, g, h in (("eps_r", ge, 1e-4 * p.eps_r[j, i]), ("sigma", gs, 1e-5)):
            pp = copy.deepcopy(p)
            getattr(pp, name)[j, i] += h
            pm = copy.deepcopy(p)
            getattr(pm, name)[j, i] -= h
            fd = (_gpu_J(pp, roms, p.nsteps) - _gpu_J(pm, roms, p.nsteps)) / (2 * h)
            assert g[j, i] == pytest.approx(fd, rel=2e-6, abs=1e-6 * np.abs(g).max()), (name, i, j)


def test_autograd_function(small):
    import torch
    from paper_1609_07114_amd.adjoint import probe_energy
    p, roms = small
    J, ge, gs = _gpu_adj(p, roms, dtype="f64")
    er = torch.tensor(p.eps_r, dtype=torch.float64, device="cuda:0", requires_grad=True)
    sg = torch.tensor(p.sigma, dtype=torch.float64, device="cuda:0", requires_grad=True)
    out = probe_energy(er, sg, p, roms, dtype="f64")
    (3.0 * out).backward()
    assert float(out.detach()) == pytest.approx(J, rel=1e-14)
    assert np.allclose(er.grad.cpu().numpy(), 3.0 * ge, rtol=1e-14, atol=0)
    assert np.allclose(sg.grad.cpu().numpy(), 3.0 * gs, rtol=1e-14, atol=0)
    with torch.no_grad():
        J2 = probe_energy(er, sg, p, roms, dtype="f64")
    assert float(J2) == pytest.approx(J, rel=1e-14)


@pytest.fixture(scope="module")
def c5_small():
    """Adjoint workload scaled to 256^2 with 8x8 blocks: the oracle's
    stored trajectory fits in memory and its model build takes seconds."""
    p = W.adjoint_c5(n=256, nsteps=600, block=8, q=24, f_bw=3e9)
    return p, osim.build_roms(p)


@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", TOL32)])
def test_c5_scaled_vs_oracle(c5_small, dtype, tol):
    p, roms = c5_small
    o = oadj.adjoint_gradient(p, roms, fp32=(dtype == "f32"))
    _compare(_gpu_adj(p, roms, dtype=dtype, ckpt=50), o, tol)


@pytest.mark.parametrize("ckpt", [256, 600])
def test_fp32_gradients_fold_every_128_steps(c5_small, ckpt):
    """FP32 runs sum the gradients in FP32 over at most 128 steps, folding
    them into FP64 at multiples of 128 steps and at every checkpoint:
    intervals that are multiples of 128, or one segment over the whole run
    (every state resident), fold at the same steps and agree bit for bit;
    the one-segment sweep also holds the oracle bar."""
    p, roms = c5_small
    ref = _gpu_adj(p, roms, dtype="f32", ckpt=128)
    got = _gpu_adj(p, roms, dtype="f32", ckpt=ckpt)
    assert got[0] == ref[0]
    assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
    if ckpt == p.nsteps:
        _compare(got, oadj.adjoint_gradient(p, roms, fp32=True), TOL32)


@pytest.fixture(scope="module")
def c5_full():
    """The full adjoint workload: 1024^2, four q=64 models (product
    builder), 4000 steps, checkpoints every 200 steps."""
    p = W.adjoint_c5()
    print("[gpu-adjoint] building C5 models", flush=True)
    return p, romgen.build_roms(p)


def test_c5_full_fp64_finite_differences(c5_full):
    """32 random unmasked cells, central differences of the GPU FP64
    forward with h = 1e-4 eps_r and 1e-4 S/m."""
    p, roms = c5_full
    J, ge, gs = _gpu_adj(p, roms, dtype="f64", ckpt=200)
    assert np.abs(ge).max() > 0 and np.abs(gs).max() > 0
    bad = []
    for (i, j) in W.fd_cells(p, count=32):
        for name, g, h in (("eps_r", ge, 1e-4 * p.eps_r[j, i]), ("sigma", gs, 1e-4)):
            pp = copy.deepcopy(p)
            getattr(pp, name)[j, i] += h
            pm = copy.deepcopy(p)
            getattr(pm, name)[j, i] -= h
            fd = (_gpu_J(pp, roms, p.nsteps) - _gpu_J(pm, roms, p.nsteps)) / (2 * h)
            err = abs(g[j, i] - fd)
            if err > 1e-5 * abs(fd) + 1e-7 * np.abs(g).max():
                bad.append((name, i, j, g[j, i], fd))
        print(f"[gpu-adjoint] fd cell ({i},{j}) done", flush=True)
    assert not bad, bad


def test_c5_full_fp32_vs_fp64(c5_full):
    """FP32 gradient maps against the FP64 run of the same workload."""
    p, roms = c5_full
    J64, ge64, gs64 = _gpu_adj(p, roms, dtype="f64", ckpt=200)
    J32, ge32, gs32 = _gpu_adj(p, roms, dtype="f32", ckpt=200)
    print(f"[gpu-adjoint] C5 FP32 vs FP64: J {abs(J32 - J64) / abs(J64):.2e} eps {rel_l2(ge32, ge64):.2e} "
          f"sigma {rel_l2(gs32, gs64):.2e}", flush=True)
    assert J32 == pytest.approx(J64, rel=1e-5)
    assert rel_l2(ge32, ge64) <= 5e-5, rel_l2(ge32, ge64)
    assert rel_l2(gs32, gs64) <= 5e-5, rel_l2(gs32, gs64)


def test_host_plan_equals_handle_workspace_size():
    """The host-only plan of the adjoint workspace (no handle) equals the
    size the handle reports, with and without absorbing layers."""
    cases = [W.random_problem(36, 70, 45, 300, nroms=2, block=(5, 4), r=2, q=10, dtype=d)
             for d in ("f32", "f64")]
    q = W.random_problem(37, 80, 60, 200, nroms=1, block=(5, 4), r=2, q=10)
    q.pml = W.Pml(5, 5, 4, 4)
    q.roms[0].i0, q.roms[0].j0 = 30, 25
    cases.append(q)
    for p in cases:
        roms = osim.build_roms(p)
        for K in (0, 7):
            plan = capi.fdtd_rom_adjoint_plan(capi.ProblemStruct.from_workload(p, roms), p.nsteps, K)
            with Simulation(p, roms) as s:
                assert capi.fdtd_rom_adjoint_workspace_size(s.h, p.nsteps, K) == plan


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ckpt", [0, 7, 250])
def test_handle_after_adjoint_stands_at_nsteps(dtype, ckpt):
    """The forward stops at the last checkpoint and the last segment's
    recompute hands the handle its state: afterwards the probe record, the
    fields and the reduced states equal those of a plain run, bit for bit,
    and the handle runs on exactly as that run does."""
    n, more = 250, 40
    p = W.random_problem(31, 30, 26, n + more, nroms=1, block=(5, 4), r=2, q=12,
                         dt_frac_coarse=0.9, f_bw=3e9)
    roms = osim.build_roms(p)
    with Simulation(p, roms, max_steps=n + more, dtype=dtype) as s:
        s.adjoint(n, ckpt_every=ckpt)
        a = (s.probes(0, n), [s.field(c) for c in range(3)], s.rom_state(0))
        s.run(more)
        a2 = (s.probes(n, more), [s.field(c) for c in range(3)])
    with Simulation(p, roms, max_steps=n + more, dtype=dtype) as s:
        s.run(n)
        b = (s.probes(0, n), [s.field(c) for c in range(3)], s.rom_state(0))
        s.run(more)
        b2 = (s.probes(n, more), [s.field(c) for c in range(3)])
    assert np.array_equal(a[0], b[0])
    for c in range(3):
        assert np.array_equal(a[1][c], b[1][c]) and np.array_equal(a2[1][c], b2[1][c]), c
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a2[0], b2[0])
