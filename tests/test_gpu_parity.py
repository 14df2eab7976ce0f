"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle
on identical seeded inputs and identical reduced models (built by the
oracle).  Bars: FP64 runs <= 1e-12 relative L2, FP32 runs <= 1e-5 relative
L2 against the oracle evaluated in FP64 with the FP32-rounded coefficients
and coupling matrices an FP32 run computes with."""
import copy
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from oracle import subgrid as osub
from paper_1609_07114_amd import capi
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _gpu_run(prob, roms, nsteps=None, dtype=None, chunks=None, x0=None):
    nsteps = prob.nsteps if nsteps is None else nsteps
    print(f"[gpu] {prob.name} {dtype or prob.dtype} steps={nsteps} roms={len(roms)}", flush=True)
    with Simulation(prob, roms, max_steps=nsteps, dtype=dtype, x0=x0) as s:
        if chunks:
            done = 0
            for c in chunks:
                s.run(c)
                done += c
            s.run(nsteps - done)
        else:
            s.run(nsteps)
        out = dict(probes=s.probes(), hz=s.field(0), ex=s.field(1), ey=s.field(2),
                   x=[s.rom_state(k) for k in range(len(roms))])
    return out


def _oracle(prob, roms, nsteps=None, fp32=False, mode="closed", init=None):
    run = osim.CoupledRun(prob, roms, mode=mode, fp32=fp32, init=init)
    nsteps = prob.nsteps if nsteps is None else nsteps
    pr = np.empty((nsteps, len(prob.probes)))
    for n in range(nsteps):
        run.step()
        pr[n] = run.probes()
    return dict(probes=pr, hz=run.f.hz * run.cell, ex=run.f.ex, ey=run.f.ey, x=run.x)


def _compare(g, o, tol, fields=True):
    assert rel_l2(g["probes"], o["probes"]) <= tol, rel_l2(g["probes"], o["probes"])
    if fields:
        for k in ("hz", "ex", "ey"):
            assert rel_l2(g[k], o[k]) <= tol, (k, rel_l2(g[k], o[k]))
        if len(g["x"]):
            # all reduced states as one vector: a region the wave has not
            # reached holds values below FP32's normal range in the oracle
            a = np.concatenate(g["x"])
            b = np.concatenate(o["x"])
            assert rel_l2(a, b) <= tol, rel_l2(a, b)


def test_c1_cavity_fp64_literal():
    """60x60 cavity, one order-40 model, 2000 steps, FP64: against the
    oracle's literal eq. (19) solve."""
    p = W.cavity_c1()
    roms = osim.build_roms(p)
    g = _gpu_run(p, roms)
    o = _oracle(p, roms, mode="literal")
    assert np.max(np.abs(o["probes"])) > 1e-3
    _compare(g, o, TOL64)


@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", TOL32)])
def test_random_two_models_full_state(dtype, tol):
    p = W.random_problem(3, 70, 45, 400, nroms=2, block=(5, 4), r=2, q=12)
    roms = osim.build_roms(p)
    g = _gpu_run(p, roms, dtype=dtype)
    o = _oracle(p, roms, fp32=(dtype == "f32"))
    _compare(g, o, tol)


@pytest.mark.parametrize("nx,ny", [(65, 33), (130, 77), (64, 64), (200, 5), (3, 90)])
@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", TOL32)])
def test_ragged_grids_no_models(nx, ny, dtype, tol):
    """Tile tails in x (64-wide waves) and y (segments), all source and
    probe components, no reduced regions."""
    p = W.random_problem(40 + nx, nx, ny, 150, nroms=0)
    g = _gpu_run(p, [], dtype=dtype)
    o = _oracle(p, [], fp32=(dtype == "f32"))
    _compare(g, o, tol)


def test_chunked_runs_equal_one_run():
    p = W.random_problem(8, 50, 40, 120, nroms=1, block=(5, 5), r=2, q=10)
    roms = osim.build_roms(p)
    a = _gpu_run(p, roms, dtype="f64")
    b = _gpu_run(p, roms, dtype="f64", chunks=[1, 1, 7, 50])
    assert np.array_equal(a["probes"], b["probes"])
    assert np.array_equal(a["hz"], b["hz"])


def test_identity_basis_r1_is_plain_yee():
    p = W.random_problem(1, 90, 70, 300, nroms=1, block=(5, 4), r=1, q=0)
    roms = osim.build_roms(p, basis="identity", clip=False)
    g = _gpu_run(p, roms, dtype="f64")
    pp = copy.deepcopy(p)
    s = p.roms[0]
    pp.eps_r[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.eps_r
    pp.sigma[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.sigma
    pp.roms = []
    ref = osim.run(pp, [])
    assert rel_l2(g["probes"], ref) <= TOL64


def test_identity_basis_r2_is_subgridding():
    p = W.random_problem(3, 40, 36, 300, nroms=2, block=(5, 4), r=2, q=0)
    roms = osim.build_roms(p, basis="identity", clip=False)
    g = _gpu_run(p, roms, dtype="f64")
    ref = osub.run(p)
    assert rel_l2(g["probes"], ref) <= TOL64


def test_initial_reduced_state_energy_decay():
    """Start from a random reduced state (no source): the run must follow
    the oracle and the oracle's storage function must not increase."""
    p = W.random_problem(9, 40, 36, 200, nroms=2, block=(5, 4), r=2, q=12)
    for s in p.sources:
        s.incr[:] = 0
    roms = osim.build_roms(p)
    rng = np.random.default_rng(3)
    x0 = [rng.standard_normal(m["Rt"].shape[0]) for m in roms]
    g = _gpu_run(p, roms, dtype="f64", x0=x0)
    init = dict(hz=np.zeros((p.ny, p.nx)), ex=np.zeros((p.ny + 1, p.nx)),
                ey=np.zeros((p.ny, p.nx + 1)), x=x0)
    o = _oracle(p, roms, init=init)
    _compare(g, o, TOL64)


def test_random_media_256_fp32():
    """Reduced C2 recipe: 256^2 random patch medium, four models of orders
    16-48, dt = 0.95 coarse CFL, 1500 steps, FP32."""
    p = W.random_media(n=256, nsteps=1500, spacing=128, offset=48, block=16,
                       qs=(16, 24, 32, 48), n_probe_side=4)
    roms = osim.build_roms(p)
    g = _gpu_run(p, roms)
    o = _oracle(p, roms, fp32=True)
    assert np.max(np.abs(o["probes"])) > 0
    _compare(g, o, TOL32)


def test_max_steps_enforced():
    p = W.random_problem(2, 30, 30, 10, nroms=0)
    with Simulation(p, [], max_steps=10) as s:
        s.run(10)
        with pytest.raises(capi.FdtdError) as e:
            s.run(1)
        assert e.value.status == capi.FDTD_ESTATE


def test_product_models_end_to_end():
    """The library's own model builder feeding the GPU run vs the oracle's
    builder feeding the oracle run (FP64): the two builds differ only by a
    change of reduced coordinates, so the probes agree to round-off."""
    from paper_1609_07114_amd import romgen
    p = W.random_media(n=256, nsteps=800, spacing=128, offset=48, block=16,
                       qs=(16, 24, 32, 48), n_probe_side=4, dtype="f64")
    lib_roms = romgen.build_roms(p)
    ora_roms = osim.build_roms(p)
    g = _gpu_run(p, lib_roms)
    o = _oracle(p, ora_roms)
    assert rel_l2(g["probes"], o["probes"]) <= 1e-9
    for k in ("hz", "ex", "ey"):
        assert rel_l2(g[k], o[k]) <= 1e-9


GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _c2_models(prob):
    """Oracle-built models of the 2048^2 workload (tests/golden/make_c2_golden.py)."""
    z = np.load(os.path.join(GOLD, "c2_models.npz"))
    return [dict(Rt=z[f"R{k}"], Ft=z[f"F{k}"], Lt=z[f"L{k}"]) for k in range(len(prob.roms))]


def test_full_size_random_media_2048_fp32_active_models():
    """The 2048^2 benchmark configuration itself (16 models, FP32), started
    from random reduced states so every model is active at once; 40 steps
    compared element by element on all fields, states and probes."""
    p = W.random_media(n=2048, nsteps=40)
    roms = _c2_models(p)
    rng = np.random.default_rng(11)
    x0 = [rng.standard_normal(m["Rt"].shape[0]) for m in roms]
    g = _gpu_run(p, roms, x0=x0)
    init = dict(hz=np.zeros((p.ny, p.nx)), ex=np.zeros((p.ny + 1, p.nx)),
                ey=np.zeros((p.ny, p.nx + 1)), x=x0)
    o = _oracle(p, roms, fp32=True, init=init)
    assert np.max(np.abs(o["hz"])) > 0
    _compare(g, o, TOL32)


def test_full_size_random_media_2048_fp32_10000_steps():
    """The whole 10,000-step 2048^2 run in the benchmark's launch
    configuration: all 64 probe series against the oracle's stored run."""
    path = os.path.join(GOLD, "c2_probes_f32.npz")
    z = np.load(path)
    ref = z["probes"].astype(np.float64)
    n = int(z["steps"])
    p = W.random_media(n=2048, nsteps=n)
    roms = _c2_models(p)
    with Simulation(p, roms, max_steps=n) as s:
        s.run(n)
        got = s.probes()
    assert np.max(np.abs(ref)) > 0
    err = rel_l2(got, ref)
    print(f"2048^2 x {n} steps: rel L2 vs oracle = {err:.3e}", flush=True)
    assert err <= TOL32


def test_graph_replays_match_eager():
    """Captured step batches replayed several times (with host reads and
    synchronisations in between, and odd remainders) give bit-identical
    results to direct launches."""
    import torch
    p = W.random_problem(8, 70, 45, 300, nroms=2, block=(5, 4), r=2, q=12, dtype="f32")
    roms = osim.build_roms(p)
    eager = _gpu_run(p, roms)
    with Simulation(p, roms, max_steps=300) as s:
        s.set_graph(16)
        mids = []
        for chunk in (40, 3, 16, 100, 141):
            s.run(chunk)
            torch.cuda.synchronize()
            mids.append(s.probes(0, s.steps_done))
        got = dict(probes=s.probes(), hz=s.field(0), ex=s.field(1), ey=s.field(2))
    assert np.array_equal(got["probes"], eager["probes"])
    for k in ("hz", "ex", "ey"):
        assert np.array_equal(got[k], eager[k])
    for m in mids:
        assert np.array_equal(m, eager["probes"][:m.shape[0]])


@pytest.mark.parametrize("nx,ny", [(130, 77), (124, 40), (125, 33), (63, 9), (3, 20)])
@pytest.mark.parametrize("seg", [4, 8, 32])
def test_tilings_match(nx, ny, seg):
    """Every tiling (rows per wave segment) gives bit-identical fields,
    including ragged tails of the 62-column tiles."""
    nroms = 2 if nx > 20 else 0
    p = W.random_problem(12 + nx, nx, ny, 120, nroms=nroms, block=(5, 4), r=2, q=12)
    roms = osim.build_roms(p)
    ref = _gpu_run(p, roms)
    with Simulation(p, roms, max_steps=120) as s:
        s.set_tiling(seg)
        s.run(120)
        got = dict(probes=s.probes(), hz=s.field(0), ex=s.field(1), ey=s.field(2))
    for k in ("probes", "hz", "ex", "ey"):
        assert np.array_equal(got[k], ref[k]), k
    o = _oracle(p, roms)
    _compare(got | dict(x=[]), o, TOL64, fields=True)


@pytest.mark.parametrize("q,block,spacing,n", [(128, 32, 128, 1024), (40, 8, 48, 400)])
def test_shared_model_mfma_gemm(q, block, spacing, n):
    """Many copies of one model: the FP32 MFMA GEMM over all copies, the
    per-copy GEMV path and the oracle agree."""
    p = W.many_copies(n=n, nsteps=200, q=q, spacing=spacing, block=block)
    assert len(p.roms) >= 16
    roms = osim.build_roms(p)
    with Simulation(p, roms, max_steps=200) as s:
        s.run(200)
        gemm = dict(probes=s.probes(), hz=s.field(0), ex=s.field(1), ey=s.field(2),
                    x=[s.rom_state(k) for k in range(len(roms))])
    with Simulation(p, roms, max_steps=200) as s:
        s.set_shared_gemm(False)
        s.run(200)
        gemv = dict(probes=s.probes(), hz=s.field(0), ex=s.field(1), ey=s.field(2))
    for k in ("probes", "hz", "ex", "ey"):
        assert rel_l2(gemm[k], gemv[k]) <= TOL32, (k, rel_l2(gemm[k], gemv[k]))
    assert np.max(np.abs(gemm["x"][0])) > 0
    o = _oracle(p, roms, fp32=True)
    _compare(gemm, o, TOL32)


def _c3_golden():
    zm = np.load(os.path.join(GOLD, "c3_model.npz"))
    z = np.load(os.path.join(GOLD, "c3_probes.npz"))
    return dict(Rt=zm["Rt"], Ft=zm["Ft"], Lt=zm["Lt"]), z


@pytest.mark.parametrize("gemm", [True, False])
def test_full_size_many_copies_4096_fp32(gemm):
    """The 4096^2 many-copies workload itself (256 regions sharing one
    oracle-built order-128 model, FP32) in the benchmark's launch
    configuration (two steps per pass, captured graph batches, the shared
    MFMA GEMM or a GEMV per copy) over the oracle's stored 1200-step run
    (tests/golden/make_c3_golden.py): all 16 probe series, a row and a
    column of the final Hz and four regions' reduced states, each within
    1e-5 relative L2 of the oracle evaluated on the same FP32-rounded
    coefficients and update matrix.  The distance to the oracle's run of
    the unrounded FP64 problem is printed beside it."""
    m, z = _c3_golden()
    n = int(z["steps"])
    p = W.many_copies(nsteps=n)
    print(f"[gpu] many copies 4096^2 x {n} steps, gemm={gemm}", flush=True)
    with Simulation(p, [m] * len(p.roms), max_steps=n) as s:
        s.set_shared_gemm(gemm)
        assert s.time_blocking()
        s.set_graph(200)
        s.run(n)
        got = s.probes()
        hz = s.field(0)
        xs = np.stack([s.rom_state(int(k)) for k in z["state_regions"]])
    ref = z["probes_f32"]
    assert np.max(np.abs(ref)) > 0
    e_p = rel_l2(got, ref)
    e_row = rel_l2(hz[p.ny // 2], z["hz_row_f32"])
    e_col = rel_l2(hz[:, int(z["hz_col_index"])], z["hz_col_f32"])
    e_x = rel_l2(xs, z["x_f32"])
    e_64 = rel_l2(got, z["probes_f64"])
    print(f"[gpu] vs oracle: probes {e_p:.2e} hz row {e_row:.2e} col {e_col:.2e} states {e_x:.2e}; "
          f"probes vs unrounded FP64 {e_64:.2e}", flush=True)
    assert np.max(np.abs(z["x_f32"])) > 0 and np.max(np.abs(z["hz_col_f32"])) > 0
    for what, e in (("probes", e_p), ("hz row", e_row), ("hz col", e_col), ("states", e_x)):
        assert e <= TOL32, (what, e)
