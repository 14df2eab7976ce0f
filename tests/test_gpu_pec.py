"""Perfectly conducting cells on the device (fdtd_grid.pec, and PEC fine
cells in the reduced models): a problem with a metal plate that runs from
the wall through a region's ring into the region, a metal corner cell and
an interior metal cell, against the oracle (FP64 <= 1e-12, FP32 <= 1e-5
relative L2 on probes, fields and reduced states), with one launch per step
and with two steps per pass, in a batch (bit-identical to its own handle),
and through the adjoint (FP64 <= 1e-12, FP32 <= 1e-5, the adjoint bars)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import sim as osim
from paper_1609_07114_amd import romgen
from paper_1609_07114_amd.batch import Batch
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu


def _oracle(p, roms, fp32):
    run = osim.CoupledRun(p, roms, mode="closed", fp32=fp32)
    pr = np.empty((p.nsteps, len(p.probes)))
    for n in range(p.nsteps):
        run.step()
        pr[n] = run.probes()
    return dict(probes=pr, hz=run.f.hz * run.cell, ex=run.f.ex, ey=run.f.ey, x=run.x)


@pytest.mark.parametrize("tb", [True, False])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_pec_problem_vs_oracle(tb, dtype, tol):
    p = W.pec_problem(11, r=2, q=12, nsteps=240, dtype=dtype, nx=90, ny=40)
    roms = osim.build_roms(p)
    assert np.all(roms[0]["Lt"][:, [2, 9, 17]] == 0)
    print(f"[gpu-pec] {dtype} tb={tb}", flush=True)
    with Simulation(p, roms) as s:
        s.set_time_blocking(tb)
        s.run(100)
        s.run(140)
        g = dict(probes=s.probes(), hz=s.field(0), ex=s.field(1), ey=s.field(2), x=[s.rom_state(0)])
    o = _oracle(p, roms, dtype == "f32")
    assert np.abs(o["probes"]).max() > 0
    for k in ("probes", "hz", "ex", "ey"):
        assert rel_l2(g[k], o[k]) <= tol, (k, rel_l2(g[k], o[k]))
    assert rel_l2(g["x"][0], o["x"][0]) <= tol
    # the metal's samples stay exactly zero
    pec = p.pec
    assert not np.any(g["hz"][pec])
    assert not np.any(g["ex"][:-1][pec]) and not np.any(g["ex"][1:][pec])
    assert not np.any(g["ey"][:, :-1][pec]) and not np.any(g["ey"][:, 1:][pec])


def test_pec_problem_library_models_and_batch():
    """The library's own models of the region with PEC fine cells, run
    alone and inside a batch with another instance: bit-identical."""
    p = W.pec_problem(12, r=2, q=12, nsteps=160, dtype="f32", nx=70, ny=30)
    other = W.random_problem(13, 50, 40, 160, nroms=1, block=(5, 4), r=2, q=10, dtype="f32")
    roms = romgen.build_roms(p)
    assert np.all(roms[0]["Lt"][:, [2, 9, 17]] == 0)
    roms_o = romgen.build_roms(other)
    with Batch([p, other], [roms, roms_o]) as bt:
        bt.run(160)
        got = bt.probes(0)
    with Simulation(p, roms) as s:
        s.run(160)
        assert np.array_equal(got, s.probes())


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_pec_adjoint_vs_oracle(dtype, tol):
    p = W.pec_problem(7, r=2, q=10, nsteps=200, dtype=dtype)
    roms = osim.build_roms(p)
    o = oadj.adjoint_gradient(p, roms, fp32=(dtype == "f32"))
    with Simulation(p, roms) as s:
        J, ge, gs = s.adjoint(p.nsteps, probe=0, ckpt_every=0)
    assert J == pytest.approx(o[0], rel=tol)
    assert rel_l2(ge, o[1]) <= tol and rel_l2(gs, o[2]) <= tol
    assert not np.any(ge[p.pec]) and not np.any(gs[p.pec])
