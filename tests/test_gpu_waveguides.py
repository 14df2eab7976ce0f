"""The paper's open-waveguide workloads on the device (Sec. VI-B, VI-C) at
their full sizes - two order-648 models in the iris guide, one order-1920
model of the copper rods - against the oracle on the same model inputs:
FP64 <= 1e-12 and FP32 <= 1e-5 relative L2 on the probe series; final
fields FP64 <= 1e-12 relative, FP32 <= 1e-5 of the field's peak norm over
the run (the layers leave a late snapshot far below the peak).  The open
guides also run together in one batch, bit-identical to single runs."""
import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from paper_1609_07114_amd.batch import Batch
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu

NSTEPS = {"E3": 2000, "E4": 1500}


@pytest.fixture(scope="module")
def cases():
    out = {}
    for name, mk in (("E3", W.iris_waveguide), ("E4", W.rods_reflection)):
        print(f"[gpu-wg] oracle models for {name}", flush=True)
        p = mk(nsteps=NSTEPS[name])
        out[name] = (p, osim.build_roms(p))
    return out


def _oracle(prob, roms, fp32):
    run = osim.CoupledRun(prob, roms, mode="closed", fp32=fp32)
    pr = np.empty((prob.nsteps, len(prob.probes)))
    peak = np.zeros(3)
    for n in range(prob.nsteps):
        run.step()
        pr[n] = run.probes()
        for c, f in enumerate((run.f.hz, run.f.ex, run.f.ey)):
            peak[c] = max(peak[c], np.linalg.norm(f))
    return pr, [run.f.hz * run.cell, run.f.ex, run.f.ey], peak


def _gpu(prob, roms, dtype):
    print(f"[gpu-wg] {prob.name} {prob.nx}x{prob.ny} {dtype} q={[s.q for s in prob.roms]}", flush=True)
    with Simulation(prob, roms, dtype=dtype) as s:
        s.run(prob.nsteps)
        return s.probes(), [s.field(c) for c in range(3)]


@pytest.mark.parametrize("name", ["E3", "E4"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_open_guides_vs_oracle(cases, name, dtype, tol):
    p, roms = cases[name]
    g = _gpu(p, roms, dtype)
    o = _oracle(p, roms, dtype == "f32")
    assert rel_l2(g[0], o[0]) <= tol, rel_l2(g[0], o[0])
    for c in range(3):
        err = np.linalg.norm(np.asarray(g[1][c], np.float64) - o[1][c])
        den = np.linalg.norm(o[1][c]) if dtype == "f64" else o[2][c]
        assert err <= tol * den, (c, err / den)


def test_open_guides_in_one_batch(cases):
    (p3, m3), (p4, m4) = cases["E3"], cases["E4"]
    empty = W.iris_waveguide(nsteps=NSTEPS["E3"], irises=False)
    me = osim.build_roms(empty)
    probs, models = [p3, p4, empty], [m3, m4, me]
    n = 600
    with Batch(probs, models, dtype="f32") as bt:
        bt.run(n)
        got = [bt.probes(k) for k in range(3)]
    for k, (p, m) in enumerate(zip(probs, models)):
        with Simulation(p, m, dtype="f32") as s:
            s.run(n)
            assert np.array_equal(got[k], s.probes()), k
