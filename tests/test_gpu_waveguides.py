"""The paper's open-waveguide workloads on the device (Sec. VI-B, VI-C) at
their full sizes - two order-648 models of the regions around the PEC
irises, one order-1920 model of the copper rods - against the oracle on the
same model inputs.

FP32: <= 1e-5 relative L2 on the probe series; the fields <= 1e-5
relative L2 (their own norm) at a step while the pulse is inside the guide,
and at the end of the run <= 1e-5 of the field's peak norm over the run
(the layers leave the last snapshot some 1e-6 of the peak, a residue whose
own-norm error measures nothing); the FP64 fields are checked the same way.

FP64: the iris guide at 1e-12 on probes and fields (the irises are PEC
cells, so the eq. (23) matrices stay well conditioned).  The rods are
copper, 5.8e7 S/m, which makes eq. (23)'s matrix M = R~ + F~ + L~ C+ L~^T
ill-conditioned (cond 3.8e6), so two backward-stable FP64 solves of it agree
only to about cond x eps; for them the bar is taken from the oracle itself:
its run with the LU route is compared with its run with the QR route (same
definition, different rounding), and for the probes and each field the
device must stay within 10x that spread or 1e-12, whichever is larger.

The open guides also run together in one batch, bit-identical to single
runs."""
import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from paper_1609_07114_amd.batch import Batch
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu

NSTEPS = {"E3": 2000, "E4": 1500}
# a step with the pulse inside the guide (fields compared on their own norm)
MID = {"E3": 200, "E4": 150}
# guides whose eq. (23) matrix is ill-conditioned (copper at 5.8e7 S/m)
ILL_CONDITIONED = {"E4"}


@pytest.fixture(scope="module")
def cases():
    out = {}
    for name, mk in (("E3", W.iris_waveguide), ("E4", W.rods_reflection)):
        print(f"[gpu-wg] oracle models for {name}", flush=True)
        p = mk(nsteps=NSTEPS[name])
        out[name] = (p, osim.build_roms(p))
    return out


def _oracle(prob, roms, fp32, solver="lu", mid=None):
    run = osim.CoupledRun(prob, roms, mode="closed", fp32=fp32, solver=solver)
    pr = np.empty((prob.nsteps, len(prob.probes)))
    peak = np.zeros(3)
    at_mid = None
    for n in range(prob.nsteps):
        run.step()
        pr[n] = run.probes()
        for c, f in enumerate((run.f.hz, run.f.ex, run.f.ey)):
            peak[c] = max(peak[c], np.linalg.norm(f))
        if n + 1 == mid:
            at_mid = [run.f.hz * run.cell, run.f.ex.copy(), run.f.ey.copy()]
    return pr, [run.f.hz * run.cell, run.f.ex, run.f.ey], peak, at_mid


def _gpu(prob, roms, dtype, mid=None):
    print(f"[gpu-wg] {prob.name} {prob.nx}x{prob.ny} {dtype} q={[s.q for s in prob.roms]}", flush=True)
    with Simulation(prob, roms, dtype=dtype) as s:
        at_mid = None
        if mid:
            s.run(mid)
            at_mid = [s.field(c) for c in range(3)]
        s.run(prob.nsteps - (mid or 0))
        return s.probes(), [s.field(c) for c in range(3)], at_mid


@pytest.mark.parametrize("name", ["E3", "E4"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_open_guides_vs_oracle(cases, name, dtype, tol):
    p, roms = cases[name]
    mid = MID[name]
    g = _gpu(p, roms, dtype, mid)
    o = _oracle(p, roms, dtype == "f32", mid=mid)

    def errors(a):
        """Probe series relative L2; each final field relative to its peak
        norm over the run; each field at the middle step relative L2."""
        return ([rel_l2(a[0], o[0])]
                + [np.linalg.norm(np.asarray(a[1][c], np.float64) - o[1][c]) / max(o[2][c], 1e-300)
                   for c in range(3)]
                + [rel_l2(a[3 if len(a) == 4 else 2][c], o[3][c]) for c in range(3)])

    names = ("probes", "hz end", "ex end", "ey end", "hz mid", "ex mid", "ey mid")
    bars = [tol] * len(names)
    if dtype == "f64" and name in ILL_CONDITIONED:
        spread = errors(_oracle(p, roms, False, solver="qr", mid=mid))
        print(f"[gpu-wg] {name} FP64 oracle LU vs QR spread {['%.2e' % v for v in spread]}", flush=True)
        bars = [max(tol, 10.0 * v) for v in spread]
    got = errors(g)
    print(f"[gpu-wg] {name} {dtype} errors {['%.2e' % v for v in got]}", flush=True)
    for c in range(3):   # the pulse is in the guide at the middle step
        assert np.linalg.norm(o[3][c]) > 1e-3 * o[2][c], c
    for what, e, b in zip(names, got, bars):
        assert e <= b, (what, e, b)


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
