"""The run call's periodic finiteness check (FDTD_EUNSTABLE), the
prepare-run call and the library's probe objective, through the C ABI.

A NaN is planted in a source increment (an input) - the kernels only ever
compute with it; nothing faults.  The check only reads the field set, so
runs with and without it are bit-identical."""
import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from paper_1609_07114_amd import capi
from paper_1609_07114_amd.sim import Simulation

pytestmark = pytest.mark.gpu


def _nan_source(p, at):
    s = p.sources[0]
    s.incr = s.incr.copy()
    s.incr[at] = np.nan
    return p


def _run(p, roms, nsteps, check=None, graph=0, tb=None, chunks=None):
    print(f"[gpu] {p.name} steps={nsteps} check={check} graph={graph} tb={tb}", flush=True)
    with Simulation(p, roms, max_steps=nsteps) as s:
        if check is not None:
            s.set_check_interval(check)
        if tb is not None:
            s.set_time_blocking(tb)
        s.set_graph(graph)
        for c in chunks or [nsteps]:
            s.run(c)
        return s.probes(), s.field(0)


@pytest.mark.parametrize("graph", [0, 16])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_nan_source_reported_as_unstable(graph, dtype):
    p = W.random_problem(5, 90, 70, 200, nroms=1, block=(5, 4), r=2, q=10, dtype=dtype)
    roms = osim.build_roms(p)
    _nan_source(p, 10)
    with Simulation(p, roms, max_steps=200) as s:
        s.set_check_interval(32)
        s.set_graph(graph)
        s.run(20)                       # no check due yet: asynchronous, no error
        with pytest.raises(capi.FdtdError) as e:
            s.run(40)                   # crosses step 32
        assert e.value.status == capi.FDTD_EUNSTABLE
        assert s.steps_done == 60       # the steps were taken
        with pytest.raises(capi.FdtdError) as e:
            s.run(40)                   # the flag stays raised
        assert e.value.status == capi.FDTD_EUNSTABLE


def test_default_interval_catches_nan():
    p = W.random_problem(6, 64, 40, 1100, nroms=0)
    _nan_source(p, 3)
    with Simulation(p, [], max_steps=1100) as s:
        assert s.check_interval() == 1024
        s.run(1000)
        with pytest.raises(capi.FdtdError) as e:
            s.run(100)
        assert e.value.status == capi.FDTD_EUNSTABLE


def test_set_state_clears_the_flag():
    p = W.random_problem(7, 70, 50, 300, nroms=1, block=(5, 4), r=2, q=10)
    roms = osim.build_roms(p)
    clean = W.random_problem(7, 70, 50, 300, nroms=1, block=(5, 4), r=2, q=10)
    _nan_source(p, 50)
    with Simulation(clean, roms, max_steps=300) as c:
        c.run(40)
        blob = c.get_state()
    with Simulation(p, roms, max_steps=300) as s:
        s.set_check_interval(16)
        with pytest.raises(capi.FdtdError):
            s.run(100)
        s.set_state(blob)               # back to the clean step-40 state
        s.set_check_interval(8)
        s.run(8)                        # checked, before the NaN's step: fine
        assert s.steps_done == 48


@pytest.mark.parametrize("check", [7, 1, 0])
@pytest.mark.parametrize("tb", [1, 0])
def test_checks_do_not_change_results(check, tb):
    """Chunking the direct launches at the check points (odd intervals
    included, which two-step runs round to whole pairs) and the check
    kernels themselves leave the results bit-identical."""
    p = W.random_problem(8, 130, 77, 150, nroms=2, block=(5, 4), r=2, q=12, dtype="f32")
    roms = osim.build_roms(p)
    ref_p, ref_h = _run(p, roms, 150, check=0, tb=tb)
    got_p, got_h = _run(p, roms, 150, check=check, tb=tb, chunks=[1, 13, 60, 76])
    assert np.array_equal(got_p, ref_p)
    assert np.array_equal(got_h, ref_h)
    g_p, g_h = _run(p, roms, 150, check=check, tb=tb, graph=12)
    assert np.array_equal(g_p, ref_p)
    assert np.array_equal(g_h, ref_h)


def test_prepare_run_then_run_matches():
    p = W.random_problem(9, 100, 60, 140, nroms=2, block=(5, 4), r=2, q=12)
    roms = osim.build_roms(p)
    ref_p, ref_h = _run(p, roms, 140, graph=20)
    with Simulation(p, roms, max_steps=140) as s:
        s.set_graph(20)
        s.run(5)                        # odd start: the graph key follows the parity
        s.prepare_run(120)
        s.run(120)
        s.prepare_run(15)               # shorter than a batch: nothing to capture
        s.run(15)
        assert np.array_equal(s.probes(), ref_p)
        assert np.array_equal(s.field(0), ref_h)


def test_probe_objective_from_library():
    p = W.random_problem(10, 60, 50, 200, nroms=1, block=(5, 4), r=2, q=10)
    roms = osim.build_roms(p)
    hz = [k for k, pr in enumerate(p.probes) if pr.comp == W.HZ]
    assert hz
    with Simulation(p, roms, max_steps=200) as s:
        s.run(200)
        pr = s.probes()
        for k in hz:
            J = s.objective(k, 0, 200)
            assert abs(J - p.dt * np.sum(pr[:, k] ** 2)) <= 1e-12 * abs(J)
            J2 = s.objective(k, 50, 100)
            assert abs(J2 - p.dt * np.sum(pr[50:150, k] ** 2)) <= 1e-12 * abs(J2)
        nonhz = [k for k, q in enumerate(p.probes) if q.comp != W.HZ]
        for k in nonhz:
            with pytest.raises(capi.FdtdError):
                s.objective(k, 0, 10)
        with pytest.raises(capi.FdtdError):
            s.objective(hz[0], 150, 100)     # rows beyond the steps taken
