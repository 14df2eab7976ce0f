"""Energy diagnostic (fdtd_rom_energy) against the oracle's storage function
and Theorem 2's monotonicity, and checkpoint / resume (state get / set),
through the C ABI.  Energy bars: FP64 <= 1e-10 relative (a sum of squares
minus the E^T K Hz cross term), FP32 <= 1e-5 against the oracle's FP32
coefficient mode."""
import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from paper_1609_07114_amd import capi
from paper_1609_07114_amd.sim import Simulation

pytestmark = pytest.mark.gpu


def _energies(prob, roms, checkpoints, dtype, x0=None):
    out = []
    with Simulation(prob, roms, dtype=dtype, x0=x0) as s:
        done = 0
        for n in checkpoints:
            s.run(n - done)
            done = n
            out.append(s.energy())
    return np.array(out)


def _oracle_energies(prob, roms, checkpoints, fp32, init=None):
    run = osim.CoupledRun(prob, roms, mode="closed", fp32=fp32, init=init)
    out, done = [], 0
    for n in checkpoints:
        for _ in range(n - done):
            run.step()
        done = n
        out.append(run.energy())
    return np.array(out)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
@pytest.mark.parametrize("lossy", [True, False])
def test_energy_matches_oracle(dtype, tol, lossy):
    p = W.random_problem(21, 70, 45, 400, nroms=2, block=(5, 4), r=2, q=12, lossy=lossy,
                         dt_frac_coarse=0.9)
    roms = osim.build_roms(p)
    cps = [1, 50, 150, 400]
    g = _energies(p, roms, cps, dtype)
    o = _oracle_energies(p, roms, cps, fp32=(dtype == "f32"))
    assert np.all(o > 0)
    assert np.all(np.abs(g - o) <= tol * np.abs(o)), (g, o)


def test_energy_constant_then_decaying_after_source():
    """Theorem 2 on the device: once the pulse has been injected, the
    energy stays constant without loss and does not increase with loss."""
    for lossy in (False, True):
        p = W.random_problem(22, 60, 50, 900, nroms=2, block=(5, 4), r=2, q=12, lossy=lossy,
                             dt_frac_coarse=0.9)
        n_src = int(np.max(np.nonzero(np.abs(p.sources[0].incr) > 1e-30 * np.abs(p.sources[0].incr).max())))
        cps = list(range(n_src + 2, 900, 40))
        e = _energies(p, osim.build_roms(p), cps, "f64")
        if lossy:
            assert np.all(np.diff(e) <= 1e-12 * e[0]), np.diff(e) / e[0]
            assert e[-1] < e[0]
        else:
            assert np.max(np.abs(e - e[0])) <= 1e-9 * e[0], (e - e[0]) / e[0]


def test_energy_of_initial_reduced_state():
    """A random initial reduced state, no source: energy at step 0 equals the
    oracle's (x0^T R~ x0 plus the interface E = L~^T x0 terms) and decays."""
    p = W.random_problem(9, 40, 36, 200, nroms=2, block=(5, 4), r=2, q=12)
    for s in p.sources:
        s.incr[:] = 0
    roms = osim.build_roms(p)
    rng = np.random.default_rng(3)
    x0 = [rng.standard_normal(m["Rt"].shape[0]) for m in roms]
    init = dict(hz=np.zeros((p.ny, p.nx)), ex=np.zeros((p.ny + 1, p.nx)),
                ey=np.zeros((p.ny, p.nx + 1)), x=x0)
    cps = [0, 10, 100, 200]
    g = _energies(p, roms, cps, "f64", x0=x0)
    o = _oracle_energies(p, roms, cps, fp32=False, init=init)
    assert np.all(np.abs(g - o) <= 1e-10 * np.abs(o)), (g, o)
    assert np.all(np.diff(g) <= 1e-12 * g[0])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_checkpoint_resume_is_exact(dtype):
    p = W.random_problem(23, 70, 45, 300, nroms=2, block=(5, 4), r=2, q=12)
    roms = osim.build_roms(p)
    with Simulation(p, roms, dtype=dtype) as s:
        s.run(100)
        st = s.get_state()
        s.run(77)
        a = s.probes(100, 77)
        fa = [s.field(c) for c in range(3)]
        xa = [s.rom_state(k) for k in range(len(roms))]
        s.set_state(st)
        assert s.steps_done == 100
        s.run(77)
        assert np.array_equal(s.probes(100, 77), a)
        assert all(np.array_equal(s.field(c), fa[c]) for c in range(3))
    with Simulation(p, roms, dtype=dtype) as s2:      # resume in a fresh handle
        s2.set_state(st)
        s2.run(77)
        assert np.array_equal(s2.probes(100, 77), a)
        assert all(np.array_equal(s2.rom_state(k), xa[k]) for k in range(len(roms)))


def test_set_state_rejects_other_shapes():
    p = W.random_problem(23, 70, 45, 50, nroms=2, block=(5, 4), r=2, q=12)
    q = W.random_problem(24, 71, 45, 50, nroms=0)
    roms = osim.build_roms(p)
    with Simulation(p, roms) as s, Simulation(q, []) as t:
        st = s.get_state()
        with pytest.raises((capi.FdtdError, ValueError)):
            t.set_state(st)


def test_cavity_stable_for_a_million_steps():
    """Sec. VI-A reports the cavity with its embedded model stable over 10^6
    steps; Theorem 2 says why (every model passive at dt, dt within the
    coarse limit): the storage function never grows once the source has
    ended.  The device run of the cavity (library-built order-40 model,
    FP64) over 10^6 steps: the energy after the pulse, at 10^4, 10^5 and
    10^6 steps is non-increasing (to 1e-9 of its value: FP64 round-off over
    the run) and positive, and the probe series stays finite and within 10x
    its peak of the first 2000 steps (an instability grows without bound)."""
    from paper_1609_07114_amd import romgen
    n = 1_000_000
    p = W.cavity_c1(nsteps=n)
    roms = romgen.build_roms(p)
    marks = [2000, 10_000, 100_000, n]
    with Simulation(p, roms, max_steps=n) as s:
        s.set_graph(1000)
        e, done = [], 0
        for m in marks:
            s.run(m - done)
            done = m
            e.append(s.energy())
            print(f"[gpu-energy] step {m}: energy {e[-1]:.6e}", flush=True)
        pr = s.probes(0, n)[:, 0]
    e = np.array(e)
    assert np.all(np.isfinite(e)) and np.all(e > 0)
    assert np.all(e[1:] <= e[:-1] * (1 + 1e-9)), e
    assert np.all(np.isfinite(pr))
    assert np.abs(pr[2000:]).max() <= 10 * np.abs(pr[:2000]).max()
