"""Material table of the coarse stencil (16-bit index per cell into the
problem's distinct (eps0 eps_r/dt, sigma/2) pairs) against the per-cell
arrays, through the C ABI: the same bit patterns reach eq. (3), so both
modes give bit-identical probes and fields - single problems in FP32 and
FP64, with models, absorbing layers, every tiling, and batches; problems
with more distinct pairs than the table holds fall back to the arrays."""
import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from paper_1609_07114_amd import capi
from paper_1609_07114_amd.batch import Batch
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu


def _run(prob, roms, mode=None, seg=None, dtype=None):
    print(f"[gpu-mat] {prob.name} {prob.nx}x{prob.ny} mode={mode} seg={seg} dtype={dtype or prob.dtype}", flush=True)
    with Simulation(prob, roms, dtype=dtype) as s:
        m, n = s.material_mode()
        if mode is not None:
            s.set_material_mode(mode)
        if seg:
            s.set_tiling(seg)
        s.run(prob.nsteps)
        return (m, n), s.probes(), [s.field(c) for c in range(3)]


def _same(a, b):
    assert np.array_equal(a[1], b[1])
    for c in range(3):
        assert np.array_equal(a[2][c], b[2][c]), c


@pytest.fixture(scope="module")
def patched():
    """Random media in 32x32 patches with two models: few distinct pairs."""
    p = W.random_media(n=256, nsteps=300, block=8, spacing=128, offset=60, qs=(12, 16), r=2, dtype="f32")
    return p, osim.build_roms(p)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_table_default_and_identical_to_arrays(patched, dtype):
    p, roms = patched
    idx = _run(p, roms, dtype=dtype)
    (mode, n) = idx[0]
    assert mode == 1 and 2 <= n <= 64 + 3, (mode, n)
    arr = _run(p, roms, mode=0, dtype=dtype)
    _same(idx, arr)


@pytest.mark.parametrize("seg", [4, 8, 16, 32])
def test_table_every_tiling(patched, seg):
    p, roms = patched
    _same(_run(p, roms, mode=1, seg=seg), _run(p, roms, mode=0, seg=seg))


def test_table_with_layers_and_oracle():
    p = W.iris_waveguide(nsteps=600)
    roms = osim.build_roms(p)
    a = _run(p, roms, dtype="f32")
    assert a[0][0] == 1
    _same(a, _run(p, roms, mode=0, dtype="f32"))
    o = osim.CoupledRun(p, roms, mode="closed", fp32=True)
    pr = np.empty((p.nsteps, len(p.probes)))
    for n in range(p.nsteps):
        o.step()
        pr[n] = o.probes()
    assert rel_l2(a[1], pr) <= 1e-5


def test_too_many_materials_fall_back():
    """A per-cell random map of 300 x 300 cells has ~90,000 distinct pairs."""
    p = W.random_problem(11, 300, 300, 50, nroms=1, block=(5, 4), r=2, q=10, dtype="f32")
    roms = osim.build_roms(p)
    with Simulation(p, roms) as s:
        assert s.material_mode() == (0, 0)
        with pytest.raises(capi.FdtdError):
            s.set_material_mode(1)
        s.run(p.nsteps)
        assert np.all(np.isfinite(s.probes()))


def test_batch_table_and_mixed(patched):
    """All instances with tables run the table variant; one instance
    without a table makes the batch read the arrays; both match single runs."""
    p, roms = patched
    q = W.iris_waveguide(nsteps=300)
    mq = osim.build_roms(q)
    big = W.random_problem(12, 300, 290, 300, nroms=1, block=(5, 4), r=2, q=10, dtype="f32")
    mb = osim.build_roms(big)
    for probs, models in (([p, q], [roms, mq]), ([p, big, q], [roms, mb, mq])):
        with Batch(probs, models, dtype="f32") as bt:
            bt.run(300)
            got = [bt.probes(k) for k in range(len(probs))]
        for k, (pp, mm) in enumerate(zip(probs, models)):
            ref = _run(pp, mm, dtype="f32")
            assert np.array_equal(got[k], ref[1]), (len(probs), k)
