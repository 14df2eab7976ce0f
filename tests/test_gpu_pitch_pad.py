"""Row padding of the device layout (fdtd_grid.pitch_pad) through the C
ABI: the stencil, the coupling, the two-step pairs, the batch and the
reverse sweep read and write the same samples whatever the pitch, so padded
and unpadded handles give the same probes, fields, energy and gradients
bit for bit."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from paper_1609_07114_amd.sim import Simulation

pytestmark = pytest.mark.gpu


def _padded(p, pad):
    q = copy.copy(p)
    q.pitch_pad = pad
    return q


def _run(p, roms, nsteps, graph=0):
    print(f"[gpu-pitch] {p.name} {p.nx}x{p.ny} {p.dtype} pad={p.pitch_pad} steps={nsteps}", flush=True)
    with Simulation(p, roms, max_steps=nsteps) as s:
        s.set_graph(graph)
        s.run(nsteps)
        return s.probes(), [s.field(c) for c in range(3)], s.energy()


def _same(a, b):
    assert np.array_equal(a[0], b[0]), np.abs(a[0] - b[0]).max()
    for c in range(3):
        assert np.array_equal(a[1][c], b[1][c]), c
    assert a[2] == b[2]


@pytest.mark.parametrize("pad", [64, 1024])
def test_shared_model_pairs_fp32(pad):
    """Copies of one model (MFMA GEMM over the copies), two steps per pass,
    graph batches, a width that is not a multiple of 64."""
    p = W.many_copies(n=700, nsteps=120, q=40, spacing=96, block=8)
    roms = osim.build_roms(p)
    _same(_run(_padded(p, pad), roms, 117, graph=20), _run(p, roms, 117, graph=20))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_random_medium_with_models(dtype):
    """Per-cell material through the 16-bit table, models of several orders."""
    p = W.random_problem(61, 203, 150, 90, nroms=3, block=(5, 4), r=2, q=10, dtype=dtype)
    roms = osim.build_roms(p)
    _same(_run(_padded(p, 128), roms, 90), _run(p, roms, 90))


def test_layers_and_adjoint():
    """Absorbing layers (one launch per step) and the reverse sweep."""
    p = W.random_problem(62, 150, 100, 200, nroms=2, block=(5, 4), r=2, q=10, dt_frac_coarse=0.9, f_bw=3e9)
    lim = [8, 8, 6, 6]   # layers two cells clear of every region and its ring
    for s in p.roms:
        lim = [min(lim[0], s.i0 - 2), min(lim[1], p.nx - s.i0 - s.ni - 2),
               min(lim[2], s.j0 - 2), min(lim[3], p.ny - s.j0 - s.nj - 2)]
    p.pml = W.Pml(*[max(0, v) for v in lim])
    assert p.pml.any
    roms = osim.build_roms(p)
    _same(_run(_padded(p, 64), roms, 150), _run(p, roms, 150))
    out = []
    for q in (p, _padded(p, 64)):
        with Simulation(q, roms, max_steps=q.nsteps) as s:
            out.append(s.adjoint(q.nsteps, ckpt_every=30))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
