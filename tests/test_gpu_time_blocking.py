"""Two steps per pass (fdtd_rom_set_time_blocking) against single-step
launches, through the C ABI.  The per-cell arithmetic is the same, so the
probe records, final fields, reduced states and energies must be
identical (np.array_equal) - across tilings, ragged grids, odd step counts,
graph batches, models near tile edges, every probe component, sources
inside far tiles, checkpoint/resume and the adjoint's forward; FP64 also
against the oracle at the forward bar."""
import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from paper_1609_07114_amd import capi
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu


def _run(prob, roms, tb, nsteps, seg=None, graph=0, dtype=None):
    print(f"[gpu-tb] {prob.name} {prob.nx}x{prob.ny} {dtype or prob.dtype} tb={tb} seg={seg} "
          f"graph={graph} steps={nsteps}", flush=True)
    with Simulation(prob, roms, max_steps=nsteps, dtype=dtype) as s:
        if seg:
            s.set_tiling(seg)
        s.set_graph(graph)
        s.set_time_blocking(tb)
        assert s.time_blocking() == tb
        s.run(nsteps)
        return s.probes(), [s.field(c) for c in range(3)], s.energy(), s.get_state()


def _same(a, b):
    assert np.array_equal(a[0], b[0]), np.abs(a[0] - b[0]).max()
    for c in range(3):
        assert np.array_equal(a[1][c], b[1][c]), (c, np.abs(a[1][c] - b[1][c]).max())
    assert a[2] == b[2]


def _with_all_probes(p, seed):
    """Probes of every component on a scatter of coarse samples (most in far
    tiles) and on the ring of port cells around each region (near tiles)."""
    rng = np.random.default_rng(seed)

    def held(i, j):
        return any(s.i0 - 1 <= i <= s.i0 + s.ni and s.j0 - 1 <= j <= s.j0 + s.nj for s in p.roms)
    probes = []
    while len(probes) < 24:
        i = int(rng.integers(1, p.nx - 1))
        j = int(rng.integers(1, p.ny - 1))
        if not held(i, j):
            probes.append(W.Probe(len(probes) % 3, i, j))
    for s in p.roms:
        probes += [W.Probe(W.HZ, s.i0 - 1, s.j0), W.Probe(W.EX, s.i0 - 1, s.j0),
                   W.Probe(W.EY, s.i0 - 1, s.j0 + 1), W.Probe(W.EY, s.i0 + s.ni + 1, s.j0),
                   W.Probe(W.HZ, s.i0 + s.ni, s.j0 + s.nj), W.Probe(W.EX, s.i0 + 2, s.j0 + s.nj + 1)]
    p.probes = probes
    return p


@pytest.fixture(scope="module")
def mixed():
    """Ragged grid (not a multiple of 62 or 64 columns), three models at
    random places, sources and every probe component."""
    p = W.random_problem(71, 203, 150, 121, nroms=3, block=(5, 4), r=2, q=12,
                         dt_frac_coarse=0.9, f_bw=3e9)
    p = _with_all_probes(p, 3)
    return p, osim.build_roms(p)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("seg", [4, 8, 16, 32])
def test_two_step_equals_single_step_every_tiling(mixed, dtype, seg):
    p, roms = mixed
    ref = _run(p, roms, False, p.nsteps, seg=seg, dtype=dtype)
    got = _run(p, roms, True, p.nsteps, seg=seg, dtype=dtype)
    _same(got, ref)


@pytest.mark.parametrize("graph", [2, 6, 64])
def test_two_step_with_graph_batches(mixed, graph):
    """Graph batches rounded to a multiple of 4 steps, an odd run length,
    and runs split into pieces of uneven length."""
    p, roms = mixed
    ref = _run(p, roms, False, p.nsteps, dtype="f32")
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f32") as s:
        s.set_graph(graph)
        s.set_time_blocking(True)
        for piece in (7, 64, 1, 30, 19):
            s.run(piece)
        got = (s.probes(), [s.field(c) for c in range(3)], s.energy())
    _same(got, ref[:3])


def test_two_step_fp64_vs_oracle(mixed):
    p, roms = mixed
    got = _run(p, roms, True, p.nsteps, dtype="f64")
    run = osim.CoupledRun(p, roms, mode="closed")
    pr = np.empty((p.nsteps, len(p.probes)))
    for n in range(p.nsteps):
        run.step()
        pr[n] = run.probes()
    assert rel_l2(got[0], pr) <= 1e-12, rel_l2(got[0], pr)
    for c, f in enumerate((run.f.hz * run.cell, run.f.ex, run.f.ey)):
        assert rel_l2(np.asarray(got[1][c], np.float64), f) <= 1e-12, c


def test_many_models_and_wide_grid():
    """Nine models on a 3x3 lattice of a 400x300 grid, FP32 material table."""
    p = W.random_problem(72, 400, 300, 60, nroms=9, block=(6, 5), r=2, q=10,
                         dtype="f32", dt_frac_coarse=0.9, f_bw=3e9)
    p = _with_all_probes(p, 4)
    roms = osim.build_roms(p)
    _same(_run(p, roms, True, 60), _run(p, roms, False, 60))


def test_no_models_no_probes_near_walls():
    p = W.random_problem(73, 130, 41, 50, nroms=0, dt_frac_coarse=0.9, f_bw=3e9)
    p.probes = [W.Probe(W.HZ, 0, 0), W.Probe(W.EX, 129, 40), W.Probe(W.EY, 129, 1), W.Probe(W.EX, 61, 1),
                W.Probe(W.EY, 62, 39)]
    _same(_run(p, [], True, 50), _run(p, [], False, 50))


def test_c2_full_size_sample():
    """The 2048^2 random-media workload (16 models, 64 probes), FP32, 120
    steps with graphs: the two-step run equals the single-step run."""
    from paper_1609_07114_amd import romgen
    p = W.random_media(nsteps=120)
    roms = romgen.build_roms(p)
    a = _run(p, roms, True, 120, graph=64)
    b = _run(p, roms, False, 120, graph=64)
    _same(a, b)


def test_resume_across_modes(mixed):
    """A state taken mid-run under two-step launches (sets traded places)
    restores into a single-step handle and continues identically."""
    p, roms = mixed
    ref = _run(p, roms, False, p.nsteps, dtype="f32")
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f32") as s:
        s.set_time_blocking(True)
        s.run(42)                      # 21 pairs: sets swapped
        st = s.get_state()
        first = s.probes(0, 42)
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f32") as s2:
        s2.set_state(st)
        s2.run(p.nsteps - 42)
        rest = s2.probes(42, p.nsteps - 42)
        assert np.array_equal(np.vstack([first, rest]), ref[0])
        for c in range(3):
            assert np.array_equal(s2.field(c), ref[1][c])


def test_adjoint_forward_under_two_steps(mixed):
    p, roms = mixed
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f64") as s:
        a = s.adjoint(p.nsteps)
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f64") as s:
        s.set_time_blocking(True)
        b = s.adjoint(p.nsteps)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_layers_refuse_two_steps():
    p = W.random_problem(74, 60, 50, 20, nroms=0, dt_frac_coarse=0.9)
    p.pml = W.Pml(5, 5, 5, 5)
    with Simulation(p, [], max_steps=20) as s:
        with pytest.raises(capi.FdtdError):
            s.set_time_blocking(True)
        assert not s.time_blocking()


def _batch_run(probs, models, tb, pieces, graph=0, seg=None, split=None):
    from paper_1609_07114_amd.batch import Batch
    with Batch(probs, models, dtype="f32") as bt:
        if seg:
            bt.set_tiling(-1, seg)
        if split is not None:
            bt.set_pair_split(-1, split)
        bt.set_graph(graph)
        bt.set_time_blocking(tb)
        assert bt.time_blocking() == tb
        for k in pieces:
            bt.run(k)
        return [bt.probes(b) for b in range(len(probs))], [[bt.field(b, c) for c in range(3)] for b in range(len(probs))]


@pytest.fixture(scope="module")
def mix():
    probs = [W.random_problem(81 + k, nx, ny, 130, nroms=nr, block=(5, 4), r=2, q=10, dtype="f32",
                              dt_frac_coarse=0.9, f_bw=3e9)
             for k, (nx, ny, nr) in enumerate([(203, 150, 3), (64, 300, 1), (130, 41, 0), (250, 250, 4)])]
    probs = [_with_all_probes(p, 5 + k) for k, p in enumerate(probs)]
    return probs, [osim.build_roms(p) for p in probs]


@pytest.mark.parametrize("graph,seg,split", [(0, None, None), (8, None, 50), (64, 4, 25), (0, 32, 90)])
def test_batch_two_step_equals_single_step(mix, graph, seg, split):
    """Four uneven instances in one batch, pairs and odd pieces, graph
    batches, every tiling, far tiles shared with the second launch: two
    steps per pass equals one launch per step, and each instance equals its
    own handle."""
    probs, models = mix
    pieces = (3, 64, 1, 40, 22)
    a = _batch_run(probs, models, True, pieces, graph, seg, split)
    b = _batch_run(probs, models, False, pieces, graph, seg)
    for k in range(len(probs)):
        assert np.array_equal(a[0][k], b[0][k]), k
        for c in range(3):
            assert np.array_equal(a[1][k][c], b[1][k][c]), (k, c)
    for k, p in enumerate(probs):
        ref = _run(p, models[k], False, sum(pieces), dtype="f32")
        assert np.array_equal(a[0][k], ref[0]), k


def test_batch_with_layers_steps_singly():
    from paper_1609_07114_amd.batch import Batch
    p = W.random_problem(90, 60, 50, 20, nroms=0, dtype="f32", dt_frac_coarse=0.9)
    q = W.random_problem(91, 60, 50, 20, nroms=0, dtype="f32", dt_frac_coarse=0.9)
    q.pml = W.Pml(5, 5, 5, 5)
    with Batch([p, q], [[], []]) as bt:
        assert not bt.time_blocking()
        with pytest.raises(capi.FdtdError):
            bt.set_time_blocking(True)


def test_profile_counts_pairs_as_units(mixed):
    """With two steps per pass the profiling events bracket each pair: 11
    steps are 5 pairs and one single launch."""
    p, roms = mixed
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f32") as s:
        s.profile(True)
        s.run(11)
        ms, units, tail_ms, tails = s.profile_read()
        assert units == 6 and tails == 1 and ms > 0
        s.set_time_blocking(False)
        s.run(4)
        ms, units, _, _ = s.profile_read()
        assert units == 4


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_step_per_cell_material(mixed, dtype):
    """Material mode 0 (per-cell arrays instead of the 16-bit table): the
    two-step kernels' other material path, against one launch per step."""
    p, roms = mixed
    out = []
    for tb in (True, False):
        with Simulation(p, roms, max_steps=p.nsteps, dtype=dtype) as s:
            s.set_material_mode(0)
            s.set_time_blocking(tb)
            s.run(p.nsteps)
            out.append((s.probes(), [s.field(c) for c in range(3)], s.energy()))
    _same(out[0], out[1])


def test_batch_two_step_without_material_tables():
    """A batch with an instance of more than 65,536 distinct materials runs
    the per-cell material variant of the batched pair."""
    probs = [W.random_problem(95, 300, 260, 60, nroms=2, block=(5, 4), r=2, q=10, dtype="f32",
                              dt_frac_coarse=0.9, f_bw=3e9),
             W.random_problem(96, 90, 70, 60, nroms=1, block=(5, 4), r=2, q=10, dtype="f32",
                              dt_frac_coarse=0.9, f_bw=3e9)]
    models = [osim.build_roms(p) for p in probs]
    with Simulation(probs[0], models[0], dtype="f32") as s:
        assert s.material_mode() == (0, 0)   # no table for this instance
    a = _batch_run(probs, models, True, (7, 53))
    b = _batch_run(probs, models, False, (7, 53))
    for k in range(2):
        assert np.array_equal(a[0][k], b[0][k]), k
        for c in range(3):
            assert np.array_equal(a[1][k][c], b[1][k][c]), (k, c)


def test_switching_modes_mid_run(mixed):
    """Two-step launches switched off after an odd number of pairs (the
    field sets have traded places) and on again: the run continues exactly
    as one launch per step throughout."""
    p, roms = mixed
    ref = _run(p, roms, False, p.nsteps, dtype="f32")
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f32") as s:
        s.set_graph(8)
        s.run(10)                      # 5 pairs
        s.set_time_blocking(False)
        s.run(11)
        s.set_time_blocking(True)
        s.run(p.nsteps - 21)
        got = (s.probes(), [s.field(c) for c in range(3)], s.energy())
    _same(got, ref[:3])


def test_restore_into_handle_with_traded_sets(mixed):
    """A state restored into a handle whose own field sets have traded
    places (an odd number of pairs run before) continues identically."""
    p, roms = mixed
    ref = _run(p, roms, False, p.nsteps, dtype="f32")
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f32") as s:
        s.run(42)
        st = s.get_state()
    with Simulation(p, roms, max_steps=p.nsteps, dtype="f32") as s2:
        s2.run(6)                      # 3 pairs: this handle's sets have traded places
        s2.set_state(st)
        s2.run(p.nsteps - 42)
        assert np.array_equal(s2.probes(42, p.nsteps - 42), ref[0][42:])
        for c in range(3):
            assert np.array_equal(s2.field(c), ref[1][c])


@pytest.mark.parametrize("split", [0, 30, 90])
def test_far_tiles_in_second_launch_bit_identical(split):
    """Far tiles moved into the second launch of each pair (any share) give
    the same bits as one launch per step, with regions, sources and graphs."""
    p = W.random_problem(91, 300, 170, 120, nroms=3, block=(5, 4), r=2, q=12, dtype="f32")
    roms = osim.build_roms(p)
    with Simulation(p, roms, max_steps=120) as s:
        s.set_time_blocking(False)
        s.run(120)
        ref = (s.probes(), s.field(0), s.field(1), s.field(2))
    with Simulation(p, roms, max_steps=120) as s:
        s.set_pair_split(split)
        s.set_graph(24)
        s.run(50)
        s.run(70)
        assert s.pair_split() == pytest.approx(split, abs=1)
        got = (s.probes(), s.field(0), s.field(1), s.field(2))
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
