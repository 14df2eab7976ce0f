"""Batched runs (fdtd_rom_batch_* through the C ABI): every instance
against its own single-problem handle (same device code on the same data:
bit-identical), against the CPU FP64 oracle (FP64 <= 1e-12, FP32 <= 1e-5
relative L2), across per-instance tile heights and graph batching, and the
autotuner's cache."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import sim as osim
from paper_1609_07114_amd import autotune, capi, romgen
from paper_1609_07114_amd.batch import Batch
from paper_1609_07114_amd.sim import Simulation
from tests._util import rel_l2

pytestmark = pytest.mark.gpu


def _single(prob, roms, nsteps, dtype):
    with Simulation(prob, roms, max_steps=nsteps, dtype=dtype) as s:
        s.run(nsteps)
        return s.probes(), [s.field(c) for c in range(3)]


def _oracle(prob, roms, nsteps, fp32):
    run = osim.CoupledRun(prob, roms, mode="closed", fp32=fp32)
    pr = np.empty((nsteps, len(prob.probes)))
    for n in range(nsteps):
        run.step()
        pr[n] = run.probes()
    return pr, [run.f.hz * run.cell, run.f.ex, run.f.ey]


def _mixed(dtype, nsteps=160):
    """Uneven grids (ragged widths), 0-2 models of different orders, lossy."""
    shapes = [(70, 45, 2, 12), (130, 77, 1, 10), (33, 20, 0, 0), (64, 64, 2, 8), (200, 9, 0, 0)]
    probs, roms = [], []
    for k, (nx, ny, nr, q) in enumerate(shapes):
        p = W.random_problem(40 + k, nx, ny, nsteps, nroms=nr, block=(5, 4), r=2, q=max(q, 2),
                             dtype=dtype)
        probs.append(p)
        roms.append(osim.build_roms(p))
    return probs, roms


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_equals_single_handles(dtype):
    probs, roms = _mixed(dtype)
    n = probs[0].nsteps
    print(f"[gpu-batch] mixed B={len(probs)} {dtype}", flush=True)
    with Batch(probs, roms, dtype=dtype) as bt:
        bt.run(n // 2)
        bt.run(n - n // 2)
        got = [(bt.probes(b), [bt.field(b, c) for c in range(3)]) for b in range(len(probs))]
    for b, (p, r) in enumerate(zip(probs, roms)):
        pr, fl = _single(p, r, n, dtype)
        assert np.array_equal(got[b][0], pr), b
        for c in range(3):
            assert np.array_equal(got[b][1][c], fl[c]), (b, c)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_batch_matches_oracle(dtype, tol):
    probs, roms = _mixed(dtype)
    n = probs[0].nsteps
    with Batch(probs, roms, dtype=dtype) as bt:
        bt.set_graph(32)
        bt.run(n)
        got = [(bt.probes(b), [bt.field(b, c) for c in range(3)]) for b in range(len(probs))]
    for b, (p, r) in enumerate(zip(probs, roms)):
        pr, fl = _oracle(p, r, n, fp32=(dtype == "f32"))
        assert rel_l2(got[b][0], pr) <= tol, (b, rel_l2(got[b][0], pr))
        for c in range(3):
            assert rel_l2(got[b][1][c], fl[c]) <= tol, (b, c)


def test_batch_tilings_and_graphs_identical():
    probs, roms = _mixed("f32")
    n = probs[0].nsteps
    ref = None
    for segs, graph in (([16] * 5, 0), ([8, 32, 16, 8, 32], 0), ([32, 8, 8, 32, 16], 40)):
        print(f"[gpu-batch] tiling {segs} graph={graph}", flush=True)
        with Batch(probs, roms) as bt:
            for b, s in enumerate(segs):
                bt.set_tiling(b, s)
            bt.set_graph(graph)
            for _ in range(4):
                bt.run(n // 4)
            out = [bt.probes(b) for b in range(len(probs))]
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                assert np.array_equal(a, b)


def test_batch_rejects_bad_input():
    probs, roms = _mixed("f32")
    probs[2].dtype = "f64"
    with pytest.raises(capi.FdtdError):
        Batch(probs, roms, dtype=None)
    probs, roms = _mixed("f32")
    with Batch(probs, roms) as bt:
        with pytest.raises(capi.FdtdError):
            bt.run(probs[0].nsteps + 1)
        with pytest.raises(capi.FdtdError):
            bt.set_tiling(7, 16)
        with pytest.raises(capi.FdtdError):
            bt.set_tiling(0, 12)


def test_autotuner_caches_choice(tmp_path):
    probs, roms = _mixed("f32", nsteps=200)
    path = str(tmp_path / "tune.json")
    seen = []
    choice = autotune.tune(probs, roms, path=path, trial_steps=8, log=seen.append)
    buckets = {autotune.bucket_of(p) for p in probs}
    assert set(choice) == buckets | {autotune.SPLIT}
    assert all(choice[b] in autotune.CANDIDATES for b in buckets)
    assert choice[autotune.SPLIT] in autotune.SPLITS
    assert len(seen) == len(autotune.CANDIDATES) * len(buckets) + len(autotune.SPLITS)
    d = json.load(open(path))
    assert all(k.endswith(tuple(choice)) for k in d)
    again = []
    assert autotune.tune(probs, roms, path=path, log=again.append) == choice
    assert again == []          # served from the cache
    with Batch(probs, roms) as bt:
        autotune.apply(bt, choice)
        bt.run(50)
        got = [bt.probes(b) for b in range(len(probs))]
    for b, (p, r) in enumerate(zip(probs, roms)):
        assert np.array_equal(got[b], _single(p, r, 50, "f32")[0][:50])


def test_c4_full_size_sampled():
    """The 64-instance batched workload (grids in [256,1024]^2, 1-8 models
    each): 800 steps batched; three instances against their own handles
    (bit-identical) and the smallest against the oracle with oracle-built
    models (probes and final fields)."""
    probs = W.batch_c4()
    print("[gpu-batch] building C4 models", flush=True)
    roms = romgen.build_roms_many(probs)
    k_or = min(range(len(probs)), key=lambda b: probs[b].nx * probs[b].ny)
    roms[k_or] = osim.build_roms(probs[k_or])
    n = 800
    with Batch(probs, roms, max_steps=n) as bt:
        bt.set_graph(100)
        bt.run(n)
        got = {b: bt.probes(b) for b in (0, 31, 63, k_or)}
        fl = [bt.field(k_or, c) for c in range(3)]
    print("[gpu-batch] C4 batch done", flush=True)
    for b in (0, 31, 63):
        pr, _ = _single(probs[b], roms[b], n, "f32")
        assert np.array_equal(got[b], pr), b
    pr, ofl = _oracle(probs[k_or], roms[k_or], n, fp32=True)
    assert np.abs(pr).max() > 0
    assert rel_l2(got[k_or], pr) <= 1e-5, rel_l2(got[k_or], pr)
    for c in range(3):
        assert rel_l2(fl[c], ofl[c]) <= 1e-5, (c, rel_l2(fl[c], ofl[c]))


def _c4_oracle_instance(b, n):
    """Spawned worker: oracle-built models of C4 instance b and the oracle's
    FP32-problem run of it over n steps (probes, final fields)."""
    import workloads as W_
    from oracle import sim as osim_
    p = W_.batch_c4()[b]
    roms = osim_.build_roms(p)
    run = osim_.CoupledRun(p, roms, mode="closed", fp32=True)
    pr = np.empty((n, len(p.probes)))
    for k in range(n):
        run.step()
        pr[k] = run.probes()
    return b, roms, pr, [run.f.hz * run.cell, run.f.ex, run.f.ey]


def test_c4_many_instances_vs_oracle():
    """Eight instances of the 64-instance workload - the five smallest grids
    and the three largest, 1 to 7 models each - run inside the full batch
    with oracle-built models (the other 56 with the library's), each against
    the oracle's run of its FP32 problem: probes and final fields within
    1e-5 relative L2, and the maximum over instances reported.  The oracle
    runs in spawned worker processes (no GPU use there)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    probs = W.batch_c4()
    order = sorted(range(len(probs)), key=lambda b: probs[b].nx * probs[b].ny)
    picked = order[:5] + order[-3:]
    n = 500
    print(f"[gpu-batch] C4 oracle for instances {picked}", flush=True)
    workers = max(1, min(len(picked), (os.cpu_count() or 2) // 2, 8))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        res = {b: (m, pr, fl) for b, m, pr, fl in ex.map(_c4_oracle_instance, picked, [n] * len(picked))}
    roms = romgen.build_roms_many(probs)
    for b in picked:
        roms[b] = res[b][0]
    print("[gpu-batch] C4 batch with oracle models", flush=True)
    with Batch(probs, roms, max_steps=n) as bt:
        bt.set_graph(100)
        bt.run(n)
        got = {b: (bt.probes(b), [bt.field(b, c) for c in range(3)]) for b in picked}
    worst = 0.0
    for b in picked:
        _, pr, fl = res[b]
        assert np.abs(pr).max() > 0, b
        e = [rel_l2(got[b][0], pr)] + [rel_l2(got[b][1][c], fl[c]) for c in range(3)]
        worst = max(worst, max(e))
        assert max(e) <= 1e-5, (b, e)
    print(f"[gpu-batch] C4 worst instance rel L2 vs oracle {worst:.2e}", flush=True)
