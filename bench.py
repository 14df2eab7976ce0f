"""Benchmark: coarse-grid FDTD with embedded reduced models on one MI355X.

Workload (default, the headline): the many-copies run - a 4096 x 4096 FP32
vacuum guide with PEC walls holding 256 identical 32x32-cell regions refined
4x (eps_r = 4, sigma = 0.01 S/m) that share one order-128 reduced model,
dt = 0.95 x the coarse CFL limit, a Gaussian Ey line source (plane wave)
on column 8, 16 Hz probes.  Eq. (23) for all 256 copies runs as one FP32
MFMA GEMM per step.  A step is one leap-frog step of the whole hot path:
coarse Hz/E stencil, every model's gather / reduced update / scatter,
probe record.  The reduced model comes from the library's host FP64
builder (setup, not timed).  `--workload c2` selects the 2048^2 random
medium instead (16 models of orders 32-96, per-cell material).

Prints one JSON line: value in Mcell-updates/s, the roofline of the
dominant kernel from HIP events over the timed region, and the oracle's
CPU rate on a bounded sample of the same workload.  Unless --no-forms, the
line also carries the other forms against the plain solver on the same GPU:
  * "random_media_2048": the 2048^2 random-medium run (16 models);
  * "batched": the 64-instance workload (grids in [256,1024]^2, 1-8 models
    each, FP32) in one launch per step (pair) with autotuned tiles, against
    the same instances run one after another by single-problem handles;
  * "hbm_resident": the random-medium recipe at 8192^2 (2.1 GB working set);
  * "adjoint": the 1024^2 probe-energy gradient (4 models q=64, 4000 steps,
    checkpoints every 200) against the forward run alone, and the FP32
    gradient's relative L2 distance to the FP64 run's;
  * "waveguides": the two open guides of Sec. VI-B/VI-C at the paper's sizes.
Errors against the oracle come from separate, untimed runs of the same
workloads with the oracle-built models stored under tests/golden (written
by scripts there that call only the oracle): "vs_oracle" is the FP32 run
against the oracle evaluated on the same FP32-rounded coefficients and
update matrices, "vs_fp64" against the oracle's run of the unrounded FP64
problem (arithmetic plus coefficient rounding).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
GOLD = os.path.join(ROOT, "tests", "golden")

METRIC = "Mcell-updates/s + % HBM roofline; batched & adjoint vs plain, 1 GPU, 1e-5 err"
PEAK_HBM_GBS = 8000.0
# device row padding of the headline grid (fdtd_grid.pitch_pad): measured
# 152.5 vs 158.1 us per pair on 4096^2 FP32 with 64 columns
HEADLINE_PITCH_PAD = 64
# Bytes per coarse cell (FP32) that one two-step pair must move at least
# (compulsory): Hz, Ex, Ey read once and written once (24 B) and the 16-bit
# material index read once (2 B) for two steps; per model the (q+np)^2
# update matrix of eq. (23) once per step (one copy per shared group).
# With one launch per step the same bytes move every step.
FIELD_BYTES_PER_CELL_F32 = 24
MATERIAL_BYTES_PER_CELL_F32 = {1: 2, 0: 8}
# The per-cell-step figure of the scope table's measurement section (24 B:
# fields, scalar coefficients; 32 B with per-cell eps_r, sigma): what a
# schedule that moves the fields every step would move.  Over a pair it
# counts two cell-steps, so "effective" rates of the two-step schedule can
# exceed the bandwidth they use.
EFFECTIVE_BYTES_PER_CELL_STEP = {"vacuum": 24, "material": 32}


def model_bytes(prob):
    """Update-matrix bytes of one step: one (q+np)^2 FP32 matrix per distinct model."""
    seen, tot = set(), 0
    for k, s in enumerate(prob.roms):
        key = s.group if s.group >= 0 else ("own", k)
        if key in seen:
            continue
        seen.add(key)
        tot += 4 * (s.q + s.n_ports) ** 2
    return tot


def unit_bytes(prob, material_mode=1, tb=True):
    """Compulsory bytes of one unit of work (FP32): a two-step pair (fields
    and material once, matrices twice) or one step launch."""
    cells = prob.nx * prob.ny
    per_cell = FIELD_BYTES_PER_CELL_F32 + MATERIAL_BYTES_PER_CELL_F32[material_mode]
    return per_cell * cells + (2 if tb else 1) * model_bytes(prob)


def stencil_roofline(prob, steps, ev_ms, mmode, tb, seg, kind):
    """Compulsory bytes per unit over the unit's average duration from the
    timed region's HIP events (unit: one step launch, or with two steps per
    pass one pair of launches), and the effective figure at the
    per-cell-step bytes of the scope table."""
    m = "true" if mmode else "false"
    if tb:
        units = steps / 2  # an odd step count ends with one single launch
        kernel = (f"step2_kernel<float,{seg},{m},false> + step2_kernel<float,{seg},{m},true> "
                  f"(one pair = two steps)")
    else:
        units = steps
        kernel = f"step_kernel<float,{seg},false,{m}>"
    alg = unit_bytes(prob, mmode, tb)
    avg_s = ev_ms / 1e3 / units
    achieved = alg / avg_s / 1e9
    eff_bytes = EFFECTIVE_BYTES_PER_CELL_STEP[kind] * prob.nx * prob.ny * (2 if tb else 1) + \
        (2 if tb else 1) * model_bytes(prob)
    eff = eff_bytes / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "kernel": kernel,
            "bytes": "compulsory",
            "bytes_per_unit": alg, "unit_of_work": "two-step pair" if tb else "step launch",
            "avg_unit_us": round(avg_s * 1e6, 3), "units": units,
            "effective": {"bytes_per_unit": eff_bytes,
                          "per_cell_step_B": EFFECTIVE_BYTES_PER_CELL_STEP[kind],
                          "achieved": round(eff, 1), "frac": round(eff / PEAK_HBM_GBS, 4)}}


KERNEL_SOURCES = ("paper_1609_07114_amd/csrc/kernels.hip", "paper_1609_07114_amd/csrc/common.hpp",
                  "paper_1609_07114_amd/csrc/device.hpp")
COUNTERS = {"c3": os.path.join(ROOT, "profiles", "step2_pair_c3_4096_hbm_counters.json"),
            "c2": os.path.join(ROOT, "profiles", "step2_pair_c2_2048_hbm_counters.json"),
            "hbm": os.path.join(ROOT, "profiles", "step2_pair_hbm_8192_counters.json")}


def kernel_source_hash():
    """Hash of the sources the step kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, material_mode, tb=False, seg=None, split=None, pitch_pad=0):
    """HBM bytes per unit (step launch, or two-step pair) from committed
    rocprofv3 counter runs, if they were taken on the current kernel source
    in the same material and stepping mode, rows per wave, pair split and
    row padding (else None)."""
    try:
        with open(COUNTERS[workload]) as fh:
            d = json.load(fh)
    except (OSError, ValueError, KeyError):
        return None
    if (d.get("kernel_source_hash") != kernel_source_hash() or d.get("material_mode", 0) != material_mode
            or bool(d.get("time_blocking", 0)) != bool(tb)
            or (seg is not None and d.get("rows_per_wave") != seg)
            or (split is not None and d.get("pair_split", 0) != split)
            or d.get("pitch_pad", 0) != pitch_pad):
        return None
    return d.get("bytes_per_unit", d.get("bytes_per_launch"))


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count()
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "cpus_available": avail}


def cpu_baseline(nsteps=20, n=4096):
    """The oracle (NumPy FP64; closed form of eq. (23) for every region;
    FP32-rounded coefficients and update matrices, the way an FP32 run is
    checked) stepping the headline workload - 4096^2 with 256 regions of
    the oracle-built order-128 model - for a bounded number of steps on its
    own problem instance (nsteps + 2 steps of sources).  Setup (the model
    build and the per-region closed forms) is not timed; BLAS is held to
    one thread, the stencil is single-threaded NumPy."""
    import numpy as np
    import workloads as W
    from oracle import sim as osim
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_info = threadpool_limits = None
    prob = W.many_copies(n=n, nsteps=nsteps + 2)
    one = W.many_copies(n=n, nsteps=nsteps + 2)
    one.roms = one.roms[:1]
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        blas = [{"api": d.get("internal_api"), "num_threads": d.get("num_threads")}
                for d in threadpool_info()] if threadpool_info else []
        t0 = time.perf_counter()
        m = osim.build_roms(one)[0]
        run = osim.CoupledRun(prob, [m] * len(prob.roms), mode="closed", fp32=True)
        t_setup = time.perf_counter() - t0
        run.step()
        run.probes()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            run.step()
            run.probes()
        dt = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    rate = prob.nx * prob.ny * nsteps / dt / 1e6
    return {"value": rate, "unit": "Mcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (NumPy FP64, closed-form eq. (23), FP32-rounded coefficients and update "
                      f"matrices) on the headline workload {prob.nx}x{prob.ny} with {len(prob.roms)} "
                      f"regions of the oracle-built q={prob.roms[0].q} model: {nsteps} steps timed after "
                      f"1 untimed step, one thread (BLAS limited to 1, NumPy stencil single-threaded)",
            "seconds": round(dt, 3), "setup_s": round(t_setup, 2),
            "host": {**host_info(), "blas_threads_during_timing": blas}}


def _timed(stream, fn):
    """Wall time and event time (ms) of fn() on `stream`, synchronised."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, e0.elapsed_time(e1)


def copy_ceiling(sizes_mib=(64, 128, 256, 512, 1024, 2048, 4096)):
    """Device-to-device copy rate (read + write bytes / time) of torch's copy
    kernel at several sizes: the practical bandwidth a streaming kernel can
    reach on this GPU, cache-resident (<= 256 MB Infinity Cache) and not."""
    import torch
    out = {}
    for mb in sizes_mib:
        n = mb << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        it = 20 if mb <= 512 else 5
        _, ms = _timed(torch.cuda.current_stream(), lambda: [b.copy_(a) for _ in range(it)])
        out[f"{mb}MiB"] = round(2 * n / (ms / it) / 1e6, 1)
        del a, b
    return {"unit": "GB/s (read+write)", "rates": out}


def bench_batched(steps=300, warmup=100, log=None):
    import numpy as np
    import workloads as W
    from paper_1609_07114_amd import autotune, romgen
    from paper_1609_07114_amd.batch import Batch
    from paper_1609_07114_amd.sim import Simulation
    probs = W.batch_c4(nsteps=max(3000, steps + warmup))
    t0 = time.perf_counter()
    roms = romgen.build_roms_many(probs)
    t_build = time.perf_counter() - t0
    cells = sum(p.nx * p.ny for p in probs)
    choice = autotune.tune(probs, roms, log=log)
    with Batch(probs, roms, max_steps=steps + warmup) as bt:
        autotune.apply(bt, choice)
        bt.set_graph(min(steps, 100))
        bt.run(warmup)          # captures the graph batch the timed run replays
        t_b, _ = _timed(bt.stream, lambda: bt.run(steps))
        pb = [bt.probes(b) for b in range(len(probs))]
    sims = [Simulation(p, r, max_steps=steps + warmup) for p, r in zip(probs, roms)]
    for s in sims:
        s.set_graph(min(steps, 100))
        s.run(warmup)
    t_p, _ = _timed(sims[0].stream, lambda: [s.run(steps) for s in sims])
    err = 0.0
    for s, a in zip(sims, pb):
        b = s.probes()
        d = np.linalg.norm(a - b)
        err = max(err, d / max(np.linalg.norm(b), 1e-300))
        s.close()
    rate_b = cells * steps / t_b / 1e6
    rate_p = cells * steps / t_p / 1e6
    return {"workload": f"{len(probs)} instances, grids in [256,1024]^2 ({cells / 1e6:.1f} M cells "
                        f"per step), {sum(len(p.roms) for p in probs)} models of orders 16-96, FP32",
            "steps": steps, "value": round(rate_b, 1), "unit": "Mcell-updates/s",
            "plain_sequential": round(rate_p, 1), "speedup": round(rate_b / rate_p, 3),
            "ms_per_step": round(t_b * 1e3 / steps, 4),
            "tiles": choice, "max_rel_l2_vs_plain": err, "model_build_s": round(t_build, 2)}


PEAK_MFMA_F32_TFLOPS = 157.3


def _rel(a, b):
    import numpy as np
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def golden_errors(workload):
    """Untimed run of the workload with the oracle-built models stored under
    tests/golden, compared with the oracle's stored probe series: FP32 run
    vs the oracle on the FP32-rounded problem ("vs_oracle") and vs the
    unrounded FP64 problem ("vs_fp64"), relative L2 over [steps x probes].
    None where the stored data are absent."""
    import numpy as np
    import workloads as W
    from paper_1609_07114_amd.sim import Simulation
    if workload == "c3":
        mpath, ppath = os.path.join(GOLD, "c3_model.npz"), os.path.join(GOLD, "c3_probes.npz")
        if not (os.path.exists(mpath) and os.path.exists(ppath)):
            return None
        z = np.load(ppath)
        n = int(z["steps"])
        prob = W.many_copies(nsteps=n)
        prob.pitch_pad = HEADLINE_PITCH_PAD
        zm = np.load(mpath)
        roms = [dict(Rt=zm["Rt"], Ft=zm["Ft"], Lt=zm["Lt"])] * len(prob.roms)
        ref32, ref64 = z["probes_f32"], z["probes_f64"]
    else:
        mpath, ppath = os.path.join(GOLD, "c2_models.npz"), os.path.join(GOLD, "c2_probes_f32.npz")
        if not (os.path.exists(mpath) and os.path.exists(ppath)):
            return None
        z = np.load(ppath)
        n = int(z["steps"])
        prob = W.random_media(n=2048, nsteps=n)
        zm = np.load(mpath)
        roms = [dict(Rt=zm[f"R{k}"], Ft=zm[f"F{k}"], Lt=zm[f"L{k}"]) for k in range(len(prob.roms))]
        ref32 = z["probes"]
        ref64 = z["probes_f64"] if "probes_f64" in z.files else None
    with Simulation(prob, roms, max_steps=n) as s:
        s.set_graph(200)
        s.run(n)
        got = s.probes()
    out = {"steps": n, "models": "oracle-built (tests/golden)", "vs_oracle": _rel(got, ref32)}
    out["vs_fp64"] = _rel(got, ref64) if ref64 is not None else None
    return out


def run_headline(prob, roms, steps, warmup, kind, workload, time_blocking=1, material_mode=None,
                 log=None):
    """Time exactly `steps` steps of one handle after `warmup` untimed ones
    (graph batches captured before the timed region), bracketed by
    synchronisation and one HIP event pair on the handle's stream."""
    import numpy as np
    import torch
    from paper_1609_07114_amd.sim import Simulation
    total = warmup + steps
    sim = Simulation(prob, roms, max_steps=total)
    seg = sim.get_tiling()
    if material_mode is not None:
        sim.set_material_mode(material_mode)
    mmode, nmat = sim.material_mode()
    sim.set_time_blocking(bool(time_blocking))
    tb = sim.time_blocking()
    gb = min(200, steps) // 4 * 4
    sim.set_graph(gb)   # steps replayed from captured graphs (the production path)
    sim.run(warmup)
    sim.prepare_run(steps)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(sim.stream)
    sim.run(steps)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev_ms = ev0.elapsed_time(ev1)
    probes = sim.probes(0, total)
    split = sim.pair_split() if tb else 0
    sim.close()
    elapsed = t1 - t0
    cells = prob.nx * prob.ny
    roof = stencil_roofline(prob, steps, ev_ms, mmode, tb, seg, kind)
    pad = getattr(prob, "pitch_pad", 0)
    roof["traffic"] = measured_traffic(workload, mmode, tb, seg, split, pad)
    roof["pair_split"] = split
    roof["pitch_pad"] = pad
    roof["material"] = {"mode": "table" if mmode else "per-cell", "entries": nmat}
    return {"value": cells * steps / elapsed / 1e6, "ms_per_step": elapsed * 1e3 / steps,
            "event_ms": ev_ms, "roofline": roof, "finite": bool(np.all(np.isfinite(probes))),
            "graph_batch": gb, "time_blocking": tb, "tiling": seg}


def bench_random_media(steps=2000, warmup=200, log=None):
    """The 2048^2 random-medium form (16 models of orders 32-96, per-cell
    material in 32x32 patches): same timing as the headline."""
    import workloads as W
    from paper_1609_07114_amd import romgen
    prob = W.random_media(n=2048, nsteps=steps + warmup)
    t0 = time.perf_counter()
    roms = romgen.build_roms(prob)
    t_build = time.perf_counter() - t0
    r = run_headline(prob, roms, steps, warmup, "material", "c2", log=log)
    return {"workload": f"random media {prob.nx}x{prob.ny}, 16 models (q 32-96), FP32, {steps} steps",
            "value": round(r["value"], 1), "unit": "Mcell-updates/s",
            "ms_per_step": round(r["ms_per_step"], 5), "roofline": r["roofline"],
            "model_build_s": round(t_build, 2), "errors": golden_errors("c2")}


def bench_gemv_vs_gemm(steps=500, warmup=52, log=None):
    """The headline workload with a GEMV per copy instead of the shared
    MFMA GEMM (same handle settings otherwise), probes compared."""
    import numpy as np
    import workloads as W
    from paper_1609_07114_amd import romgen
    from paper_1609_07114_amd.sim import Simulation
    prob = W.many_copies(nsteps=steps + warmup)
    roms = romgen.build_roms(prob)
    cells = prob.nx * prob.ny
    res = {}
    for mode in ("gemm", "gemv"):
        with Simulation(prob, roms) as s:
            s.set_shared_gemm(mode == "gemm")
            s.set_graph(100)
            s.run(warmup)
            s.prepare_run(steps)
            t, ev = _timed(s.stream, lambda: s.run(steps))
            res[mode] = (t, ev, s.probes())
    q = prob.roms[0].q
    m = q + prob.roms[0].n_ports
    flops = 2.0 * m * m * len(prob.roms)                   # one GEMM (m x m) . (m x copies) per step
    t_g = res["gemm"][1] / 1e3 / steps
    return {"workload": f"{prob.nx}x{prob.ny} vacuum, {len(prob.roms)} copies of one model q={q}, "
                        f"FP32, {steps} steps",
            "gemm": round(cells * steps / res["gemm"][0] / 1e6, 1),
            "gemv_per_copy": round(cells * steps / res["gemv"][0] / 1e6, 1), "unit": "Mcell-updates/s",
            "gemm_flop_per_step": flops,
            "gemm_tflops_over_step": round(flops / t_g / 1e12, 3),
            "mfma_frac_of_fp32_peak_over_step": round(flops / t_g / 1e12 / PEAK_MFMA_F32_TFLOPS, 5),
            "rel_l2_gemm_vs_gemv": _rel(res["gemm"][2], res["gemv"][2])}


def bench_hbm_resident(n=8192, steps=400, warmup=52, log=None):
    """The random-media recipe at n^2 (a working set well beyond the 256 MB
    Infinity Cache): the stencil's HBM-bound rate."""
    import workloads as W
    from paper_1609_07114_amd import romgen
    prob = W.random_media(n=n, nsteps=steps + warmup)
    roms = romgen.build_roms(prob)
    r = run_headline(prob, roms, steps, warmup, "material", "hbm", log=log)
    return {"workload": f"random media {n}x{n}, {len(prob.roms)} models (q 32-96), FP32, {steps} steps",
            "value": round(r["value"], 1), "unit": "Mcell-updates/s",
            "ms_per_step": round(r["ms_per_step"], 5), "roofline": r["roofline"]}


def bench_adjoint(ckpt=200, log=None):
    import numpy as np
    import workloads as W
    from paper_1609_07114_amd import capi, romgen
    from paper_1609_07114_amd.sim import Simulation
    prob = W.adjoint_c5()
    roms = romgen.build_roms(prob, keep=True)   # builder states kept for the gradients below
    n = prob.nsteps
    # both timed runs start with their graph batches captured (prepare_run):
    # the forward's for the whole run, the adjoint's for its checkpoint
    # segments, which its forward replays
    with Simulation(prob, roms) as s:
        s.set_graph(100)
        s.prepare_run(n)
        t_f, _ = _timed(s.stream, lambda: s.run(n))
    with Simulation(prob, roms) as s:      # untimed pass: allocator, code paths
        s.set_graph(100)
        s.adjoint(n, ckpt_every=ckpt)
    with Simulation(prob, roms) as s:
        s.set_graph(100)
        s.prepare_run(ckpt)
        res = {}
        t_a, _ = _timed(s.stream, lambda: res.setdefault("r", s.adjoint(n, ckpt_every=ckpt)))
        J32, ge32, gs32 = res["r"]
    # every forward state resident in HBM: one segment of n steps, so the
    # recompute is the only forward (12.6 MB per FP32 step, ~50 GB at 4000
    # steps of the 288 GB); an untimed call first leaves the workspace in
    # torch's cache
    for _ in range(2):
        with Simulation(prob, roms) as s:
            s.set_graph(100)
            res = {}
            t_r, _ = _timed(s.stream, lambda: res.setdefault("r", s.adjoint(n, ckpt_every=n)))
            ws_all = capi.fdtd_rom_adjoint_workspace_size(s.h, n, n)
    ger, gsr = res["r"][1], res["r"][2]
    with Simulation(prob, roms, dtype="f64") as s:
        J64, ge64, gs64 = s.adjoint(n, ckpt_every=ckpt)
    # the same sweep with the gradients through the models: dJ/dG summed on
    # the device, then the closed form and the builder on the host (fine
    # cells of every region, basis held)
    with Simulation(prob, roms) as s:
        s.set_graph(100)
        s.prepare_run(ckpt)
        res = {}
        t_m, _ = _timed(s.stream, lambda: res.setdefault("m", s.adjoint_models(n, ckpt_every=ckpt)))
    _, _, _, mods32 = res["m"]
    t0 = time.perf_counter()
    fine32 = romgen.build_vjps(prob, mods32, roms=roms)
    t_b = time.perf_counter() - t0
    with Simulation(prob, roms, dtype="f64") as s:
        _, _, _, mods64 = s.adjoint_models(n, ckpt_every=ckpt)
    fine64 = romgen.build_vjps(prob, mods64, roms=roms)
    cells = prob.nx * prob.ny
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    fe32 = np.concatenate([f[0].ravel() for f in fine32])
    fe64 = np.concatenate([f[0].ravel() for f in fine64])
    fs32 = np.concatenate([f[1].ravel() for f in fine32])
    fs64 = np.concatenate([f[1].ravel() for f in fine64])
    return {"workload": f"{prob.nx}x{prob.ny}, 4 models q=64, {n} steps, checkpoint every {ckpt}, FP32",
            "forward_s": round(t_f, 4), "adjoint_s": round(t_a, 4),
            "ratio_vs_forward": round(t_a / t_f, 2),
            "value": round(cells * n / t_a / 1e6, 1), "unit": "Mcell-updates/s (forward+reverse)",
            "J_rel_err_vs_f64": abs(J32 - J64) / abs(J64),
            "grad_eps_rel_l2_vs_f64": rel(ge32, ge64), "grad_sigma_rel_l2_vs_f64": rel(gs32, gs64),
            "all_states_resident": {"ckpt_every": n, "workspace_GB": round(ws_all / 1e9, 1),
                                    "adjoint_s": round(t_r, 4), "ratio_vs_forward": round(t_r / t_f, 2),
                                    "grad_eps_rel_l2_vs_checkpointed": rel(ger, ge32),
                                    "grad_sigma_rel_l2_vs_checkpointed": rel(gsr, gs32),
                                    "grad_eps_rel_l2_vs_f64": rel(ger, ge64),
                                    "grad_sigma_rel_l2_vs_f64": rel(gsr, gs64)},
            "through_models": {"adjoint_models_s": round(t_m, 4),
                               "build_vjp_host_s": round(t_b, 4),
                               "build_vjp_note": "host FP64, regions in parallel threads, from the builder states kept at the build",
                               "ratio_vs_forward": round((t_m + t_b) / t_f, 2),
                               "fine_eps_rel_l2_vs_f64": rel(fe32, fe64),
                               "fine_sigma_rel_l2_vs_f64": rel(fs32, fs64)}}


# The paper's whole-run times of the proposed method (model building
# included) for the two open guides: Matlab on one 3.6 GHz CPU, step counts
# not stated (Tabs. II, III).  Context only.
PAPER_RUNTIME_S = {"E3": 118.5, "E4": 23.8}


def bench_waveguides(steps=None, log=None):
    """The open-waveguide experiments at the paper's sizes (Sec. VI-B: two
    order-648 models; Sec. VI-C: one order-1920 model of four copper rods),
    models built on the host by the library, then the full run on the
    device from captured graphs.  Each step is one launch whose cost is the
    coupling blocks streaming the update matrices: their bytes per step are
    sum over models of (q + ports)^2 x element size."""
    import numpy as np
    import workloads as W
    from paper_1609_07114_amd import romgen
    from paper_1609_07114_amd.sim import Simulation
    out = {}
    for name, mk, n in (("E3", W.iris_waveguide, 4000), ("E4", W.rods_reflection, 2000)):
        n = steps or n
        prob = mk(nsteps=n)
        t0 = time.perf_counter()
        roms = romgen.build_roms(prob)
        t_build = time.perf_counter() - t0
        res = {}
        for dt_name in ("f32", "f64"):
            es = 4 if dt_name == "f32" else 8
            gbytes = sum((s.q + s.n_ports) ** 2 * es for s in prob.roms)
            with Simulation(prob, roms, dtype=dt_name) as sm:
                # capture and first replays on this handle, untimed; the rest
                # of the run is timed and scaled to the whole run
                w = min(200, n // 4)
                sm.set_graph(min(n, 200))
                sm.run(w)
                t, ev = _timed(sm.stream, lambda: sm.run(n - w))
                t = t * n / (n - w)
                ev = ev * n / (n - w)
                pr = sm.probes()
            res[dt_name] = {"run_s": round(t, 4), "us_per_step": round(ev * 1e3 / n, 3),
                            "matrix_bytes_per_step": gbytes,
                            "matrix_GBps": round(gbytes / (ev / 1e3 / n) / 1e9, 1),
                            "finite": bool(np.all(np.isfinite(pr)))}
        out[name] = {"workload": f"{prob.name} {prob.nx}x{prob.ny}, models q={[s.q for s in prob.roms]}, "
                                 f"{n} steps, CFL number {prob.dt / W.courant_dt(prob.dx / prob.roms[0].r, prob.dy / prob.roms[0].r, 1.0):.2f}",
                     "model_build_s": round(t_build, 2), **res,
                     "total_s_f64": round(t_build + res["f64"]["run_s"], 3),
                     "paper_runtime_s": PAPER_RUNTIME_S[name],
                     "paper_context": "Matlab, one 3.6 GHz CPU, step count not stated"}
        if log:
            log(f"{name}: build {t_build:.2f} s, f32 {res['f32']['us_per_step']} us/step, "
                f"f64 {res['f64']['us_per_step']} us/step")
    return out


def bench_sweep(steps=None, log=None, count=64):
    """A design sweep of the iris guide (Sec. VI-B): ``count`` guides with
    different apertures (two order-648 models each) as one batch - one launch
    per step over every guide, replayed from captured graphs - against the
    same guides run one after another through single-problem handles.  Each
    batched step streams every guide's model rows ((q+np)^2 FP32 per region,
    3.8 MB per guide)."""
    import numpy as np
    import workloads as W
    from paper_1609_07114_amd import romgen
    from paper_1609_07114_amd.batch import Batch
    from paper_1609_07114_amd.sim import Simulation
    n = steps or 2000
    probs = W.iris_sweep(count=count, nsteps=n)
    t0 = time.perf_counter()
    roms = romgen.build_roms_many(probs)
    t_build = time.perf_counter() - t0
    w = min(200, n // 4)
    with Batch(probs, roms, max_steps=n) as bt:
        bt.set_graph(min(n, 200))
        bt.run(w)
        t_b, ev_b = _timed(bt.stream, lambda: bt.run(n - w))
        pb = [bt.probes(b) for b in range(count)]
    t_p = 0.0
    err = 0.0
    for p, r, a in zip(probs, roms, pb):
        with Simulation(p, r, max_steps=n) as s:
            s.set_graph(min(n, 200))
            s.run(w)
            t, _ = _timed(s.stream, lambda: s.run(n - w))
            t_p += t
            b = s.probes()
            err = max(err, float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)))
    rows = sum((sp.q + sp.n_ports) ** 2 * 4 for p in probs for sp in p.roms)
    per = ev_b / 1e3 / (n - w)
    return {"workload": f"{count} iris guides (apertures 4-26 fine cells), 2 models q=648 each, FP32, "
                        f"{n} steps ({w} untimed)",
            "guide_steps_per_s": round(count * (n - w) / t_b, 1),
            "sequential_guide_steps_per_s": round(count * (n - w) / t_p, 1),
            "speedup": round(t_p / t_b, 2), "us_per_batched_step": round(per * 1e6, 2),
            "model_bytes_per_step": rows, "model_GBps": round(rows / per / 1e9, 1),
            "max_rel_l2_vs_single": err, "model_build_s": round(t_build, 2)}


# Tabs. II and III: whole-run Matlab times of the method variants on one
# 3.6 GHz CPU (model building included), context only.
PAPER_VARIANT_S = {"E3": {"coarse": 28.9, "mor_only": 245.4, "cfl_only": 484.3, "proposed": 118.5},
                   "E4": {"coarse": 4.0, "mor_only": 68.4, "cfl_only": 537.2, "proposed": 23.8}}


def bench_ablations(steps=None, log=None, dtype="f64"):
    """The method variants of Tabs. II and III on the two open guides over
    the same simulated time: all-coarse Yee, MOR only (reduced models at the
    fine step, no clip), CFL extension only (identity basis + eq. (27) clip,
    a dense update of the whole restricted fine model per region) and the
    proposed method.  Per variant: host model build, handle creation (the
    FP64 closed form of eq. (23), passivity check, upload) and the device
    run from captured graphs."""
    import numpy as np
    import workloads as W
    from paper_1609_07114_amd import romgen
    from paper_1609_07114_amd.sim import Simulation
    out = {}
    for name, mk, n in (("E3", W.iris_waveguide, 4000), ("E4", W.rods_reflection, 2000)):
        n = steps or n
        res = {}
        for mode in ("coarse", "mor_only", "cfl_only", "proposed"):
            prob = W.ablation(mk, mode, n)
            cfg = W.ABLATIONS[mode]
            t0 = time.perf_counter()
            roms = romgen.build_roms(prob, basis=cfg["basis"], clip=cfg["clip"]) if prob.roms else []
            t_build = time.perf_counter() - t0
            for s, m in zip(prob.roms, roms):
                s.q = m["Rt"].shape[0]
            t0 = time.perf_counter()
            sim = Simulation(prob, roms, dtype=dtype)
            t_setup = time.perf_counter() - t0
            # graph capture and first replays on this handle, untimed; the
            # rest of the run is timed and scaled to the whole run
            w = min(200, prob.nsteps // 4)
            sim.set_graph(min(prob.nsteps, 200))
            sim.run(w)
            t_rest, ev = _timed(sim.stream, lambda: sim.run(prob.nsteps - w))
            t_run = t_rest * prob.nsteps / (prob.nsteps - w)
            pr = sim.probes()
            sim.close()
            res[mode] = {"steps": prob.nsteps, "model_states": [s.q for s in prob.roms],
                         "model_build_s": round(t_build, 3), "setup_s": round(t_setup, 3),
                         "run_s": round(t_run, 4), "us_per_step": round(ev * 1e3 / (prob.nsteps - w), 2),
                         "total_s": round(t_build + t_setup + t_run, 3),
                         "finite": bool(np.all(np.isfinite(pr))),
                         "paper_runtime_s": PAPER_VARIANT_S[name][mode]}
            if log:
                log(f"{name} {mode}: build {t_build:.1f} s, setup {t_setup:.1f} s, run {t_run:.3f} s "
                    f"({res[mode]['us_per_step']} us/step, {prob.nsteps} steps)")
        out[name] = {"dtype": dtype, "variants": res,
                     "paper_context": "Matlab, one 3.6 GHz CPU, model building included, step counts not stated"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", choices=["c3", "c2"], default="c3",
                    help="c3: 4096^2, 256 copies of one q=128 model (default); c2: 2048^2 random medium")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps timed for cpu_baseline (about 20 s of one host core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the other forms")
    ap.add_argument("--no-errors", action="store_true", help="skip the untimed runs against the oracle's data")
    ap.add_argument("--only", choices=["batched", "gemv_vs_gemm", "adjoint", "hbm_resident", "waveguides",
                                       "ablations", "sweep", "random_media"], default=None,
                    help="run one form alone and print its JSON (profiling)")
    ap.add_argument("--form-steps", type=int, default=None, help="timed steps of the form run by --only")
    ap.add_argument("--copy-ceiling", action="store_true", help="only measure device copy rates and exit")
    ap.add_argument("--material-mode", type=int, choices=[0, 1], default=None,
                    help="0: per-cell material arrays, 1: 16-bit index + table (default: table when available)")
    ap.add_argument("--time-blocking", type=int, choices=[0, 1], default=1,
                    help="two steps per pass over the grid (1, default) or one launch per step (0)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1609_07114_amd import romgen

    if not torch.cuda.is_available():
        print("bench.py: no ROCm GPU visible", file=sys.stderr)
        sys.exit(1)
    log = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
    if args.copy_ceiling:
        print(json.dumps({"copy_ceiling": copy_ceiling()}), flush=True)
        return
    if args.calibrate_copy_mib:
        nb = args.calibrate_copy_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only:
        kw = {} if args.form_steps is None or args.only == "adjoint" else {"steps": args.form_steps}
        fn = {"batched": bench_batched, "gemv_vs_gemm": bench_gemv_vs_gemm, "adjoint": bench_adjoint,
              "hbm_resident": bench_hbm_resident, "waveguides": bench_waveguides,
              "ablations": bench_ablations, "sweep": bench_sweep, "random_media": bench_random_media}[args.only]
        print(json.dumps({args.only: fn(log=log, **kw)}), flush=True)
        return
    total = args.warmup + args.steps
    if args.workload == "c3":
        prob = W.many_copies(nsteps=total)
        # 64 unused columns per device row: 3.7 % faster on this grid (rows
        # of 16 KB fall unevenly on the memory channels); results identical
        prob.pitch_pad = HEADLINE_PITCH_PAD
        kind = "vacuum"
        desc = (f"C3 many copies {prob.nx}x{prob.ny} vacuum, {len(prob.roms)} embedded 32x32-cell regions "
                f"(r=4, eps_r=4, sigma=0.01) sharing one q={prob.roms[0].q} model (FP32 MFMA GEMM over the "
                f"copies), dt=0.95 coarse CFL, Ey plane-wave line source, {len(prob.probes)} probes, device rows "
                f"padded by {prob.pitch_pad} columns")
    else:
        prob = W.random_media(n=2048, nsteps=total)
        kind = "material"
        desc = (f"C2 random media {prob.nx}x{prob.ny}, 16 embedded 32x32-cell models (r=4, q in "
                f"32/48/64/96), dt=0.95 coarse CFL, 64 probes")
    t0 = time.perf_counter()
    roms = romgen.build_roms(prob)
    t_build = time.perf_counter() - t0
    log(f"{len(roms)} reduced models built in {t_build:.1f} s")

    r = run_headline(prob, roms, args.steps, args.warmup, kind, args.workload, args.time_blocking,
                     args.material_mode, log=log)
    tb = r["time_blocking"]
    out = {
        "metric": METRIC, "value": round(r["value"], 1), "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc + (", two steps per pass" if tb else ""),
                   "nx": prob.nx, "ny": prob.ny, "n_models": len(prob.roms),
                   "orders": sorted({s.q for s in prob.roms}), "parallelism": "single GPU"},
        "roofline": r["roofline"],
        "model_build_s": round(t_build, 2),
        "finite": r["finite"],
    }
    log(f"GPU {r['value']:.0f} Mcell-updates/s, {r['ms_per_step']:.4f} ms/step, "
        f"frac {r['roofline']['frac']}")
    if not args.no_errors:
        out["errors"] = golden_errors(args.workload)
        log(f"errors {out['errors']}")
    if not args.no_forms:
        out["gemv_vs_gemm"] = bench_gemv_vs_gemm(log=log)
        log(f"gemm {out['gemv_vs_gemm']['gemm']:.0f} vs gemv {out['gemv_vs_gemm']['gemv_per_copy']:.0f} Mcell/s")
        if args.workload != "c2":
            out["random_media_2048"] = bench_random_media(log=log)
            log(f"random media 2048^2 {out['random_media_2048']['value']:.0f} Mcell/s")
        out["batched"] = bench_batched(log=log)
        log(f"batched {out['batched']['value']:.0f} vs plain {out['batched']['plain_sequential']:.0f} Mcell/s")
        out["hbm_resident"] = bench_hbm_resident(log=log)
        log(f"hbm-resident 8192^2: {out['hbm_resident']['roofline']['achieved']:.0f} GB/s")
        out["adjoint"] = bench_adjoint(log=log)
        log(f"adjoint {out['adjoint']['ratio_vs_forward']}x forward, every state resident "
            f"{out['adjoint']['all_states_resident']['ratio_vs_forward']}x")
        out["waveguides"] = bench_waveguides(log=log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
        log(f"cpu baseline {out['cpu_baseline']['value']:.1f} Mcell/s")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
