"""Benchmark: coarse-grid FDTD with embedded reduced models on one MI355X.

Workload (default): the 2048 x 2048 FP32 random-medium run - eps_r in
[1, 10], sigma in [0, 0.05] S/m per 32x32 patch (seeded), 16 embedded
32x32-cell regions refined 4x with orders {32, 48, 64, 96}, dt = 0.95 x the
coarse vacuum CFL limit, 10,000 steps, 64 probes.  A step is one leap-frog
step of the whole hot path: fused Hz/E stencil, every model's gather /
reduced update / scatter, probe record.  Reduced models come from the
library's host FP64 builder (setup, not timed).

Prints one JSON line (metric, value in Mcell-updates/s, roofline of the
stencil kernel from HIP events, oracle CPU baseline on a bounded sample).
Unless --no-forms, the line also carries the two other forms against the
plain solver on the same GPU:
  * "batched": the 64-instance workload (grids in [256,1024]^2, 1-8 models
    each, FP32) in one launch per step with autotuned tiles, against the
    same instances run one after another by single-problem handles;
  * "hbm_resident": the same recipe at 8192^2 (2.1 GB working set), the
    stencil's HBM-bound rate;
  * "many_copies": 4096^2 vacuum with 256 copies of one order-128 model,
    eq. (23) for all copies as one FP32 MFMA GEMM per step, against the
    same run with a GEMV per copy;
  * "adjoint": the 1024^2 probe-energy gradient (4 models q=64, 4000 steps,
    checkpoints every 200) against the forward run alone, and the FP32
    gradient's relative L2 distance to the FP64 run's.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s + % HBM roofline; batched & adjoint vs plain, 1 GPU, 1e-5 err"
PEAK_HBM_GBS = 8000.0
# algorithmic bytes of one step launch (FP32): per coarse cell Hz, Ex, Ey read
# + write (24 B) and the material - a 16-bit table index (2 B; the table of
# distinct (a, b) pairs is a few KB) or the per-cell pair (a, b) (8 B); per
# model the (q+np)^2 update matrix of eq. (23) read once
FIELD_BYTES_PER_CELL_F32 = 24
MATERIAL_BYTES_PER_CELL_F32 = {1: 2, 0: 8}


def step_bytes(prob, material_mode=1):
    cells = prob.nx * prob.ny
    mats = sum(4 * (s.q + s.n_ports) ** 2 for s in prob.roms)
    return (FIELD_BYTES_PER_CELL_F32 + MATERIAL_BYTES_PER_CELL_F32[material_mode]) * cells + mats


def pair_bytes(prob, material_mode=1):
    """Algorithmic bytes of one two-step pair of launches (FP32): the fields
    read and written once and the material read once for two steps, the
    update matrices read once per step."""
    cells = prob.nx * prob.ny
    mats = sum(4 * (s.q + s.n_ports) ** 2 for s in prob.roms)
    return (FIELD_BYTES_PER_CELL_F32 + MATERIAL_BYTES_PER_CELL_F32[material_mode]) * cells + 2 * mats


def stencil_roofline(prob, steps, ev_ms, mmode, tb, seg):
    """Algorithmic bytes per unit over the unit's average duration from the
    timed region's HIP events: the unit is one step launch, or with two
    steps per pass one pair of launches."""
    m = "true" if mmode else "false"
    if tb:
        units = steps / 2  # an odd step count ends with one single launch
        alg = pair_bytes(prob, mmode)
        kernel = f"step2_kernel<float,{seg},{m},false> + step2_kernel<float,{seg},{m},true> (one pair = two steps)"
    else:
        units = steps
        alg = step_bytes(prob, mmode)
        kernel = f"step_kernel<float,{seg},false,{m}>"
    avg_s = ev_ms / 1e3 / units
    return alg, avg_s, units, kernel
COUNTERS_FILE = os.path.join(ROOT, "profiles", "stencil_c2_2048_hbm_counters.json")


KERNEL_SOURCES = ("paper_1609_07114_amd/csrc/kernels.hip", "paper_1609_07114_amd/csrc/common.hpp",
                  "paper_1609_07114_amd/csrc/device.hpp")


def kernel_source_hash():
    """Hash of the sources the step kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(material_mode, tb=False):
    """HBM bytes per unit (step launch, or two-step pair) from committed
    rocprofv3 counter runs, if they were taken on the current kernel source
    in the same material and stepping mode (else None)."""
    try:
        with open(COUNTERS_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if (d.get("kernel_source_hash") != kernel_source_hash() or d.get("material_mode", 0) != material_mode
            or bool(d.get("time_blocking", 0)) != bool(tb)):
        return None
    return d.get("bytes_per_unit", d.get("bytes_per_launch"))


def cpu_baseline(prob, nsteps):
    """The oracle (NumPy FP64, closed form of eq. (23)) stepping the same
    grid for a bounded number of steps.  Model matrices are placeholders of
    the same orders (building oracle models is setup and is not timed)."""
    import numpy as np
    from oracle import sim as osim
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    rng = np.random.default_rng(0)
    roms = []
    for s in prob.roms:
        q, npt = s.q, s.n_ports
        roms.append(dict(Rt=np.eye(q), Ft=np.zeros((q, q)),
                         Lt=1e-3 * rng.standard_normal((q, npt))))
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        run = osim.CoupledRun(prob, roms, mode="closed", fp32=True)
        run.step()
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
            "sample": f"oracle NumPy FP64 (closed-form eq. (23), FP32-rounded coefficients) on the "
                      f"same {prob.nx}x{prob.ny} grid with {len(prob.roms)} models of the same "
                      f"orders, {nsteps} steps after 1 untimed step, single thread; model "
                      f"matrices are same-shape placeholders",
            "seconds": dt}


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


def bench_batched(steps=300, warmup=30, log=None):
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
        bt.run(warmup)
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


def bench_many_copies(steps=500, warmup=50, log=None):
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
            t, ev = _timed(s.stream, lambda: s.run(steps))
            res[mode] = (t, ev, s.probes())
    q = prob.roms[0].q
    m = -(-(q + prob.roms[0].n_ports) // 64) * 64          # padded rows of the update matrix
    flops = 2.0 * m * m * len(prob.roms)                   # one GEMM (m x m) . (m x copies) per step
    t_g = res["gemm"][1] / 1e3 / steps
    pg, pv = res["gemm"][2], res["gemv"][2]
    return {"workload": f"{prob.nx}x{prob.ny} vacuum, {len(prob.roms)} copies of one model "
                        f"q={q} (np={prob.roms[0].n_ports}), FP32, {steps} steps",
            "value": round(cells * steps / res["gemm"][0] / 1e6, 1), "unit": "Mcell-updates/s",
            "gemv_per_copy": round(cells * steps / res["gemv"][0] / 1e6, 1),
            "ms_per_step": round(res["gemm"][0] * 1e3 / steps, 4),
            "gemm_flop_per_step": flops,
            "gemm_tflops_over_step": round(flops / t_g / 1e12, 3),
            "mfma_frac_of_fp32_peak_over_step": round(flops / t_g / 1e12 / PEAK_MFMA_F32_TFLOPS, 5),
            "rel_l2_gemm_vs_gemv": float(np.linalg.norm(pg - pv) / max(np.linalg.norm(pv), 1e-300))}


def bench_hbm_resident(n=8192, steps=400, warmup=50, log=None):
    """The random-media recipe at n^2 (a working set well beyond the 256 MB
    Infinity Cache): the stencil's HBM-bound rate."""
    import workloads as W
    from paper_1609_07114_amd import romgen
    from paper_1609_07114_amd.sim import Simulation
    prob = W.random_media(n=n, nsteps=steps + warmup)
    roms = romgen.build_roms(prob)
    with Simulation(prob, roms) as s:
        seg = s.get_tiling()
        mmode, nmat = s.material_mode()
        tb = s.time_blocking()
        s.set_graph(min(steps, 200))
        s.run(warmup)
        t, ev = _timed(s.stream, lambda: s.run(steps))
    cells = prob.nx * prob.ny
    alg, avg, units, kernel = stencil_roofline(prob, steps, ev, mmode, tb, seg)
    return {"workload": f"random media {n}x{n}, 16 models (q 32-96), FP32, {steps} steps",
            "value": round(cells * steps / t / 1e6, 1), "unit": "Mcell-updates/s",
            "ms_per_step": round(t * 1e3 / steps, 4), "time_blocking": tb,
            "kernel": kernel,
            "material": {"mode": "table" if mmode else "per-cell", "entries": nmat},
            "bytes_per_unit": alg, "achieved_GBps": round(alg / avg / 1e9, 1),
            "frac_of_8TBps": round(alg / avg / 1e9 / PEAK_HBM_GBS, 4)}


def bench_adjoint(ckpt=200, log=None):
    import numpy as np
    import workloads as W
    from paper_1609_07114_amd import romgen
    from paper_1609_07114_amd.sim import Simulation
    prob = W.adjoint_c5()
    roms = romgen.build_roms(prob)
    n = prob.nsteps
    with Simulation(prob, roms) as s:
        s.set_graph(100)
        t_f, _ = _timed(s.stream, lambda: s.run(n))
    with Simulation(prob, roms) as s:      # untimed pass: graph capture, allocator
        s.set_graph(100)
        s.adjoint(n, ckpt_every=ckpt)
    with Simulation(prob, roms) as s:
        s.set_graph(100)
        res = {}
        t_a, _ = _timed(s.stream, lambda: res.setdefault("r", s.adjoint(n, ckpt_every=ckpt)))
        J32, ge32, gs32 = res["r"]
    with Simulation(prob, roms, dtype="f64") as s:
        J64, ge64, gs64 = s.adjoint(n, ckpt_every=ckpt)
    cells = prob.nx * prob.ny
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"workload": f"{prob.nx}x{prob.ny}, 4 models q=64, {n} steps, checkpoint every {ckpt}, FP32",
            "forward_s": round(t_f, 4), "adjoint_s": round(t_a, 4),
            "ratio_vs_forward": round(t_a / t_f, 2),
            "value": round(cells * n / t_a / 1e6, 1), "unit": "Mcell-updates/s (forward+reverse)",
            "J_rel_err_vs_f64": abs(J32 - J64) / abs(J64),
            "grad_eps_rel_l2_vs_f64": rel(ge32, ge64), "grad_sigma_rel_l2_vs_f64": rel(gs32, gs64)}


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
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=2048, help="grid size (default: the 2048^2 workload)")
    ap.add_argument("--cpu-steps", type=int, default=400,
                    help="oracle steps timed for cpu_baseline (about 20 s of one host core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched, many-copies and adjoint forms")
    ap.add_argument("--only", choices=["batched", "many_copies", "adjoint", "hbm_resident", "waveguides",
                                       "ablations", "sweep"], default=None,
                    help="run one form alone and print its JSON (profiling)")
    ap.add_argument("--form-steps", type=int, default=None, help="timed steps of the batched / many-copies form")
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

    import torch
    import workloads as W
    from paper_1609_07114_amd import romgen
    from paper_1609_07114_amd.sim import Simulation

    if not torch.cuda.is_available():
        print("bench.py: no ROCm GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_ceiling:
        print(json.dumps({"copy_ceiling": copy_ceiling()}), flush=True)
        return
    if args.only:
        log = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
        kw = {} if args.form_steps is None or args.only == "adjoint" else {"steps": args.form_steps}
        fn = {"batched": bench_batched, "many_copies": bench_many_copies, "adjoint": bench_adjoint,
              "hbm_resident": bench_hbm_resident, "waveguides": bench_waveguides,
              "ablations": bench_ablations, "sweep": bench_sweep}[args.only]
        print(json.dumps({args.only: fn(log=log, **kw)}), flush=True)
        return
    total = args.warmup + args.steps
    prob = W.random_media(n=args.n, nsteps=total)
    t0 = time.perf_counter()
    roms = romgen.build_roms(prob)
    t_build = time.perf_counter() - t0
    print(f"bench: {len(roms)} reduced models built in {t_build:.1f} s", file=sys.stderr, flush=True)

    if args.calibrate_copy_mib:
        nb = args.calibrate_copy_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    sim = Simulation(prob, roms, max_steps=total)
    seg = sim.get_tiling()
    if args.material_mode is not None:
        sim.set_material_mode(args.material_mode)
    mmode, nmat = sim.material_mode()
    sim.set_time_blocking(bool(args.time_blocking))
    tb = sim.time_blocking()
    sim.set_graph(200)   # steps replayed from captured graphs (the production path)
    sim.run(args.warmup)
    torch.cuda.synchronize()
    # timed region: K step launches on the simulation's stream, bracketed by
    # synchronisation and by one HIP event pair on that stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(sim.stream)
    sim.run(args.steps)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev_ms = ev0.elapsed_time(ev1)
    probes = sim.probes(0, total)
    sim.close()
    import numpy as np
    finite = bool(np.all(np.isfinite(probes)))

    elapsed = t1 - t0
    ms_step = elapsed * 1e3 / args.steps
    cells = prob.nx * prob.ny
    value = cells * args.steps / elapsed / 1e6
    # one launch per step, or one pair of launches per two steps; the
    # region's event time also holds the run's closing probe-flush and tick
    # launches (~8 us over all K steps)
    alg_bytes, st_avg_s, units, kernel = stencil_roofline(prob, args.steps, ev_ms, mmode, tb, seg)
    achieved = alg_bytes / st_avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(mmode, tb),
                "kernel": kernel, "time_blocking": tb,
                "material": {"mode": "table" if mmode else "per-cell", "entries": nmat},
                "bytes_per_unit": alg_bytes, "unit_of_work": "two-step pair" if tb else "step launch",
                "avg_unit_us": round(st_avg_s * 1e6, 3), "units": units}
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"C2 random media {prob.nx}x{prob.ny}, 16 embedded 32x32-cell "
                               f"models (r=4, q in 32/48/64/96), dt=0.95 coarse CFL, "
                               f"{args.steps} timed steps, 64 probes"
                               + (", two steps per pass" if tb else ""),
                   "nx": prob.nx, "ny": prob.ny, "n_models": len(prob.roms),
                   "orders": sorted({s.q for s in prob.roms}), "parallelism": "single GPU"},
        "roofline": roofline,
        "model_build_s": round(t_build, 2),
        "finite": finite,
    }
    print(f"bench: GPU {value:.0f} Mcell-updates/s, {ms_step:.4f} ms/step", file=sys.stderr, flush=True)
    if not args.no_forms:
        log = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
        out["batched"] = bench_batched(log=log)
        log(f"batched {out['batched']['value']:.0f} vs plain {out['batched']['plain_sequential']:.0f} Mcell/s")
        out["hbm_resident"] = bench_hbm_resident(log=log)
        log(f"hbm-resident 8192^2: {out['hbm_resident']['achieved_GBps']:.0f} GB/s")
        out["many_copies"] = bench_many_copies(log=log)
        log(f"many copies {out['many_copies']['value']:.0f} Mcell/s (GEMV {out['many_copies']['gemv_per_copy']:.0f})")
        out["adjoint"] = bench_adjoint(log=log)
        log(f"adjoint {out['adjoint']['ratio_vs_forward']}x forward")
        out["waveguides"] = bench_waveguides(log=log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
