"""Tile autotuner for batched runs.

Two knobs.  Rows per stencil wave (4, 8, 16 or 32) per size bucket: short
segments give more workgroups (better for small grids), long ones recompute
fewer halo rows.  Then, for two steps per pass, the share of every
instance's far tiles that a pair's second launch advances (0, 25 or 50 %):
far tiles may run in either launch, and in the second they run beside the
coupling blocks and band blocks, whose chains of dependent loads would
otherwise run alone there.  In a batch the instances share the GPU, so the
best choice depends on the whole mix; the tuner times the batch itself.
Instances are grouped into size buckets; starting from 16 rows everywhere
and no split, each bucket (largest first) takes the candidate with the
shortest measured step time while the others stay fixed, then the split is
chosen the same way.  Trials run on a scratch batch built from the same
problems, so the caller's state is not touched.  Choices are cached in a
JSON file keyed by "<gfx arch>|<dtype>|<bucket>" and "<gfx arch>|<dtype>|split"
(FDTD_ROM_AUTOTUNE_CACHE overrides the default path
~/.cache/fdtd_rom/autotune.json)."""
from __future__ import annotations

import json
import os

CANDIDATES = (4, 8, 16, 32)
SPLITS = (0, 25, 50)
SPLIT = "split"
# (name, upper bound on coarse cells)
BUCKETS = (("s", 1 << 17), ("m", 1 << 19), ("l", 1 << 62))


def bucket_of(prob) -> str:
    cells = prob.nx * prob.ny
    for name, hi in BUCKETS:
        if cells <= hi:
            return name
    return BUCKETS[-1][0]


def cache_path() -> str:
    env = os.environ.get("FDTD_ROM_AUTOTUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "fdtd_rom", "autotune.json")


def load_cache(path=None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(d: dict, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _arch(device) -> str:
    import torch
    name = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "gpu")
    return name.split(":")[0]


def _key(arch, dtype, bucket):
    return f"{arch}|{dtype}|{bucket}"


def _time_steps(batch, steps) -> float:
    """Mean ms per step over `steps` steps (events on the batch's stream)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.run(steps)
    e1.record(batch.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(probs, rom_mats, dtype=None, trial_steps=40, device="cuda:0", cache=None,
         path=None, log=None):
    """Return {bucket: rows, ..., "split": percent} for the buckets present
    in probs, timing only knobs missing from the cache; updates the cache
    file."""
    from .batch import Batch
    dtype = dtype or probs[0].dtype
    arch = _arch(device)
    cache = load_cache(path) if cache is None else cache
    buckets = [bucket_of(p) for p in probs]
    present = [name for name, _ in reversed(BUCKETS) if name in buckets]   # largest first
    choice = {b: int(cache[_key(arch, dtype, b)]) for b in present if _key(arch, dtype, b) in cache}
    if _key(arch, dtype, SPLIT) in cache:
        choice[SPLIT] = int(cache[_key(arch, dtype, SPLIT)])
    todo = [b for b in present if b not in choice]
    tune_split = SPLIT not in choice
    if not todo and not tune_split:
        return choice
    warm = 8
    trials = len(todo) * len(CANDIDATES) + (len(SPLITS) if tune_split else 0)
    avail = min(p.nsteps for p in probs)
    trial_steps = max(2, min(trial_steps, (avail - warm) // (2 * trials)))
    cap = warm + 2 * trials * trial_steps
    if cap > avail:
        raise ValueError(f"problems allow {avail} steps; autotuning needs {cap}")
    cur = {b: choice.get(b, 16) for b in present}
    with Batch(probs, rom_mats, max_steps=cap, dtype=dtype, device=device) as bt:
        bt.set_graph(trial_steps)

        def set_all():
            for k, b in enumerate(buckets):
                bt.set_tiling(k, cur[b])

        set_all()
        bt.set_pair_split(-1, choice.get(SPLIT, 0))
        bt.run(warm)
        for b in todo:
            best = None
            for seg in CANDIDATES:
                cur[b] = seg
                set_all()
                bt.run(trial_steps)             # graph capture + first replay
                ms = _time_steps(bt, trial_steps)
                if log:
                    log(f"autotune {b}: rows={seg} {ms * 1e3:.1f} us/step")
                if best is None or ms < best[1]:
                    best = (seg, ms)
            cur[b] = best[0]
            choice[b] = best[0]
            cache[_key(arch, dtype, b)] = best[0]
        set_all()
        if tune_split:
            best = None
            for pct in SPLITS:
                bt.set_pair_split(-1, pct)
                bt.run(trial_steps)             # graph capture + first replay
                ms = _time_steps(bt, trial_steps)
                if log:
                    log(f"autotune split={pct}% {ms * 1e3:.1f} us/step")
                if best is None or ms < best[1]:
                    best = (pct, ms)
            choice[SPLIT] = best[0]
            cache[_key(arch, dtype, SPLIT)] = best[0]
    save_cache(cache, path)
    return choice


def apply(batch, choice):
    """Set every instance's rows per wave (and the pair split, when the
    choice holds one) from a tune() choice."""
    for k, p in enumerate(batch.probs):
        batch.set_tiling(k, choice[bucket_of(p)])
    if SPLIT in choice:
        batch.set_pair_split(-1, choice[SPLIT])
