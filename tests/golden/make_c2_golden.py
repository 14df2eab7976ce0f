"""Write the oracle's reference data for the 2048^2 random-media workload.

Calls only ``oracle`` (and the seeded ``workloads`` recipe):
  * c2_models.npz  - the 16 reduced models built by the oracle's builder
                     (R~, F~, L~ per region, keys R{k}, F{k}, L{k});
  * c2_probes_f32.npz - probe series [nsteps, 64] of the oracle run of the
                     FP32 problem (FP64 arithmetic on the FP32-rounded
                     coefficients and closed-form matrices), stored as
                     float32, plus the run length.

Usage: python tests/golden/make_c2_golden.py [--steps 10000] [--models-only]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import rom as orom  # noqa: E402
from oracle import sim as osim  # noqa: E402


def build_models(prob):
    out = []
    for k, s in enumerate(prob.roms):
        t0 = time.time()
        m = orom.build_rom(s.eps_r, s.sigma, s.r, prob.dx, prob.dy, prob.dt, s.q, s.f_max)
        out.append(dict(Rt=m["Rt"], Ft=m["Ft"], Lt=m["Lt"]))
        print(f"model {k}: q={s.q} built in {time.time() - t0:.1f} s", flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--models-only", action="store_true")
    a = ap.parse_args()
    prob = W.random_media(n=2048, nsteps=a.steps)
    mpath = os.path.join(HERE, "c2_models.npz")
    if os.path.exists(mpath):
        z = np.load(mpath)
        models = [dict(Rt=z[f"R{k}"], Ft=z[f"F{k}"], Lt=z[f"L{k}"]) for k in range(len(prob.roms))]
    else:
        models = build_models(prob)
        np.savez_compressed(mpath, **{f"{n}{k}": m[key] for k, m in enumerate(models)
                                      for n, key in (("R", "Rt"), ("F", "Ft"), ("L", "Lt"))})
    if a.models_only:
        return
    run = osim.CoupledRun(prob, models, mode="closed", fp32=True)
    pr = np.empty((a.steps, len(prob.probes)))
    t0 = time.time()
    for n in range(a.steps):
        run.step()
        pr[n] = run.probes()
        if n % 500 == 0:
            print(f"step {n} {time.time() - t0:.0f} s max|probe|={np.abs(pr[:n + 1]).max():.3e}",
                  flush=True)
    np.savez_compressed(os.path.join(HERE, "c2_probes_f32.npz"), probes=pr.astype(np.float32),
                        steps=np.int64(a.steps))


if __name__ == "__main__":
    main()
