"""Write the oracle's reference data for the 4096^2 many-copies workload
(vacuum guide, 256 regions sharing one order-128 model, Ey plane-wave line
source, FP32 problem).

Calls only ``oracle`` (and the seeded ``workloads`` recipe):
  * c3_model.npz  - the shared reduced model built by the oracle's builder
                    (Rt, Ft, Lt);
  * c3_probes.npz - over ``steps`` steps:
      probes_f32   [steps, 16] oracle run of the FP32 problem (FP64
                   arithmetic on the FP32-rounded stencil coefficients and
                   eq. (23) update matrix, what an FP32 run computes with);
      probes_f64   [steps, 16] oracle run of the unrounded FP64 problem
                   (the error of an FP32 run against it is the error
                   against FP64: arithmetic plus coefficient rounding);
      hz_row_f32   Hz on row ny/2 after the last step (FP32 problem);
      hz_col_f32   Hz on column 300 after the last step (FP32 problem);
      x_f32        reduced states of regions 0, 17, 128, 255 after the last
                   step (FP32 problem), [4, q];
      steps.

Usage: python tests/golden/make_c3_golden.py [--steps 1200] [--which f32|f64|both]
The two runs are independent; ``--which`` lets them run as two processes
and merges into the same file.
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

STATE_REGIONS = (0, 17, 128, 255)
COL = 300


def model(prob):
    mpath = os.path.join(HERE, "c3_model.npz")
    if os.path.exists(mpath):
        z = np.load(mpath)
        return dict(Rt=z["Rt"], Ft=z["Ft"], Lt=z["Lt"])
    s = prob.roms[0]
    t0 = time.time()
    m = orom.build_rom(s.eps_r, s.sigma, s.r, prob.dx, prob.dy, prob.dt, s.q, s.f_max)
    print(f"model q={s.q} built in {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(mpath, Rt=m["Rt"], Ft=m["Ft"], Lt=m["Lt"])
    return dict(Rt=m["Rt"], Ft=m["Ft"], Lt=m["Lt"])


def run(prob, m, steps, fp32):
    roms = [m] * len(prob.roms)
    t0 = time.time()
    r = osim.CoupledRun(prob, roms, mode="closed", fp32=fp32)
    print(f"fp32={fp32}: set up in {time.time() - t0:.0f} s", flush=True)
    pr = np.empty((steps, len(prob.probes)))
    t0 = time.time()
    for n in range(steps):
        r.step()
        pr[n] = r.probes()
        if n % 100 == 0:
            print(f"fp32={fp32} step {n} {time.time() - t0:.0f} s max|probe|={np.abs(pr[:n + 1]).max():.3e}",
                  flush=True)
    hz = r.f.hz * r.cell
    return dict(probes=pr, hz_row=hz[prob.ny // 2].copy(), hz_col=hz[:, COL].copy(),
                x=np.stack([r.x[k] for k in STATE_REGIONS]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1200)
    ap.add_argument("--which", choices=["f32", "f64", "both"], default="both")
    a = ap.parse_args()
    prob = W.many_copies(nsteps=a.steps)
    m = model(prob)
    out = {}
    for tag in (("f32", "f64") if a.which == "both" else (a.which,)):
        res = run(prob, m, a.steps, fp32=(tag == "f32"))
        out[f"probes_{tag}"] = res["probes"]
        if tag == "f32":
            out.update(hz_row_f32=res["hz_row"], hz_col_f32=res["hz_col"], x_f32=res["x"])
        np.savez_compressed(os.path.join(HERE, f"_c3_part_{tag}.npz"), steps=np.int64(a.steps),
                            **{k: v for k, v in out.items() if k.endswith(tag)})
    parts = {}
    for tag in ("f32", "f64"):
        p = os.path.join(HERE, f"_c3_part_{tag}.npz")
        if os.path.exists(p):
            z = np.load(p)
            if int(z["steps"]) == a.steps:
                parts.update({k: z[k] for k in z.files if k != "steps"})
    if all(k in parts for k in ("probes_f32", "probes_f64")):
        np.savez_compressed(os.path.join(HERE, "c3_probes.npz"), steps=np.int64(a.steps),
                            state_regions=np.array(STATE_REGIONS), hz_col_index=np.int64(COL), **parts)
        for tag in ("f32", "f64"):
            os.remove(os.path.join(HERE, f"_c3_part_{tag}.npz"))
        print("wrote c3_probes.npz", flush=True)


if __name__ == "__main__":
    main()
