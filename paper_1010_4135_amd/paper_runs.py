"""The paper's shock-bubble and shock-droplet runs (Sec. 4 (2)) on the GPU.

For each of the light bubble and the heavy droplet: the interior 298 x 78 x
78 grid of the paper's (0:301, 0:81, 0:81) nodes, (c1, c2, eta0) = (2, 6,
4), dx = 0.001, dt = tau = 1e-5, 10000 steps (t = 0.1), run in FP64 and in
FP32 with FP64 moments and equilibrium.  Reports the stability admission,
the autotuned launch shape and store kind, health, the change of the domain
totals (the faces are open, so the totals move by the fluxes through them:
relative change of mass and energy, change of each momentum component per
unit of initial mass), the FP32 run's relative L1 distance to the FP64 run
per field, and the time; writes the density on the paper's
section z = 40 (interior plane 38) at t = 0.1 of every run to
<out>/<kind>_<precision>_z40.npy and a JSON summary to <out>/summary.json.

    python -m paper_1010_4135_amd.paper_runs [--out DIR] [--steps N]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import inputs, lbm3d, metrics


def run(out_dir: str, steps: int = 10000, kinds=("bubble", "droplet"), precisions=("fp64", "fp32_t64")) -> dict:
    os.makedirs(out_dir, exist_ok=True)
    summary = {"grid": [298, 78, 78], "steps": steps, "t": steps * inputs.PAPER_BUBBLE_MODEL["dt"],
               "model": inputs.PAPER_BUBBLE_MODEL, "runs": {}}
    for kind in kinds:
        case = inputs.paper_shock_bubble(kind, steps=steps)
        rc, om = lbm3d.lbm3d_admit(case.params, case.fields)
        ref = None
        for prec in precisions:
            prm = dict(case.params, precision=prec)
            with lbm3d.Solver(prm) as s:
                s.init(*case.fields)
                tile = s.tune()  # launch shape for this grid (the state is unchanged)
                stores = "non-temporal" if s.streaming() else "plain"
                c0 = s.conserved()
                ms = s.step_timed(steps)
                health, done = s.status()
                m = s.moments(allow_nonfinite=True)
                c1 = s.conserved()
            mass0 = float(c0[0])
            row = {"admission": {"status": lbm3d.lbm3d_strerror(rc), "max_omega": round(om, 6)}, "tile": list(tile),
                   "stores": stores, "health": health, "steps_done": done, "device_ms": round(ms, 2),
                   "mlups": round(case.sites * steps / (ms / 1e3) / 1e6, 1),
                   "totals_t0": [float(v) for v in c0], "totals_end": [float(v) for v in c1],
                   "change_of_totals": {"mass_relative": float((c1[0] - c0[0]) / c0[0]),
                                        "momentum_per_initial_mass": [float((c1[k] - c0[k]) / mass0) for k in (1, 2, 3)],
                                        "energy_relative": float((c1[4] - c0[4]) / c0[4])}}
            if prec == "fp64":
                ref = m
            elif ref is not None:
                row["rel_l1_vs_fp64"] = {k: float(f"{v:.3e}") for k, v in metrics.rel_l1(m, ref).items()}
            rho = m[0]
            np.save(os.path.join(out_dir, f"{kind}_{prec}_z40.npy"), np.ascontiguousarray(rho[38]))
            row["rho_z40"] = {"min": float(rho[38].min()), "max": float(rho[38].max()),
                              "mean": float(rho[38].mean())}
            summary["runs"][f"{kind}_{prec}"] = row
            print(f"[paper run] {kind} {prec}: " + json.dumps({k: v for k, v in row.items()
                                                             if k not in ("totals_t0", "totals_end")}),
                  flush=True)
    with open(os.path.join(out_dir, "summary.json"), "w") as fh:
        json.dump(summary, fh, indent=1)
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="paper_runs_out")
    ap.add_argument("--steps", type=int, default=10000)
    a = ap.parse_args()
    run(a.out, a.steps)


if __name__ == "__main__":
    main()
