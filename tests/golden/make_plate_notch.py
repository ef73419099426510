"""Writes plate_notch_l1.json: oracle results of the notched-plate benchmark
(the box stand-in for the paper's Section 5 plate with a hole, level 1) in
its two time discretizations, (a) one step and (b) eight steps to t = 1/4.

Calls oracle/ only.  Per load step it stores the Newton history (PCGP
iterations, plastic elements, stopping criterion), the plastic element
count, max |u| and ||u|| over untorn DOFs, and u at every 251st untorn DOF.
Run from the repository root:  python tests/golden/make_plate_notch.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle.newton import Solver  # noqa: E402

STRIDE = 251


def run(steps):
    w = W.plate_notch(1, steps=steps)
    o = Solver(w, "tfeti")
    out = []
    for k in range(steps):
        h = o.load_step()
        u = o.global_displacement()
        out.append(dict(
            load_factor=w.load_factor(k + 1),
            newton=[dict(pcg_iters=int(r["pcg_iters"]), plastic_el=int(r["plastic_el"]), crit=float(r["crit"]))
                    for r in h],
            plastic_el=int((o.kappa > 0).any(axis=1).sum()),
            u_max=float(np.abs(u).max()),
            u_norm=float(np.linalg.norm(u)),
            u_sample=[float(v) for v in u[::STRIDE]],
        ))
        print(f"steps={steps} load step {k + 1}: {len(h)} Newton iterations, "
              f"{out[-1]['plastic_el']} plastic elements", flush=True)
    return out


def main():
    res = {"workload": "plate_notch level 1", "stride": STRIDE, "a": run(1), "b": run(8)}
    with open(os.path.join(HERE, "plate_notch_l1.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
