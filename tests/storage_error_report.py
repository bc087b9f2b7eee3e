"""Error of reduced population storage (FP32 / FP16 deviations from w_q) against
the FP64 oracle on the 128^3 sub-run of the 512^3 precision variant: the dense
suspension generator at 128^3 with 375 spheres of D = 12 (16 % solids, as the
full case), 300 coupled steps.

Two steps, because the oracle needs ~20 minutes on one core:

    python tests/storage_error_report.py oracle REF.npz [steps]   # CPU, oracle only
    python tests/storage_error_report.py gpu REF.npz [steps]      # GPU, compares

The first runs only the oracle and stores its fields and sphere states; the
second runs the GPU library with FP64, FP32 and FP16 storage on the same seeded
input and prints one JSON line of errors against the stored oracle result:
velocity field (max and rms over fluid cells, relative to max / rms |u|),
resolved force per sphere (max relative to max |F|, median of per-sphere
relative errors) and positions (max |dx| / D).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

from paper_2003_01490_amd import workloads as W  # noqa: E402


def workload():
    return W.dense(0, n=128, count=375)


def run_oracle(out, steps):
    from harness import oracle_domain

    wl = workload()
    o = oracle_domain(wl)
    t = time.time()
    for k in range(0, steps, 25):
        o.step(min(25, steps - k))
        print(f"oracle {min(k + 25, steps)} steps {time.time() - t:.0f}s", flush=True)
    S = [o.sphere(i) for i in range(len(wl.R))]
    np.savez_compressed(out, vel=o.field("vel"), flags=o.flags()[0], x=np.array([s["x"] for s in S]),
                        u=np.array([s["u"] for s in S]), F_fp=np.array([s["F_fp"] for s in S]), steps=steps)


def run_gpu(ref_path, steps):
    from harness import gpu_domain

    ref = np.load(ref_path)
    assert int(ref["steps"]) == steps
    wl = workload()
    fluid = ref["flags"] <= 1
    uref = ref["vel"]
    umag = np.sqrt((uref ** 2).sum(0))[fluid]
    Fmag = np.linalg.norm(ref["F_fp"], axis=1)
    out = {"workload": "dense 128^3, 375 spheres D=12, %d steps" % steps}
    for storage, tag in ((0, "f64"), (1, "f32"), (2, "f16")):
        g = gpu_domain(wl, storage=storage)
        g.step(steps)
        g.sync()
        s = g.spheres()
        du = np.sqrt(((g.field("vel") - uref) ** 2).sum(0))[fluid]
        dF = np.linalg.norm(s["F_fp"] - ref["F_fp"], axis=1)
        out[tag] = {
            "vel_max_err_over_max_u": float(du.max() / umag.max()),
            "vel_rms_err_over_rms_u": float(np.sqrt((du ** 2).mean()) / np.sqrt((umag ** 2).mean())),
            "F_fp_max_err_over_max_F": float(dF.max() / Fmag.max()),
            "F_fp_median_rel_err": float(np.median(dF / Fmag)),
            "x_max_err_over_D": float(np.abs(s["x"] - ref["x"]).max() / 12.0),
            "flags_equal": bool(np.array_equal(g.field("flags"), ref["flags"])),
        }
        g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    n = int(sys.argv[3]) if len(sys.argv) > 3 else 300
    run_oracle(path, n) if mode == "oracle" else run_gpu(path, n)
