"""Writes sphere_wall_oracle_2000.json: the FP64 oracle's sphere states over
the first 2,000 steps of the sphere-wall collision on 128 x 128 x 256 cells
(Sec. 4.4: D_p = 20, St = 100, prescribed approach at u_s = 0.028 with
c_acc = 10, seed 0).  Only the oracle runs here; the file is keyed by the
workload's parameters and the oracle's source hash, and the GPU test refuses
a stale file.  About 80 minutes on one core:

    python tests/golden/make_sphere_wall_oracle.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from harness import oracle_domain, oracle_fingerprint, workload_key  # noqa: E402
from paper_2003_01490_amd import workloads as W  # noqa: E402

STEPS = 2000
CHECKPOINTS = [1, 2, 5, 10, 20] + list(range(50, STEPS + 1, 50))
KEYS = ("x", "u", "w", "F_fp", "F_raw", "F_tot", "F_lub", "F_col", "T_fp", "T_raw")


def main(out=os.path.join(HERE, "sphere_wall_oracle_2000.json")):
    wl = W.sphere_wall(0)
    o = oracle_domain(wl)
    rec = []
    done, t0 = 0, time.time()
    for chk in CHECKPOINTS:
        o.step(chk - done)
        done = chk
        s = o.sphere(0)
        r = {"step": chk, "mode": int(s["mode"])}
        r.update({k: [float(v) for v in s[k]] for k in KEYS})
        rec.append(r)
        print(f"step {chk} z {s['x'][2]:.6f} uz {s['u'][2]:.3e} ({time.time() - t0:.0f} s)", flush=True)
    doc = {"cite": "Sec. 4.4 (sphere-wall collision, St = 100 row of Tab. sphereWallCollision) on a "
                   "128 x 128 x 256 lattice; oracle sphere states at the listed steps",
           "workload": "sphere_wall seed 0", "oracle_sha256": oracle_fingerprint(),
           "key": workload_key(wl), "records": rec}
    with open(out, "w") as f:
        json.dump(doc, f, indent=0)
        f.write("\n")


if __name__ == "__main__":
    main()
