"""The whole four-way coupled path against a number the paper prints.

Sphere-wall collision at St = 27 (Sec. 4.4.2 / 4.4.3, parameter set SW9 with
n_sub = 10): a sphere of D_p = 20 in a 12 x 12 x 48 D_p domain is ramped to
u_s = 0.02 by Eq. (artificial_acceleration), released one diameter above the
bottom wall, collides (linear spring-dashpot with T_c = 2.31 D_p / c_s,
lubrication with delta_min of Eq. lubricationGapSize) and rebounds.  The
rebound height H_r of Eq. (rebound_height) -- the largest gap after the first
contact, in diameters -- is read at the first apex (the library's rebound stop
rule).  The paper's ten perturbed runs give 0.3269 to 0.3276, average 0.3274
(Table sphereWallCollision_nsub_D20; tests/golden).  The start here is
perturbed by the seeded U[-1/2, 1/2] in z.  The bound is 1 % of the printed
average: five times the spread of the paper's runs, which leaves room for
FP32 population storage and for the readings of the paper's silences, and is
still far below what a wrong force, lubrication or contact term does to H_r
(the paper's own Figs. show several per cent for modest parameter changes).
About 49,000 steps on 55 M cells: ~90 s on one MI355X.
"""
import json
import os

import numpy as np
import pytest

from paper_2003_01490_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


@pytest.mark.timeout(900)
def test_rebound_height_st27_matches_table():
    from paper_2003_01490_amd import lbmdem as L

    ref = GOLD["rebound_height_st27_nsub"]
    k = ref["n_sub"].index(10)
    avg, lo, hi = ref["average"][k], ref["min"][k], ref["max"][k]
    wl = W.rebound_st27(0)
    keys = {f[0] for f in L.Config._fields_}
    p = {key: v for key, v in wl.params.items() if key in keys}
    cfg = L.default_config(**p, storage=L.STORE_F32, max_radius=float(wl.R[0]))
    print(f"[case] St = {wl.meta['St']:.2f} rebound, {cfg.nx}x{cfg.ny}x{cfg.nz}, D 20, FP32", flush=True)
    dom = L.Domain(cfg, device="cuda:0")
    dom.add_spheres(wl.x, wl.R, wl.rho)
    r = wl.ramp
    dom.set_mode(0, L.PRESCRIBED, r["u_target"], r["c_acc"], r["t_st"], r["release_gap"])
    dom.set_stop_rule(L.STOP_REBOUND, 80000)
    D = 2.0 * wl.R[0]
    while True:
        dom.step(5000)
        dom.sync()
        steps, stopped = dom.progress()
        s = dom.sphere(0)
        print(f"  step {steps} gap/D {(s['x'][2] - 1.0 - wl.R[0]) / D:.4f} u_z {s['u'][2]:.5f} "
              f"mode {s['mode']}", flush=True)
        if stopped:
            break
    assert steps < 80000, "no rebound apex within the step cap"
    s = dom.sphere(0)
    H_r = (s["x"][2] - 1.0 - wl.R[0]) / D
    print(f"  H_r {H_r:.5f}; paper (n_sub = 10): {lo} .. {hi}, average {avg}", flush=True)
    assert abs(s["u"][2]) < 1e-4  # at the apex
    assert abs(H_r - avg) <= 0.01 * avg
    dom.close()
