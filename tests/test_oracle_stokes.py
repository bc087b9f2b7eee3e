"""Stokes flow through a periodic array of fixed spheres (Sec. 2.4).

The normalized force C of Sec. 2.4.2 must reach the printed reference 2.842
with TRT-type operators independently of the viscosity, while SRT's drag moves
with the relaxation rate (Sec. 2.4.3).  Coarser than the paper (D = 8 instead
of 20, L = 2 D as printed) so that the oracle finishes in seconds.
"""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _drag(tau, coll, D=8.0, steps=2000):
    L = int(GOLD["stokes_array"]["L_over_D"] * D)
    nu = (tau - 0.5) / 3
    a = 1e-7
    cfg = O.make_config(nx=L, ny=L, nz=L, walls=(0, 0, 0), nu=nu, collision=coll,
                        body_force=(a, 0, 0), max_spheres=1)
    d = O.RefDomain(cfg)
    s = d.add_sphere((L / 2, L / 2, L / 2), D / 2, 2.0)
    d.set_mode(s, O.MODE_FIXED)
    d.step(steps)
    F = d.sphere(s)["F_raw"][0]
    ubar = d.field("vel")[0].sum() / L ** 3
    return (F + np.pi / 6 * D ** 3 * a) / (3 * np.pi * nu * D * ubar)


def test_stokes_array_drag_trt_ab_viscosity_independent():
    cref = GOLD["stokes_array"]["C_ref"]
    c1 = _drag(1.0, O.TRT_AB)
    c2 = _drag(1.5, O.TRT_AB)
    assert abs(c1 / cref - 1) < 5e-3
    assert abs(c1 - c2) < 1e-4


def test_stokes_array_drag_srt_depends_on_viscosity():
    cref = GOLD["stokes_array"]["C_ref"]
    assert abs(_drag(1.5, O.SRT) / cref - 1) > 0.05
