"""The fused step (map_kernel 3: particle links and momentum exchange formed
inside the sweep, geometric mapping update) against the separate boundary
passes and against the closed-ball rule, at every storage precision.

* With every sphere held fixed, nothing but the link arithmetic and the sums
  differ between the paths: the boundary values are the same FP64 expressions
  rounded to the storage type, so the PDF fields must be equal bit for bit at
  FP64, FP32 and FP16 (the dense 96^3 suspension, and rows wider than one
  tile with walls moving on both z sides), while forces and torques, summed
  in another order, agree to rounding.
* At the full size of the dense suspension (384^3, 10,000 spheres, FP32):
  closure of the momentum exchange at rest, the mapping of sampled spheres
  after 20 free steps against a brute-force evaluation of the closed-ball rule,
  and the trajectories against the one-block-per-sphere pass.
(The parity of the fused path with the FP64 oracle is in test_gpu_parity.py
and test_gpu_dense.py, parametrised over the boundary pass.)
"""
import numpy as np
import pytest

from paper_2003_01490_amd import workloads as W

from harness import gpu_domain, random_pdf

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _fix_all(g, P):
    from paper_2003_01490_amd import lbmdem as L

    for i in range(P):
        g.set_mode(i, L.FIXED)


def _same_fields_and_close_forces(a, b, tag):
    fa, fb = a.field("pdf"), b.field("pdf")
    assert np.array_equal(a.field("flags"), b.field("flags")), f"{tag}: flags differ"
    assert np.array_equal(fa, fb), f"{tag}: pdf differs, max {np.abs(fa - fb).max():.2e}"
    sa, sb = a.spheres(), b.spheres()
    Fs = max(float(np.abs(sb["F_fp"]).max()), 1e-300)
    eF = float(np.abs(sa["F_fp"] - sb["F_fp"]).max() / Fs)
    eT = float(np.abs(sa["T_fp"] - sb["T_fp"]).max() / Fs)
    print(f"  {tag}: fields equal bit for bit; forces {eF:.1e}, torques {eT:.1e} (of max |F|)", flush=True)
    assert eF < 1e-12 and eT < 1e-11, (eF, eT)


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_fused_equals_ball_pass_with_fixed_spheres(storage):
    wl = W.dense(0, n=96, count=156)
    P = len(wl.R)
    _case(f"dense 96^3, {P} fixed spheres, storage {storage}: fused against one block per sphere")
    f = random_pdf((96, 96, 96), seed=41, u0=(0.01, -0.005, 0.002))
    gs = []
    for mk in (2, 3):
        g = gpu_domain(wl, storage=storage, map_kernel=mk)
        _fix_all(g, P)
        g.set_pdf(f)
        gs.append(g)
    for chk in (1, 12):
        for g in gs:
            g.step(1 if chk == 1 else chk - 1)
        _same_fields_and_close_forces(gs[1], gs[0], f"step {chk}")


@pytest.mark.parametrize("storage", [1, 2])
def test_fused_wide_rows_with_moving_walls(storage):
    """384-cell rows (swept as 128 x 2 tiles), z walls moving in x, fixed
    spheres near the walls and across the periodic x boundary: fused against
    the slab pass, bit for bit."""
    n = (384, 24, 30)
    _case(f"wide rows {n}, 6 fixed spheres, storage {storage}: fused against slab blocks")
    x = np.array([[3.0, 12.2, 8.1], [381.5, 5.3, 20.7], [130.2, 18.0, 6.4], [255.9, 11.1, 15.0],
                  [200.0, 2.0, 24.5], [64.1, 22.9, 12.2]])
    R = np.array([4.0, 4.3, 3.8, 4.6, 3.5, 4.1])
    wl = W.Workload("wide", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 1), nu=0.02, max_spheres=6,
                                          wall_u_lo=(0.01, 0.0, 0.0), wall_u_hi=(-0.02, 0.0, 0.0)),
                    x, R, np.full(6, 2.0), np.zeros((6, 3)), np.zeros((6, 3)), 0)
    f = random_pdf(n, seed=33, u0=(0.02, 0.0, 0.0))
    gs = []
    for mk in (1, 3):
        g = gpu_domain(wl, storage=storage, map_kernel=mk)
        _fix_all(g, 6)
        g.set_pdf(f)
        gs.append(g)
    for g in gs:
        g.step(9)
    _same_fields_and_close_forces(gs[1], gs[0], "9 steps")


def _expected_codes(box_lo, box_hi, centres, R, dab, n, walls):
    from test_gpu_dense import _expected_codes as ec

    return ec(box_lo, box_hi, centres, R, dab, n, walls)


def test_fused_full_size_dense():
    from paper_2003_01490_amd import lbmdem as L

    wl = W.dense(0, n=384, count=10000, steps=1000)
    P = len(wl.R)
    _case(f"dense 384^3, {P} spheres, FP32 storage, fused against one block per sphere")
    g = gpu_domain(wl, storage=L.STORE_F32, map_kernel=3)
    g.step(1)
    g.sync()
    s = g.spheres()
    fmax, tmax = float(np.abs(s["F_fp"]).max()), float(np.abs(s["T_fp"]).max())
    print(f"  step 1: max |F_fp| {fmax:.2e}  max |T_fp| {tmax:.2e}", flush=True)
    assert fmax < 1e-11 and tmax < 1e-10  # closure at rest (missing links included)
    b = gpu_domain(wl, storage=L.STORE_F32, map_kernel=2)
    b.step(1)
    for k in (5, 20):
        g.step(k - (1 if k == 5 else 5))
        b.step(k - (1 if k == 5 else 5))
        sg, sb = g.spheres(), b.spheres()
        ex = float(np.abs(sg["x"] - sb["x"]).max() / 12.0)
        Fs = float(np.abs(sb["F_fp"]).max())
        ef = float(np.abs(sg["F_fp"] - sb["F_fp"]).max() / Fs)
        print(f"  step {k}: |dx|/D {ex:.1e}, |dF_fp|/max|F| {ef:.1e}", flush=True)
        assert ex < 1e-9 and ef < 1e-6
    b.close()
    n = (384, 384, 384)
    walls = (0, 0, 1)
    x = g.spheres()["x"]
    flags, owner = g.field("flags"), g.field("owner")
    rng = np.random.default_rng(7)
    R = wl.R
    reach = np.sqrt(3.0) * (R.max() + 3.0) + R.max() + 2.0 + 1.0
    for i in rng.choice(P, 40, replace=False):
        lo = np.floor(x[i] - R[i] - 3).astype(int)
        hi = np.floor(x[i] + R[i] + 3).astype(int) + 1
        lo[2], hi[2] = max(lo[2], 0), min(hi[2], n[2])
        dd = x - x[i]
        for a in range(2):
            dd[:, a] -= n[a] * np.round(dd[:, a] / n[a])
        near = np.nonzero(np.linalg.norm(dd, axis=1) < reach)[0]
        (K, J, I), code, own = _expected_codes(lo, hi, x[near], R[near], 2.0, n, walls)
        own = np.where(own >= 0, near[np.maximum(own, 0)], -1)
        assert np.array_equal(flags[K, J, I], code), f"flags of sphere {i} box differ"
        sol = code == 2
        assert np.array_equal(owner[K, J, I][sol], own[sol]), f"owners of sphere {i} box differ"
    print("  mapping of 40 sampled sphere boxes bit-exact after 20 steps", flush=True)
    g.close()
