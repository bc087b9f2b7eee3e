"""GPU (HIP library through the C-ABI) against the FP64 oracle.

FP64 storage: f, rho and u within 1e-12 of max|f|, positions within 1e-12 D,
cell flags and owners bit for bit.  Sphere velocities, angular velocities,
forces and torques within 1e-12 of the trajectory's largest |u| and |F|,
except where a test states a larger bound: those quantities come from the
momentum-exchange sum over thousands of links whose net value is 1e-3 to
1e-5 of their absolute sum, so summing in another order leaves relative
errors of ~1e-16 times that ratio; each larger bound sits 3 to 10 times above
the largest error the test has shown.  The velocity field relative to its own
max|u| (vel_rel, which divides f-level rounding by |u|/|f| ~ 1e-3) has such
bounds as well.  Every bound goes through harness.check(), which prints the
observed maxima at the end of the session.  Reduced storage (FP32, FP16
deviations from w_q): errors against the oracle are printed and held to the
bounds stated in each test.
"""
import numpy as np
import pytest

import oracle as O
from paper_2003_01490_amd import workloads as W

from harness import (Scales, check, check_all, exact_tie_counts, fp64_bounds, gpu_domain, oracle_domain, random_pdf,
                     sphere_errs, weight)

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _compare_fields(g, o, tol=TOL, vel_rel=1e-12):
    cg, og = g.flags()
    co, oo = o.flags()
    assert np.array_equal(cg, co), "flags differ"
    sol = co == O.SOLID
    assert np.array_equal(og[sol], oo[sol]), "owners differ"
    fg, fo = g.field("pdf"), o.field("pdf")
    fs = np.abs(fo).max()
    fl = co <= O.SHELL
    rg, ro = g.field("rho"), o.field("rho")
    ug, uo = g.field("vel"), o.field("vel")
    errs = {
        "pdf": float(np.abs(fg - fo).max() / fs),
        "rho": float(np.abs(rg[fl] - ro[fl]).max() / fs),
        "vel": float(np.abs(ug - uo).max() / fs),
    }
    rel_u = float(np.abs(ug - uo).max() / max(np.abs(uo).max(), 1e-300))
    print("  field errors", errs, f"u rel {rel_u:.1e}", flush=True)
    for k, e in errs.items():
        check(k, e, tol)
    if np.abs(uo).max() > 0.0:
        check("vel_rel", rel_u, vel_rel)


@pytest.mark.parametrize("coll", [O.TRT_AB, O.TRT_B, O.TRT, O.SRT])
def test_fluid_only_periodic_random_pdf(coll):
    n = (17, 12, 9)  # ragged x, several blocks in y and z
    _case(f"fluid periodic {n} collision {coll}")
    wl = W.Workload("fluid", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 0), nu=0.03,
                                           collision=coll, max_spheres=1),
                    np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), 0)
    f = random_pdf(n, seed=coll, u0=(0.02, -0.01, 0.015))
    o = oracle_domain(wl)
    g = gpu_domain(wl)
    o.set_pdf(f)
    g.set_pdf(f)
    o.step(25)
    g.step(25)
    _compare_fields(g, o)


@pytest.mark.parametrize("storage,n", [(0, (320, 5, 7)), (1, (384, 4, 6)), (1, (512, 4, 5)), (2, (320, 5, 7))])
def test_wide_rows(storage, n):
    """Rows wider than 256 cells: 320-wide FP64 rows are swept in 64-cell
    pieces (parity at 1e-12 against the oracle); 384-wide FP32 rows in 128 x 2
    pieces and 512-wide FP32 rows in 256 x 1 pieces with ordinary loads (the
    sweeps of the dense 384^3 and 512^3 FP32 workloads), and 320-wide FP16
    rows in one block each, against the oracle
    within a bound of the reduced precision: per step at most one rounding of
    the stored deviation (2^-24 relative at FP32, 2^-11 at FP16) plus, at FP32,
    16 roundings of the FP32 collision (moments, equilibrium, relaxation), on
    deviations of at most ~0.05, summed over the 12 steps.  z walls moving in x
    on both sides, so the wall branch runs in wide rows too."""
    _case(f"wide rows {n} storage {storage}")
    wl = W.Workload("wide", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 1), nu=0.02,
                                          max_spheres=1, wall_u_lo=(0.01, 0.0, 0.0), wall_u_hi=(-0.02, 0.0, 0.0)),
                    np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), 0)
    f = random_pdf(n, seed=31, u0=(0.02, -0.01, 0.0))
    o = oracle_domain(wl)
    g = gpu_domain(wl, storage=storage)
    o.set_pdf(f)
    g.set_pdf(f)
    o.step(12)
    g.step(12)
    if storage == 0:
        _compare_fields(g, o)
        return
    fo, fg = o.field("pdf"), g.field("pdf")
    code = o.flags()[0]
    fl = code <= O.SHELL
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None, None, None]
    dev = np.abs(fo - w)[:, fl].max()
    err = np.abs(fg - fo)[:, fl].max()
    bound = 12 * (2.0 ** -11 if storage == 2 else 17 * 2.0 ** -24) * dev
    print(f"  storage {storage} wide rows: max |df| {err:.2e}, max |f - w| {dev:.2e}, bound {bound:.2e}",
          flush=True)
    check("pdf", err, bound)


@pytest.mark.parametrize("coll,mk", [(O.TRT_AB, 0), (O.TRT_B, 0), (O.SRT, 0), (O.TRT_AB, 3)])
def test_body_force_fluid_and_fixed_sphere(coll, mk):
    """Guo forcing (the oracle's moment-space form against the sweep's
    velocity-space form): a periodic random field under a body force, then a
    fixed sphere in it (momentum exchange and the shell under forcing)."""
    n = (17, 12, 16)
    a = (2e-5, -1e-5, 3e-5)
    _case(f"body force {a} on {n}, collision {coll}, map_kernel {mk}")
    wl = W.Workload("forced", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 0), nu=0.03,
                                            collision=coll, max_spheres=1, body_force=a),
                    np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), 0)
    f = random_pdf(n, seed=11 + coll, u0=(0.01, 0.0, -0.005))
    o = oracle_domain(wl)
    g = gpu_domain(wl)
    o.set_pdf(f)
    g.set_pdf(f)
    o.step(10)
    g.step(10)
    _compare_fields(g, o, vel_rel=2e-11)
    wl.x, wl.R, wl.rho = np.array([[8.3, 6.1, 7.7]]), np.array([3.2]), np.array([1.0])
    wl.u, wl.w = np.zeros((1, 3)), np.zeros((1, 3))
    o, g = oracle_domain(wl), gpu_domain(wl, map_kernel=mk)
    o.set_mode(0, O.MODE_FIXED)
    from paper_2003_01490_amd import lbmdem as L
    g.set_mode(0, L.FIXED)
    for _ in range(4):
        o.step(15)
        g.step(15)
        so, sg = o.sphere(0), g.sphere(0)
        Fs = max(np.abs(so["F_raw"]).max(), 1e-300)
        check("F_raw", np.abs(sg["F_raw"] - so["F_raw"]).max() / Fs, 2e-11)
        check("T_raw", np.abs(sg["T_raw"] - so["T_raw"]).max() / (Fs * 3.2), 1e-12)
    _compare_fields(g, o, vel_rel=2e-11)


def test_density_probe_against_oracle_field():
    """lbmdem_probe_density: trilinear interpolation of the cell-centre
    densities, against the same interpolation of the oracle's density field
    (FP64 storage, settling workload after 60 steps), NaN next to solid or
    wall cells."""
    wl = W.settling_32(0)
    _case("density probe, settling_32 after 60 steps")
    o, g = oracle_domain(wl), gpu_domain(wl)
    o.step(60)
    g.step(60)
    rho = o.field("rho")  # (nz, ny, nx)
    code = o.flags()[0]
    rng = np.random.default_rng(5)
    pts = np.column_stack([rng.uniform(0, 32, 200), rng.uniform(0, 32, 200), rng.uniform(1.5, 30.5, 200)])
    got = g.probe_density(pts)
    for p, v in zip(pts, got):
        s = p - 0.5
        i0 = np.floor(s).astype(int)
        t = s - i0
        ref, fluid = 0.0, True
        for c in range(8):
            o3 = [(c >> a) & 1 for a in range(3)]
            ii = [(i0[0] + o3[0]) % 32, (i0[1] + o3[1]) % 32, i0[2] + o3[2]]
            w = np.prod([t[a] if o3[a] else 1 - t[a] for a in range(3)])
            fluid = fluid and code[ii[2], ii[1], ii[0]] <= O.SHELL
            ref += w * rho[ii[2], ii[1], ii[0]]
        if fluid:
            check("rho", abs(v - ref), 1e-12, p)
        else:
            assert np.isnan(v), (p, v)


def test_couette_channel_and_moving_walls():
    n = (8, 6, 14)
    _case(f"couette {n}")
    wl = W.Workload("couette", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 1), nu=0.1,
                                             wall_u_hi=(0.02, 0.005, 0.0),
                                             wall_u_lo=(-0.01, 0.0, 0.0), max_spheres=1),
                    np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), 0)
    f = random_pdf(n, seed=11)
    o, g = oracle_domain(wl), gpu_domain(wl)
    o.set_pdf(f)
    g.set_pdf(f)
    o.step(60)
    g.step(60)
    _compare_fields(g, o)


# boundary pass: automatic (slab), one block per sphere, fused into the sweep
@pytest.mark.parametrize("mk", [0, 2, 3])
def test_walls_on_all_axes(mk):
    n = (12, 11, 10)
    _case(f"closed box {n} map_kernel {mk}")
    wl = W.Workload("box", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(1, 1, 1), nu=0.05,
                                         max_spheres=2),
                    np.array([[4.3, 5.1, 4.9], [8.0, 5.5, 5.2]]), np.array([1.9, 1.7]),
                    np.array([2.0, 3.0]), np.array([[0.01, 0.0, -0.005], [-0.01, 0.002, 0.0]]),
                    np.zeros((2, 3)), 40)
    f = random_pdf(n, seed=12)
    o, g = oracle_domain(wl), gpu_domain(wl, map_kernel=mk)
    o.set_pdf(f)
    g.set_pdf(f)
    o.step(wl.steps)
    g.step(wl.steps)
    _compare_fields(g, o)
    for i in range(2):
        e = sphere_errs(g.sphere(i), o.sphere(i), 2 * wl.R[i])
        print("  sphere", i, {k: f"{v:.1e}" for k, v in e.items()}, flush=True)
        check_all(e, fp64_bounds(u=1e-11, w=2e-12, F_fp=2e-11, F_raw=2e-11, F_tot=2e-11, F_lub=1e-11))


@pytest.mark.parametrize("storage", [0, 1, 2])
# boundary pass: automatic (slab), one block per sphere, fused into the sweep
@pytest.mark.parametrize("mk", [0, 2, 3])
def test_mapping_bit_exact(storage, mk):
    n = (30, 28, 26)
    _case(f"mapping {n} storage {storage} map_kernel {mk}")
    rng = np.random.default_rng(5)
    xs, Rs = [], []
    # centres on cell centres with Pythagorean radii: cell centres lie exactly
    # on the R = 5 and R = 3 surfaces and on the R + delta_aB shell surfaces,
    # and the two R = 5 spheres touch at one cell centre (owner: lower id)
    cand = [([10.5, 10.5, 10.5], 5.0), ([20.5, 10.5, 10.5], 5.0), ([5.5, 20.5, 18.5], 3.0)]
    on_surface, on_shell, shared = exact_tie_counts(n, (0, 0, 1), cand)
    assert on_surface >= 60 and on_shell >= 100 and shared == 1
    for x, R in cand:
        xs.append(x)
        Rs.append(R)
    while len(xs) < 9:
        R = rng.uniform(1.2, 3.5)
        x = [rng.uniform(0, n[0]), rng.uniform(0, n[1]), rng.uniform(1.5 + R, n[2] - 1.5 - R)]
        def dist(y):
            v = np.array(x) - np.array(y)
            v[:2] -= np.round(v[:2] / np.array(n[:2])) * np.array(n[:2])  # periodic x, y
            return np.linalg.norm(v)
        ok = all(dist(y) > R + r + 0.05 for y, r in zip(xs, Rs))
        if ok:
            xs.append(x)
            Rs.append(R)
    wl = W.Workload("map", W.base_params(nx=n[0], ny=n[1], nz=n[2], max_spheres=len(xs)),
                    np.array(xs), np.array(Rs), np.full(len(xs), 2.0), np.zeros((len(xs), 3)),
                    np.zeros((len(xs), 3)), 0)
    o, g = oracle_domain(wl), gpu_domain(wl, storage=storage, map_kernel=mk)
    cg, og = g.flags()
    co, oo = o.flags()
    assert np.array_equal(cg, co)
    sol = co == O.SOLID
    assert sol.sum() > 100 and np.array_equal(og[sol], oo[sol])
    assert co[10, 10, 15] == O.SOLID and og[10, 10, 15] == 0  # the shared tie cell


# boundary pass: automatic (slab), fused into the sweep (the domain is too
# narrow for the one-block-per-sphere pass's staged cube)
@pytest.mark.parametrize("mk", [0, 3])
def test_fixed_sphere_forces_on_random_field(mk):
    n = (20, 18, 22)
    _case(f"fixed sphere forces {n} map_kernel {mk}")
    wl = W.Workload("fixed", W.base_params(nx=n[0], ny=n[1], nz=n[2], nu=0.02, max_spheres=2),
                    np.array([[9.3, 8.7, 11.2], [2.0, 3.0, 1.0 + 3.1 + 0.3]]), np.array([4.1, 3.1]),
                    np.array([2.0, 2.0]), np.array([[0.01, -0.02, 0.005], [0.0, 0.0, 0.0]]),
                    np.array([[0.001, 0.002, -0.003], [0.0, 0.001, 0.0]]), 0)
    f = random_pdf(n, seed=3, u0=(0.01, 0.0, -0.01))
    o, g = oracle_domain(wl), gpu_domain(wl, map_kernel=mk)
    for dom in (o, g):
        for i in range(2):
            dom.set_mode(i, O.MODE_FIXED)
        dom.set_pdf(f)
    for step in range(6):
        o.step(1)
        g.step(1)
        for i in range(2):
            so, sg = o.sphere(i), g.sphere(i)
            scale = np.abs(so["F_raw"]).max()
            check("F_raw", np.abs(sg["F_raw"] - so["F_raw"]).max() / scale, TOL, (step, i))
            tscale = max(np.abs(so["T_raw"]).max(), scale)
            check("T_raw", np.abs(sg["T_raw"] - so["T_raw"]).max() / tscale, TOL, (step, i))
    _compare_fields(g, o)


@pytest.mark.parametrize("seed,mk", [(0, 0), (1, 0), (0, 3)])
def test_settling_sphere_32_fp64(seed, mk):
    wl = W.settling_32(seed)
    _case(f"settling_32 seed {seed} FP64, {wl.steps} steps, map_kernel {mk}")
    o, g = oracle_domain(wl), gpu_domain(wl, map_kernel=mk)
    sc = Scales(weight(wl))
    done = 0
    for chk in (1, 10, 60, 150, 300):
        o.step(chk - done)
        g.step(chk - done)
        done = chk
        so = o.sphere(0)
        e = sphere_errs(g.sphere(0), so, 2 * wl.R[0], sc.update(so))
        print(f"  step {chk}", {k: f"{v:.1e}" for k, v in e.items()}, flush=True)
        check_all(e, fp64_bounds(u=1e-10, w=2e-12, F_fp=5e-11, F_raw=5e-11, F_tot=5e-11, T_fp=1e-12,
                                 T_raw=2e-12))
    _compare_fields(g, o, vel_rel=2e-10)


# boundary pass: automatic (slab), one block per sphere, fused into the sweep
@pytest.mark.parametrize("mk", [0, 2, 3])
def test_contact_variant_fp64(mk):
    """Contact and lubrication with the wall; the workgroup DEM kernel (LDS
    variant) and the one-thread-per-sphere one side by side."""
    wl = W.contact_32(0)
    _case(f"contact_32 FP64, {wl.steps} steps, DEM kernels 1 and 2, map_kernel {mk}")
    o = oracle_domain(wl)
    gs = [gpu_domain(wl, dem_kernel=1, map_kernel=mk), gpu_domain(wl, dem_kernel=2, map_kernel=mk)]
    sc = Scales(weight(wl))
    saw_contact = saw_lub = False
    done = 0
    for chk in (20, 60, 100, 150, 200, 300):
        o.step(chk - done)
        for g in gs:
            g.step(chk - done)
        done = chk
        so = o.sphere(0)
        saw_contact |= bool(np.abs(so["F_col"]).max() > 0)
        saw_lub |= bool(np.abs(so["F_lub"]).max() > 0)
        scale = sc.update(so)
        for k, g in enumerate(gs):
            e = sphere_errs(g.sphere(0), so, 2 * wl.R[0], scale)
            print(f"  step {chk} kernel {k + 1} gap {so['x'][2] - 1 - wl.R[0]:.4f}",
                  {kk: f"{v:.1e}" for kk, v in e.items()}, flush=True)
            check_all(e, fp64_bounds(u=1e-11, w=2e-12, F_fp=2e-11, F_raw=2e-11, F_tot=1e-11, F_lub=2e-11,
                                     T_raw=2e-12))
        a, b = gs[0].sphere(0), gs[1].sphere(0)
        assert all(np.array_equal(a[k], b[k]) for k in ("x", "u", "w", "F_tot", "T_tot")), "DEM kernels differ"
    assert saw_contact or saw_lub
    for g in gs:
        _compare_fields(g, o, vel_rel=5e-11)


# boundary pass: automatic (slab), one block per sphere, fused into the sweep
@pytest.mark.parametrize("mk", [0, 2, 3])
def test_two_spheres_oblique_collision_fp64(mk):
    n = (40, 24, 24)
    _case(f"two spheres colliding, periodic, DEM kernels 1 and 2, map_kernel {mk}")
    wl = W.Workload("pair", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 1), nu=0.02,
                                          tc=30.0, max_spheres=2),
                    np.array([[12.0, 12.1, 11.8], [12.0 + 8.45, 12.9, 12.2]]), np.array([4.0, 4.2]),
                    np.array([2.0, 3.0]), np.array([[0.04, 0.0, 0.0], [-0.04, 0.0, 0.0]]),
                    np.zeros((2, 3)), 120)
    o = oracle_domain(wl)
    gs = [gpu_domain(wl, dem_kernel=1, map_kernel=mk), gpu_domain(wl, dem_kernel=2, map_kernel=mk)]
    done = 0
    saw = False
    sc = [Scales(), Scales()]
    for chk in (10, 30, 50, 80, 120):
        o.step(chk - done)
        for g in gs:
            g.step(chk - done)
        done = chk
        for i in range(2):
            so = o.sphere(i)
            saw |= bool(np.abs(so["F_col"]).max() > 0)
            scale = sc[i].update(so)
            for k, g in enumerate(gs):
                e = sphere_errs(g.sphere(i), so, 8.0, scale)
                print(f"  step {chk} sphere {i} kernel {k + 1}", {kk: f"{v:.1e}" for kk, v in e.items()},
                      flush=True)
                check_all(e, fp64_bounds(u=2e-12), (chk, i))
    assert saw
    for g in gs:
        _compare_fields(g, o, vel_rel=1e-11)


# boundary pass: automatic (slab), one block per sphere, fused into the sweep
@pytest.mark.parametrize("mk", [0, 2, 3])
def test_prescribed_ramp_and_release(mk):
    n = (24, 24, 40)
    _case(f"prescribed ramp and release, map_kernel {mk}")
    wl = W.Workload("ramp", W.base_params(nx=n[0], ny=n[1], nz=n[2], nu=0.02,
                                          gravity=(0, 0, -2e-5), max_spheres=1),
                    np.array([[12.2, 11.9, 24.0]]), np.array([4.0]), np.array([3.0]),
                    np.zeros((1, 3)), np.zeros((1, 3)), 200,
                    ramp=dict(u_target=(0.0, 0.0, -0.04), c_acc=10.0, t_st=60.0, release_gap=12.0))
    o, g = oracle_domain(wl), gpu_domain(wl, map_kernel=mk)
    done = 0
    released = False
    sc = Scales(weight(wl))
    for chk in (20, 80, 140, 200):
        o.step(chk - done)
        g.step(chk - done)
        done = chk
        so, sg = o.sphere(0), g.sphere(0)
        released |= so["mode"] == O.MODE_FREE
        assert sg["mode"] == so["mode"]
        e = sphere_errs(sg, so, 8.0, sc.update(so))
        print(f"  step {chk}", {k: f"{v:.1e}" for k, v in e.items()}, flush=True)
        check_all(e, fp64_bounds(), chk)
    assert released
    _compare_fields(g, o, vel_rel=5e-12)


# boundary pass: automatic (slab), one block per sphere (geometric mapping
# update; at 18^3 its staged cube keeps whole rows), fused into the sweep
@pytest.mark.parametrize("mk", [0, 2, 3])
def test_update_spheres_reconstructs(mk):
    n = (18, 18, 18)
    _case(f"teleport + reconstruction, map_kernel {mk}")
    wl = W.Workload("tele", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 0), nu=0.04,
                                          max_spheres=1),
                    np.array([[8.3, 8.9, 9.1]]), np.array([3.6]), np.array([2.0]),
                    np.array([[0.01, 0.02, 0.0]]), np.array([[0.0, 0.0, 0.01]]), 0)
    f = random_pdf(n, seed=9, u0=(0.02, 0.0, 0.0))
    o, g = oracle_domain(wl), gpu_domain(wl, map_kernel=mk)
    for dom in (o, g):
        dom.set_mode(0, O.MODE_FIXED)
        dom.set_pdf(f)
        dom.step(3)
    for x in ([9.1, 9.4, 8.2], [17.5, 0.4, 9.0]):  # second one wraps the periodic corner
        o.update_sphere(0, x=x)
        g.update_spheres([0], x=np.array([x]))
        _compare_fields(g, o)
        o.step(2)
        g.step(2)
        _compare_fields(g, o)


def test_wide_rows_block_shape():
    n = (300, 5, 6)  # rows wider than one block, not a multiple of 256
    _case(f"wide rows {n}")
    wl = W.Workload("wide", W.base_params(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 1), nu=0.05,
                                          max_spheres=1),
                    np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), 0)
    f = random_pdf(n, seed=21, u0=(0.03, 0.0, 0.0))
    o, g = oracle_domain(wl), gpu_domain(wl)
    o.set_pdf(f)
    g.set_pdf(f)
    o.step(10)
    g.step(10)
    _compare_fields(g, o)


@pytest.mark.parametrize("storage,tol_u,tol_f", [(1, 1e-5, 1e-4), (2, 2e-2, 5e-2)])
def test_reduced_storage_error_vs_oracle(storage, tol_u, tol_f):
    wl = W.settling_32(0)
    _case(f"settling_32 storage {storage}")
    o, g = oracle_domain(wl), gpu_domain(wl, storage=storage)
    o.step(100)
    g.step(100)
    so, sg = o.sphere(0), g.sphere(0)
    uo, ug = o.field("vel"), g.field("vel")
    eu = float(np.abs(ug - uo).max() / np.abs(uo).max())
    ef = float(np.abs(sg["F_fp"] - so["F_fp"]).max() / np.abs(so["F_fp"]).max())
    ex = float(np.abs(sg["x"] - so["x"]).max() / (2 * wl.R[0]))
    print(f"  storage {storage}: |du|/|u| {eu:.2e}  |dF|/|F| {ef:.2e}  |dx|/D {ex:.2e}", flush=True)
    assert eu < tol_u and ef < tol_f


def test_empty_domain_and_state_errors():
    from paper_2003_01490_amd import lbmdem as L

    _case("errors and empty domain")
    wl = W.Workload("empty", W.base_params(nx=8, ny=8, nz=8, max_spheres=2),
                    np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), 0)
    g = gpu_domain(wl)
    g.step(3)
    g.sync()
    assert g.num_spheres() == 0
    assert g.try_add_spheres([[4.0, 4.0, 1.5]], 1.0, 2.0) == L.EOVERLAP     # crosses the wall
    assert g.try_add_spheres([[4.0, 4.0, 4.0]], 9.0, 2.0) == L.EINVAL       # R > max_radius
    assert g.try_add_spheres([[2.0, 2.0, 3.0], [3.0, 2.0, 3.0]], 0.8, 2.0) == L.EOVERLAP
    g.add_spheres([[2.0, 2.0, 3.0], [6.0, 6.0, 4.0]], 0.8, 2.0)
    assert g.try_add_spheres([[4.0, 2.0, 5.0]], 0.5, 2.0) == L.ECAPACITY
    g.step(2)
    g.sync()


def _state_bits(g):
    out = [g.field("pdf"), g.field("flags"), g.field("owner")]
    s = g.spheres()
    out += [s[k] for k in sorted(s)]
    for i in range(g.num_spheres()):
        st = g.sphere(i)
        out += [np.asarray(st[k]) for k in sorted(st)]
    return out


def _bitwise_equal(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("dem_kernel,mk", [(1, 0), (2, 0), (2, 2), (2, 3)])
def test_checkpoint_restore_bitwise(dem_kernel, mk):
    """Continuing from a checkpoint equals continuing the saved domain bit for
    bit (contact history, averaging memory, boundary values included)."""
    from paper_2003_01490_amd import lbmdem as L

    wl = W.dense(3, n=48, count=40, D=8.0, min_gap=0.2, u_rms=0.05, nu=0.01)
    _case(f"checkpoint, agitated 48^3, DEM kernel {dem_kernel}, map_kernel {mk}")
    g = gpu_domain(wl, dem_kernel=dem_kernel, map_kernel=mk)
    g.step(30)
    blob = g.save()
    g.step(40)
    ref = _state_bits(g)
    h = gpu_domain(wl, dem_kernel=dem_kernel, map_kernel=mk)
    h.step(3)  # a different state, overwritten by the restore
    h.restore(blob)
    h.step(40)
    assert _bitwise_equal(_state_bits(h), ref), "restored domain diverged"
    g.restore(blob)  # the saved domain itself, rewound
    g.step(40)
    assert _bitwise_equal(_state_bits(g), ref), "rewound domain diverged"
    other = gpu_domain(wl, dem_kernel=dem_kernel, nu=0.011)
    with pytest.raises(L.LbmdemError):
        other.restore(blob)


def test_unstable_state_is_reported_and_isolated():
    """A non-finite particle state (forced from the host: a NaN velocity) is
    reported as LBMDEM_EUNSTABLE by the domain's sync and fails only that
    domain; a domain stepped beside it in the same batch ends bit for bit as
    when stepped alone."""
    from paper_2003_01490_amd import lbmdem as L
    import torch

    wl = W.settling_32(0)
    _case("unstable state: NaN velocity, alone and in a batch")
    g = gpu_domain(wl, storage=1)
    g.step(2)
    g.sync()
    g.update_spheres([0], u=np.array([[np.nan, 0.0, 0.0]]))
    g.step(2)
    with pytest.raises(L.LbmdemError) as e:
        g.sync()
    assert e.value.code == L.EUNSTABLE
    with pytest.raises(L.LbmdemError) as e:
        g.step(1)
    assert e.value.code == L.ESTATE
    g.close()
    stream = torch.cuda.Stream()
    alone = gpu_domain(wl, storage=1, stream=stream, map_kernel=1)
    alone.step(20)
    alone.sync()
    ref = alone.spheres()
    pair = [gpu_domain(wl, storage=1, stream=stream, map_kernel=1) for _ in range(2)]
    b = L.Batch(stream, 1 << 34)
    for d in pair:
        b.admit(d)
    b.step(2)
    pair[1].update_spheres([0], u=np.array([[0.0, np.nan, 0.0]]))
    b.step(18)
    pair[0].sync()  # raises on any failure
    with pytest.raises(L.LbmdemError) as e:
        pair[1].sync()
    assert e.value.code == L.EUNSTABLE
    got = pair[0].spheres()
    assert all(np.array_equal(got[k], ref[k]) for k in ref), "the healthy domain was disturbed"
    b.close()


def test_one_harness_drives_both_interfaces():
    """The same ctypes code (tests/abi_harness.py) drives the GPU library's
    lbmdem_* calls and the oracle's lbmdem_ref_* mirror: contact with the wall
    and lubrication (contact_32, FP64 storage, 200 steps), sphere state and
    fields compared as in test_contact_variant_fp64."""
    from abi_harness import AbiDomain, config_from
    from paper_2003_01490_amd import lbmdem as L

    wl = W.contact_32(0)
    _case("contact_32 FP64 through one harness: lbmdem_* against lbmdem_ref_*")
    doms = []
    for lib, prefix in ((L.lib(), "lbmdem_"), (O.lib(), "lbmdem_ref_")):
        cfg = config_from(wl.params, lib, prefix, storage=0, max_radius=float(wl.R[0]),
                          max_spheres=max(len(wl.R), 1))
        dom = AbiDomain(lib, prefix, cfg)
        dom.add_spheres(wl.x, wl.R, wl.rho, u=wl.u, w=wl.w)
        doms.append(dom)
    g, o = doms
    sc = Scales(weight(wl))
    done = 0
    for chk in (20, 100, 200):
        for dom in doms:
            dom.step(chk - done)
        done = chk
        so = o.sphere(0)
        e = sphere_errs(g.sphere(0), so, 2 * wl.R[0], sc.update(so))
        print(f"  step {chk}", {k: f"{v:.1e}" for k, v in e.items()}, flush=True)
        check_all(e, fp64_bounds(u=1e-11, w=2e-12, F_fp=2e-11, F_raw=2e-11, F_tot=1e-11, F_lub=2e-11,
                                 T_raw=2e-12), chk)
    assert np.array_equal(g.field("flags"), o.field("flags"))
    sol = o.field("flags") == O.SOLID
    assert np.array_equal(g.field("owner")[sol], o.field("owner")[sol])
    fo = o.field("pdf")
    check("pdf", float(np.abs(g.field("pdf") - fo).max() / np.abs(fo).max()), TOL)
    for dom in doms:
        dom.close()


@pytest.mark.parametrize("storage", [0, 1])
def test_density_out_of_range_is_reported(storage):
    """The sampled density check of lbmdem_sync: a fluid at rho = 1.6 (set
    from the host, a state no stable run reaches) is reported as
    LBMDEM_EUNSTABLE and fails the domain; the same field at rho = 1.4 and a
    domain beside the failed one stay healthy."""
    from paper_2003_01490_amd import lbmdem as L

    n = (24, 20, 18)
    _case(f"density range check, storage {storage}")
    wl = W.Workload("rho", W.base_params(nx=n[0], ny=n[1], nz=n[2], nu=0.05, max_spheres=1),
                    np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), 0)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None, None, None]
    ok, bad = gpu_domain(wl, storage=storage), gpu_domain(wl, storage=storage)
    ok.set_pdf(np.broadcast_to(1.4 * w, (19,) + n[::-1]))
    bad.set_pdf(np.broadcast_to(1.6 * w, (19,) + n[::-1]))
    for d in (ok, bad):
        d.step(1)
    ok.sync()
    with pytest.raises(L.LbmdemError) as e:
        bad.sync()
    assert e.value.code == L.EUNSTABLE and "density" in str(e.value)
    with pytest.raises(L.LbmdemError) as e:
        bad.step(1)
    assert e.value.code == L.ESTATE
    ok.step(3)
    ok.sync()
    for d in (ok, bad):
        d.close()


@pytest.mark.parametrize("wlname,mk", [("contact", 0), ("dense", 0), ("dense", 3)])
def test_step_graph_equals_direct_launches(wlname, mk):
    """A domain stepped by replaying one captured step graph ends bit for bit
    as one stepped by direct launches: through a wall contact (one sphere,
    prescribed-free DEM, overlap of sweep and DEM on two streams) and in the
    dense 96^3 suspension (many-sphere DEM chain; the fused step too), over
    several replays with host reads between them, and across a re-capture
    after a sphere is added."""
    import torch
    from paper_2003_01490_amd import lbmdem as L

    wl = W.contact_32(0) if wlname == "contact" else W.dense(0, n=96, count=156)
    _case(f"step graph against direct launches: {wlname}, map_kernel {mk}")
    stream = torch.cuda.Stream()
    extra = max(len(wl.R), 1) + 1
    a = gpu_domain(wl, storage=1, stream=stream, map_kernel=mk, max_spheres=extra)
    b = gpu_domain(wl, storage=1, stream=stream, map_kernel=mk, max_spheres=extra)
    b.set_graph(True)
    for chunk in (1, 7, 30):
        a.step(chunk)
        b.step(chunk)
        sa, sb = a.spheres(), b.spheres()
        assert all(np.array_equal(sa[k], sb[k]) for k in sa), f"spheres differ after a chunk of {chunk}"
    R = 2.0
    placed = None
    for fx in np.linspace(0.1, 0.9, 9):
        for fy in np.linspace(0.1, 0.9, 9):
            x = np.array([[wl.params["nx"] * fx + 0.25, wl.params["ny"] * fy, wl.params["nz"] - 2.5 - R]])
            try:
                a.add_spheres(x, np.array([R]), np.array([2.0]))
            except L.LbmdemError as e:
                assert e.code == L.EOVERLAP
                continue
            placed = x
            break
        if placed is not None:
            break
    assert placed is not None, "no free place for the added sphere"
    b.add_spheres(placed, np.array([R]), np.array([2.0]))
    a.step(12)
    b.step(12)
    sa, sb = a.spheres(), b.spheres()
    assert all(np.array_equal(sa[k], sb[k]) for k in sa), "spheres differ after the re-capture"
    assert np.array_equal(a.field("pdf"), b.field("pdf"))
    for d in (a, b):
        d.close()
