"""Pins of the oracle's discrete element part (Secs. 3.1, 4.1, App. B).

- velocity-Verlet (Eqs. velocity_verlet_1/2) integrates a constant force exactly;
- the linear spring-dashpot with k_n, d_n of Eq. (normalDEMparameters) gives a
  dry contact of duration T_c and restitution e_dry (closed form of the damped
  oscillator, which the paper uses to define the parameters);
- dry oblique impact in gross sliding: rigid-body impulse theory gives
  Psi_out = Psi_in - 3.5 mu (1 + e); this also fixes the order of the cross
  product in the surface velocity (Sec. 4.5: u_t = u_p,t - R w_y);
- lubrication: the kappa_r -> infinity limit of the sphere-sphere terms equals
  the sphere-wall terms; pair forces are antisymmetric; the force-rotation and
  torque-translation couplings obey reciprocity; the step function and the
  minimal gap behave as Eqs. (lubrication_correction_step_function/gap_size) say;
- parameter relations against the numbers the paper prints (tests/golden).
"""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_velocity_verlet_constant_force_is_exact():
    g = np.array([1e-5, -2e-5, 3e-6])
    cfg = O.make_config(nx=40, ny=40, nz=40, walls=(0, 0, 0), gravity=g, n_sub=7, max_spheres=1)
    d = O.RefDomain(cfg)
    x0, u0 = np.array([10.3, 20.1, 5.7]), np.array([0.01, 0.002, -0.003])
    R, rho = 2.0, 3.0
    sid = d.add_sphere(x0, R, rho, u=u0)
    acc = g * (rho - 1.0) / rho  # V (rho_p - rho_f) g / (rho_p V)
    for _ in range(50):
        d.dem_step()
    t = 50.0
    s = d.sphere(sid)
    np.testing.assert_allclose(s["u"], u0 + acc * t, rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(s["x"], x0 + u0 * t + 0.5 * acc * t * t, rtol=1e-12)


def _dry_wall_impact(e, tc, n_sub, u_in, R=5.0, mu=0.0, nu_p=0.25, lub=0):
    n = int(4 * R + 20)
    cfg = O.make_config(nx=n, ny=n, nz=n, walls=(0, 0, 1), e_dry=e, tc=tc, n_sub=n_sub,
                        friction=mu, poisson_ratio=nu_p, lub_mask=lub, max_spheres=1)
    d = O.RefDomain(cfg)
    z0 = 1.0 + R + 0.3
    sid = d.add_sphere((n / 2, n / 2, z0), R, 2.0, u=u_in)
    t, t_start, t_end = 0, None, None
    pre = post = None
    while t < 100000:
        s = d.sphere(sid)
        gap = s["x"][2] - 1.0 - R
        d.dem_step()
        t += 1
        s2 = d.sphere(sid)
        gap2 = s2["x"][2] - 1.0 - R
        if t_start is None and gap2 < 0:
            # linear interpolation of the crossing inside the step
            t_start = t - 1 + gap / (gap - gap2)
            pre = s
        if t_start is not None and t_end is None and gap2 >= 0 and gap < 0:
            t_end = t - 1 + gap / (gap - gap2)
            post = s2
            break
    return t_start, t_end, pre, post


@pytest.mark.parametrize("e", [0.97, 0.83, 0.5])
def test_dry_normal_collision_duration_and_restitution(e):
    tc = 400.0
    ts, te, pre, post = _dry_wall_impact(e, tc, 1, (0, 0, -0.01))
    assert abs((te - ts) - tc) < 1.0
    e_meas = -post["u"][2] / pre["u"][2]
    assert abs(e_meas - e) < 2e-3


def test_collision_time_guideline_against_printed_values():
    g = GOLD["collision_time_guideline"]
    cfg = O.make_config(tc=-1.0)
    for D, obs in zip(g["D"], g["Tc_observed"]):
        assert abs(O.collision_time(cfg, D) / obs - 1) < 1e-3


def test_min_gap_relation_against_table():
    g = GOLD["min_gap_relation"]
    cfg = O.make_config(dmin=-1.0)
    for D, best, printed in zip(g["D"], g["best_fit"], g["relation_printed"]):
        v = O.min_gap(cfg, D / 2)
        assert round(v, 3) == pytest.approx(printed, abs=1e-12)
        assert abs(v - best) < 1.5e-3


def test_resolution_estimate():
    """Sec. 4.4.4: the minimal gap reaches the normal cut-off near R_p = 90."""
    cfg = O.make_config(dmin=-1.0)
    R = [r for r in np.linspace(50, 150, 2001) if O.min_gap(cfg, r) >= 2 / 3][0]
    assert abs(R - GOLD["resolution_estimate"]["R_p"]) < 3


@pytest.mark.parametrize("psi_in", [3.0, 6.0])
def test_dry_oblique_sliding_impact(psi_in):
    """TD case of Table (obliqueCollision): e 0.83, nu_p 0.22, mu 0.12.  The
    overlap is kept small against R so that the rigid-contact impulse theory
    applies (the contact point sits at R + delta/2 from the centre)."""
    e, mu, nu_p = 0.83, 0.12, 0.22
    un = -0.01
    R = 20.0
    ts, te, pre, post = _dry_wall_impact(e, 60.0, 20, (psi_in * -un, 0, un), R=R, mu=mu,
                                         nu_p=nu_p)
    psi_out = -(post["u"][0] - R * post["w"][1]) / pre["u"][2]
    expect = psi_in - 3.5 * mu * (1 + e)
    assert abs(psi_out - expect) < 3e-3 * psi_in


def test_lubrication_wall_is_large_radius_limit_of_pair():
    cfg = O.make_config(nx=50, ny=50, nz=50, walls=(0, 0, 1), dmin=0.0)
    rng = np.random.default_rng(0)
    Ri = 3.0
    for _ in range(5):
        gap = rng.uniform(0.05, 0.45)
        xi = np.array([20.0, 21.0, 1.0 + Ri + gap])
        ui, wi = rng.standard_normal(3) * 0.01, rng.standard_normal(3) * 0.001
        Fw, Tw = O.lubrication(cfg, xi, ui, wi, Ri, wall=4)
        errs = []
        for Rj in (1e4, 1e5, 1e6):
            xj = np.array([20.0, 21.0, 1.0 - Rj])
            Fp, Tp = O.lubrication(cfg, xi, ui, wi, Ri, xj=xj, Rj=Rj, wall=-1)
            errs.append(max(np.linalg.norm(Fp - Fw) / np.linalg.norm(Fw),
                            np.linalg.norm(Tp - Tw) / np.linalg.norm(Tw)))
        # O(1/kappa_r) convergence to the wall terms
        assert errs[-1] < 1e-4
        assert errs[0] / errs[1] > 5 and errs[1] / errs[2] > 5
        assert np.abs(Fw).max() > 0 and np.abs(Tw).max() > 0


def test_lubrication_pair_forces_are_antisymmetric():
    cfg = O.make_config(dmin=0.0)
    rng = np.random.default_rng(1)
    for _ in range(5):
        Ri, Rj = rng.uniform(2, 6, 2)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        gap = rng.uniform(0.05, 0.45)
        xj = np.array([10.0, 10.0, 10.0])
        xi = xj + (Ri + Rj + gap) * n
        ui, uj, wi, wj = (rng.standard_normal(3) * 0.01 for _ in range(4))
        Fi, _ = O.lubrication(cfg, xi, ui, wi, Ri, xj=xj, uj=uj, wj=wj, Rj=Rj)
        Fj, _ = O.lubrication(cfg, xj, uj, wj, Rj, xj=xi, uj=ui, wj=wi, Rj=Ri)
        np.testing.assert_allclose(Fi, -Fj, rtol=1e-12, atol=1e-18)


def _jac(fun, n=3, h=1.0):
    cols = []
    for b in range(n):
        e = np.zeros(n)
        e[b] = h
        cols.append(fun(e) - fun(-e))
    return np.array(cols).T / (2 * h)


@pytest.mark.parametrize("wall", [True, False])
def test_lubrication_reciprocity(wall):
    """Force from rotation and torque from translation are transposes of each
    other (Lorentz reciprocity of the Stokes resistance)."""
    cfg = O.make_config(nx=50, ny=50, nz=50, walls=(0, 0, 1), dmin=0.0, lub_mask=6)
    R = 4.0
    gap = 0.2
    xi = np.array([20.0, 20.0, 1.0 + R + gap])
    if wall:
        kw = dict(wall=4)
    else:
        kw = dict(xj=xi - np.array([0.0, 0.0, 2 * R + gap]), Rj=R, wall=-1)
    dFdw = _jac(lambda wv: O.lubrication(cfg, xi, np.zeros(3), wv, R, **kw)[0])
    dTdu = _jac(lambda uv: O.lubrication(cfg, xi, uv, np.zeros(3), R, **kw)[1])
    assert np.abs(dFdw).max() > 0
    np.testing.assert_allclose(dTdu, dFdw.T, rtol=1e-12, atol=1e-16)


def test_lubrication_step_function_and_min_gap():
    cfg = O.make_config(nx=50, ny=50, nz=50, walls=(0, 0, 1), dmin=0.01)
    R = 4.0
    u = np.array([0.003, -0.002, -0.01])
    w = np.array([0.001, 0.002, 0.0])
    def F(gap):
        return O.lubrication(cfg, [20, 20, 1 + R + gap], u, w, R, wall=4)
    for gap in (-0.1, 0.0, 2 / 3 + 1e-9, 1.0):
        f, t = F(gap)
        if gap >= 0.5:
            assert np.all(f[:2] == 0) and np.all(t == 0)
        if gap <= 0 or gap >= 2 / 3:
            assert np.all(f == 0) and np.all(t == 0)
    np.testing.assert_array_equal(F(0.004)[0], F(0.01)[0])
    assert np.all(np.abs(F(0.02)[0]) < np.abs(F(0.01)[0]))
    # normal only between the tangential and normal cut-offs
    f, t = F(0.6)
    assert f[2] != 0 and f[0] == 0 and np.all(t == 0)
    # sphere-wall normal: -6 pi mu R^2 (1/d - 1/cut) u_n with kappa -> inf
    f, _ = O.lubrication(O.make_config(nx=50, ny=50, nz=50, walls=(0, 0, 1), dmin=0.01, lub_mask=1),
                         [20, 20, 1 + R + 0.2], u, w, R, wall=4)
    assert f[2] == pytest.approx(-6 * np.pi * cfg.nu * R * R * (1 / 0.2 - 1.5) * u[2], rel=1e-14)


def test_tangential_spring_reset_at_separation_and_sticking():
    """Low-angle impact sticks (the tangential spring stores energy and the
    contact point reverses); the history is cleared after separation."""
    ts, te, pre, post = _dry_wall_impact(0.9, 300.0, 1, (0.002, 0, -0.01), mu=0.5, nu_p=0.3)
    R = 5.0
    ucp_out = post["u"][0] - R * post["w"][1]
    assert ucp_out < 0.002 * 0.5  # sticking removes most of the slip
    assert te - ts > 0


def test_prescribed_ramp_and_release_at_the_wall_ahead():
    """Eq. (artificial_acceleration): u = u_s (1 - exp(-c_acc t / t_St)) with t
    advanced per sub-step; the ramp is switched off once the gap to the wall
    the sphere approaches (Sec. 4.4.2: the bottom wall for a settling sphere)
    falls below the release gap.  A start closer than that to the wall behind
    it must not release the sphere."""
    R, n = 2.0, 24
    cfg = O.make_config(nx=n, ny=n, nz=n, walls=(0, 0, 1), n_sub=10, max_spheres=1,
                        gravity=(0.0, 0.0, -1e-4))
    d = O.RefDomain(cfg)
    z0 = (n - 1.0) - R - 1.0  # gap 1 to the top wall plane, behind the sphere
    sid = d.add_sphere((n / 2, n / 2, z0), R, 3.0)
    u_s, c_acc, t_st, gap_r = 0.5, 10.0, 40.0, 4.0
    d.set_mode(sid, O.MODE_PRESCRIBED, (0.0, 0.0, -u_s), c_acc, t_st, gap_r)
    released_at = None
    for k in range(1, 60):
        d.dem_step()
        s = d.sphere(sid)
        gap_bottom = s["x"][2] - 1.0 - R
        if released_at is None and s["mode"] == O.MODE_FREE:
            released_at = (k, gap_bottom)
            break
        assert s["mode"] == O.MODE_PRESCRIBED
        assert gap_bottom >= gap_r - u_s / cfg.n_sub  # released within one sub-step of the gap
        assert s["u"][2] == pytest.approx(-u_s * (1.0 - np.exp(-c_acc * k / t_st)), rel=1e-12)
    assert released_at is not None, "never released above the bottom wall"
    assert released_at[1] < gap_r


LUB = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lubrication_coefficients.json")))


def _frac(s):
    a, _, b = s.partition("/")
    return float(a) / float(b or 1)


def _perp_frame(rng):
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    t = np.cross(n, rng.standard_normal(3))
    t /= np.linalg.norm(t)
    return n, t, np.cross(n, t)


@pytest.mark.parametrize("case", range(len(LUB["cases"]) + 1))
def test_lubrication_coefficients_at_fixed_radius_ratios(case):
    """D3: the pair corrections of Sec. 3.1 at kappa_r = 1, 2 and 1/2 (and the
    sphere-wall limit) against coefficients worked out by hand from the
    printed expressions (tests/golden/lubrication_coefficients.json), term by
    term: a normal approach gives only the normal force, a tangential
    translation only the tt force and torque, rotations only the tr force and
    torque, with the rotation about the line of centres dropped from the
    torque."""
    wall = case == len(LUB["cases"])
    cf = LUB["wall"] if wall else LUB["cases"][case]
    cut_n, cut_t, cut_r = 2.0 / 3.0, 0.5, 0.45
    cfg = O.make_config(nx=60, ny=60, nz=60, walls=(0, 0, 1), nu=0.07, dmin=0.001,
                        cut_n=cut_n, cut_tt=cut_t, cut_tr=cut_r)
    mu = cfg.nu
    rng = np.random.default_rng(11 + case)
    Ri, gap = 3.0, 0.2
    if wall:
        n, t, s = np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
        xi = np.array([30.0, 30.0, 1.0 + Ri + gap])
        kw = dict(wall=4)
    else:
        n, t, s = _perp_frame(rng)
        Rj = Ri * _frac(cf["kappa"])
        xj = np.array([30.0, 30.0, 30.0])
        xi = xj + (Ri + Rj + gap) * n
        kw = dict(xj=xj, Rj=Rj, wall=-1)
    z = np.zeros(3)
    Ln, Lt, Lr = 1.0 / gap - 1.0 / cut_n, np.log(gap / cut_t), np.log(gap / cut_r)

    def lub(ui=z, wi=z, uj=z, wj=z):
        return O.lubrication(cfg, xi, ui, wi, Ri, uj=uj, wj=wj, **kw)

    # normal approach
    a = 0.013
    F, T = lub(ui=a * n)
    np.testing.assert_allclose(F, -6 * np.pi * mu * Ri ** 2 * _frac(cf["normal"]) * Ln * a * n, rtol=1e-13, atol=1e-18)
    assert np.abs(T).max() < 1e-15  # u_ij x n vanishes up to rounding
    # tangential translation (relative velocity of the pair)
    b = 0.021
    uj = z if wall else 0.5 * b * t
    F, T = lub(ui=1.5 * b * t, uj=uj)
    urel = 1.5 * b * t - uj
    np.testing.assert_allclose(F, 6 * np.pi * mu * Ri * _frac(cf["tt_force"]) * Lt * urel, rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(T, 8 * np.pi * mu * Ri ** 2 * _frac(cf["tt_torque"]) * Lt * np.cross(urel, n),
                               rtol=1e-13, atol=1e-18)
    # rotations, including a component about the line of centres
    wi = 0.004 * t - 0.003 * s + 0.002 * n
    wj = z if wall else -0.001 * t + 0.005 * s - 0.003 * n
    F, T = lub(wi=wi, wj=wj)
    va, vb = (_frac(v) for v in cf["tr_force_vector"])
    expF = -6 * np.pi * mu * Ri ** 2 * _frac(cf["tr_force"]) * Lr * np.cross(va * wi + vb * wj, n)
    av = wi + _frac(cf["tr_torque_wj"]) * wj
    expT = 8 * np.pi * mu * Ri ** 3 * _frac(cf["tr_torque"]) * Lr * (av - av.dot(n) * n)
    np.testing.assert_allclose(F, expF, rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(T, expT, rtol=1e-13, atol=1e-18)


def test_tangential_stick_branch_rolls_without_slipping():
    """Stick branch of the tangential contact (Sec. 4.1.2).  A sphere resting on
    the wall under gravity is given a tangential velocity v0; with a large
    friction coefficient the contact sticks.  While it sticks, the contact-point
    velocity v = u_x - R_c w_y (R_c = R + delta/2 the arm to the contact point)
    obeys m_t dv/dt = -k_t s - d_t v, ds/dt = v, with k_t = kappa_p k_n and
    d_t = sqrt(kappa_p) d_n (Eq. tangentialCollisionParameters, k_n and d_n of
    Eq. normalDEMparameters) and the effective mass m_t = 1 / (1/m + R_c^2 / I):
    a damped oscillator from v(0) = v0, s(0) = 0.  The tangential impulse acts on
    u and w with the same arm, so m u R_c + I w_y is conserved and the sphere
    ends rolling at u = v0 / (1 + I / (m R_c^2)) (5/7 v0 for R_c = R)."""
    R, rho, e, Tc, nu_p, g = 4.0, 2.0, 0.3, 40.0, 0.23, 1e-4
    n = 40
    cfg = O.make_config(nx=n, ny=n, nz=n, walls=(0, 0, 1), e_dry=e, tc=Tc, n_sub=10, friction=100.0,
                        poisson_ratio=nu_p, lub_mask=0, gravity=(0.0, 0.0, -g), max_spheres=1)
    d = O.RefDomain(cfg)
    sid = d.add_sphere((n / 2, n / 2, 1.0 + R), R, rho)     # touching the wall plane
    for _ in range(2000):                                     # settle onto the spring
        d.dem_step()
    s = d.sphere(sid)
    assert abs(s["u"][2]) < 1e-12 and s["F_col"][2] > 0
    delta = s["x"][2] - 1.0 - R
    Rc = R + 0.5 * delta
    m = rho * 4.0 / 3.0 * np.pi * R ** 3
    I = 0.4 * m * R * R
    kn = m * (np.pi ** 2 + np.log(e) ** 2) / Tc ** 2
    dn = -2.0 * m * np.log(e) / Tc
    kp = 2.0 * (1.0 - nu_p) / (2.0 - nu_p)
    mt = 1.0 / (1.0 / m + Rc * Rc / I)
    w0, gam = np.sqrt(kp * kn / mt), np.sqrt(kp) * dn / (2.0 * mt)
    wd = np.sqrt(w0 * w0 - gam * gam)
    v0 = 1e-3
    d.update_sphere(sid, u=(v0, 0.0, 0.0), w=(0.0, 0.0, 0.0))
    err = 0.0
    for k in range(1, 61):                                    # about one oscillation period
        d.dem_step()
        s = d.sphere(sid)
        v = s["u"][0] - Rc * s["w"][1]
        expect = v0 * np.exp(-gam * k) * (np.cos(wd * k) - gam / wd * np.sin(wd * k))
        err = max(err, abs(v - expect))
    assert err < 0.01 * v0
    for _ in range(600):
        d.dem_step()
    s = d.sphere(sid)
    assert abs(s["u"][0] - Rc * s["w"][1]) < 1e-9 * v0
    assert s["u"][0] == pytest.approx(v0 / (1.0 + I / (m * Rc * Rc)), rel=1e-6)
