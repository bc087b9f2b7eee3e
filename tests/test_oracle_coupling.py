"""Pins of the oracle's fluid-particle coupling (Sec. 2.2).

- mapping: cell centres inside (or on) a sphere are solid; exact integer
  arithmetic on dyadic positions decides every cell, shells included;
- momentum-exchange closure: in a resting fluid the force and torque on any
  mapped sphere vanish, also when links are missing at a wall or at another
  sphere, which is what the 2 w_q c_q compensation is for;
- Galilean invariance of the coupled step: a sphere translating with a uniform
  flow leaves the uniform equilibrium untouched, through CLI, momentum
  exchange, re-mapping and reconstruction (Eq. PDF_reconstruction);
- reconstruction at rest gives w_q exactly;
- momentum balance: at steady state the resolved force on a fixed sphere equals
  the body-force input into the fluid;
- mirror symmetry of a settling sphere on a lattice symmetry plane.
"""
import numpy as np
import pytest

import oracle as O
from harness import exact_tie_counts as _tie_counts


def _exact_flags(n, walls, spheres, delta_ab=2.0, scale=1 << 11):
    """Integer re-statement: positions are multiples of 2^-10, so with the
    factor 2^11 all cell-centre offsets are integers."""
    nx, ny, nz = n
    code = np.zeros((nz, ny, nx), dtype=np.uint8)
    owner = -np.ones((nz, ny, nx), dtype=np.int64)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                ijk = (i, j, k)
                if any(walls[a] and ijk[a] in (0, n[a] - 1) for a in range(3)):
                    code[k, j, i] = O.WALL
                    continue
                shell = False
                own = -1
                for sid, (x, R) in enumerate(spheres):
                    d2 = 0
                    for a in range(3):
                        v = (2 * ijk[a] + 1) * (scale // 2) - int(round(x[a] * scale))
                        if not walls[a]:
                            L = n[a] * scale
                            if 2 * v > L:
                                v -= L
                            elif 2 * v < -L:
                                v += L
                        d2 += v * v
                    Ri = int(round(R * scale))
                    Rs = int(round((R + delta_ab) * scale))
                    if d2 <= Ri * Ri and own < 0:
                        own = sid
                    if d2 <= Rs * Rs:
                        shell = True
                if own >= 0:
                    code[k, j, i] = O.SOLID
                    owner[k, j, i] = own
                else:
                    code[k, j, i] = O.SHELL if shell else O.FLUID
    return code, owner


# Centres on cell centres with Pythagorean radii: offsets such as (3, 4, 0) and
# (5, 0, 0) put cell centres exactly on the R = 5 surface, (2, 3, 6) and
# (7, 0, 0) exactly on the R + delta_aB = 7 shell surface, and the two R = 5
# spheres touch at one cell centre, which lies on both surfaces.
TIE_LATTICE = (26, 21, 22)
TIE_SPHERES = [((10.5, 10.5, 10.5), 5.0), ((20.5, 10.5, 10.5), 5.0), ((5.5, 17.5, 16.5), 3.0)]


def test_mapping_ties_closed_ball_and_lowest_id():
    """Sec. 2.2: a cell is solid when its centre is contained in the particle,
    read as the closed ball (d^2 <= R^2); the TRT+aB shell is closed as well;
    a cell centre on two spheres belongs to the lower id."""
    n, walls = TIE_LATTICE, (0, 0, 1)
    cfg = O.make_config(nx=n[0], ny=n[1], nz=n[2], walls=walls, max_spheres=3)
    d = O.RefDomain(cfg)
    for x, R in TIE_SPHERES:
        d.add_sphere(x, R, 2.0)
    on_surface, on_shell, shared = _tie_counts(n, walls, TIE_SPHERES)
    assert on_surface >= 60 and on_shell >= 100 and shared == 1
    code, owner = d.flags()
    ecode, eowner = _exact_flags(n, walls, TIE_SPHERES)
    assert np.array_equal(code, ecode)
    sol = ecode == O.SOLID
    assert np.array_equal(owner[sol], eowner[sol])
    # surface cells are solid (closed ball), shell-surface cells are shell
    assert code[10, 14, 13] == O.SOLID and code[10, 10, 5] == O.SOLID     # (3, 4, 0) and (-5, 0, 0)
    assert code[10, 10, 3] == O.SHELL and code[16, 13, 12] == O.SHELL     # (-7, 0, 0) and (2, 3, 6)
    assert code[10, 10, 2] == O.FLUID                                      # just outside the shell
    # the touching cell (15, 10, 10) is on both surfaces: the lower id owns it
    assert code[10, 10, 15] == O.SOLID and owner[10, 10, 15] == 0


@pytest.mark.parametrize("seed", range(4))
def test_mapping_matches_exact_integer_classification(seed):
    rng = np.random.default_rng(seed)
    n = (12, 11, 14)
    walls = (0, 0, 1)
    cfg = O.make_config(nx=n[0], ny=n[1], nz=n[2], walls=walls, max_spheres=3)
    d = O.RefDomain(cfg)
    spheres = []
    # random dyadic placements (ties are covered by the placements above)
    for sid in range(3):
        for _ in range(200):
            R = rng.integers(1 * 1024, 3 * 1024) / 1024.0
            x = [rng.integers(0, n[a] * 1024) / 1024.0 for a in range(3)]
            if d.try_add_sphere(x, R, 2.0) >= 0:
                spheres.append((x, R))
                break
    code, owner = d.flags()
    ecode, eowner = _exact_flags(n, walls, spheres)
    assert np.array_equal(code, ecode)
    sol = ecode == O.SOLID
    assert np.array_equal(owner[sol], eowner[sol])
    assert (code == O.SOLID).sum() > 0


def test_mapping_is_mirror_symmetric_on_symmetry_points():
    cfg = O.make_config(nx=16, ny=16, nz=18, walls=(0, 0, 1), max_spheres=1)
    d = O.RefDomain(cfg)
    d.add_sphere((8.0, 8.0, 9.0), 3.7, 2.0)
    code, _ = d.flags()
    assert np.array_equal(code, code[:, :, ::-1])
    assert np.array_equal(code, code[:, ::-1, :])
    assert np.array_equal(code, code[::-1, :, :])
    assert np.array_equal(code, code.transpose(0, 2, 1))


def _count_missing_links(code, owner, sid, walls):
    c, _, _ = O.lattice()
    nz, ny, nx = code.shape
    cnt = 0
    for k, j, i in zip(*np.nonzero((code == O.SOLID) & (owner == sid))):
        for q in range(1, 19):
            zi, zj, zk = (i - c[q, 0]) % nx, (j - c[q, 1]) % ny, (k - c[q, 2]) % nz
            cz = code[zk, zj, zi]
            if cz == O.WALL or (cz == O.SOLID and owner[zk, zj, zi] != sid):
                cnt += 1
    return cnt


@pytest.mark.parametrize("boundary", [0, 1])
def test_momentum_exchange_closure_in_resting_fluid(boundary):
    """M1: F = T = 0 at rest, with missing links at the wall and between spheres."""
    cfg = O.make_config(nx=20, ny=16, nz=16, walls=(0, 0, 1), boundary=boundary, max_spheres=3)
    d = O.RefDomain(cfg)
    d.add_sphere((6.3, 7.7, 1.0 + 3.6 + 0.15), 3.6, 2.0)    # 0.15 above the wall plane
    d.add_sphere((6.3 + 7.2 + 0.3, 7.9, 8.4), 3.6, 2.0)     # apart
    for sid in range(d.num_spheres()):
        d.set_mode(sid, O.MODE_FIXED)
    code, owner = d.flags()
    assert _count_missing_links(code, owner, 0, (0, 0, 1)) > 0
    d.step(1)
    for sid in range(d.num_spheres()):
        s = d.sphere(sid)
        assert np.abs(s["F_raw"]).max() < 1e-14
        assert np.abs(s["T_raw"]).max() < 1e-13


def test_momentum_exchange_closure_between_close_spheres():
    cfg = O.make_config(nx=24, ny=14, nz=14, walls=(0, 0, 0), max_spheres=2)
    d = O.RefDomain(cfg)
    d.add_sphere((7.31, 7.02, 6.87), 3.4, 2.0)
    d.add_sphere((7.31 + 6.8 + 0.12, 7.02, 6.87), 3.4, 2.0)
    for sid in range(2):
        d.set_mode(sid, O.MODE_FIXED)
    code, owner = d.flags()
    assert _count_missing_links(code, owner, 0, (0, 0, 0)) > 0
    d.step(1)
    for sid in range(2):
        s = d.sphere(sid)
        assert np.abs(s["F_raw"]).max() < 1e-14
        assert np.abs(s["T_raw"]).max() < 1e-13


@pytest.mark.parametrize("boundary", [0, 1])
def test_galilean_invariance_of_comoving_sphere(boundary):
    """A sphere moving with a uniform flow: the field stays f^eq(1, u0) exactly,
    the resolved force is zero, and uncovered cells are reconstructed to it."""
    n = 14
    u0 = np.array([0.031, -0.017, 0.011])
    cfg = O.make_config(nx=n, ny=n, nz=n, walls=(0, 0, 0), boundary=boundary, nu=0.04,
                        max_spheres=1)
    d = O.RefDomain(cfg)
    c, w, _ = O.lattice()
    feq = O.equilibrium(1.0, u0)
    d.set_pdf(np.tile(feq[:, None, None, None], (1, n, n, n)))
    x = np.array([6.9, 7.3, 7.05])
    sid = d.add_sphere(x, 3.3, 2.0, u=u0)
    d.set_mode(sid, O.MODE_FIXED)
    d.update_sphere(sid, u=u0)
    recon = 0
    for step in range(30):
        d.step(1)
        code0, _ = d.flags()
        x = x + u0 * 7.0  # move fast so cells get uncovered every step
        x = np.mod(x, n)
        d.update_sphere(sid, x=x)
        code1, _ = d.flags()
        recon += int(((code0 == O.SOLID) & (code1 != O.SOLID)).sum())
        s = d.sphere(sid)
        assert np.abs(s["F_raw"]).max() < 1e-13
        pdf = d.field("pdf")
        fl = code1 <= O.SHELL
        dev = np.abs(pdf[:, fl] - feq[:, None]).max()
        assert dev < 1e-14, (step, dev)
    assert recon > 20


def test_reconstruction_at_rest_gives_weights():
    n = 12
    cfg = O.make_config(nx=n, ny=n, nz=n, walls=(0, 0, 0), max_spheres=1)
    d = O.RefDomain(cfg)
    _, w, _ = O.lattice()
    sid = d.add_sphere((6.1, 5.9, 6.3), 3.1, 2.0)
    d.set_mode(sid, O.MODE_FIXED)
    code0, _ = d.flags()
    d.update_sphere(sid, x=(6.9, 5.2, 6.8))
    code1, _ = d.flags()
    newly = (code0 == O.SOLID) & (code1 <= O.SHELL)
    assert newly.sum() > 5
    pdf = d.field("pdf")
    assert np.abs(pdf[:, newly] - w[:, None]).max() < 1e-16


def _designed_linear_field(n, x0, rho_grad, u0, G):
    """Equilibrium distributions of a density and a velocity that are linear in
    the cell-centre position: rho = 1 + a.(x - x0), u = u0 + G (x - x0)."""
    c, w, _ = O.lattice()
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.stack([i + 0.5 - x0[0], j + 0.5 - x0[1], k + 0.5 - x0[2]])
    rho = 1.0 + np.einsum("a,a...->...", rho_grad, r)
    u = np.asarray(u0)[:, None, None, None] + np.einsum("ab,b...->a...", G, r)
    cu = np.einsum("qa,a...->q...", c.astype(float), u)
    usq = (u * u).sum(0)
    return w[:, None, None, None] * (rho + 3 * cu + 4.5 * cu * cu - 1.5 * usq)


def test_reconstruction_gradient_term():
    """Eq. (PDF_reconstruction) with a non-zero velocity gradient.  The fluid
    around a sphere carries a density and a velocity linear in space (central
    differences of it are exact); the sphere is moved so that cells are
    uncovered.  Each rebuilt cell must (a) have the moments the formula is
    built to have: sum f = rho_bar (mean density of the neighbours fluid before
    and after), sum f c = rho_bar u_t (u_t the rigid-body velocity there) and
    sum f c c = rho_bar c_s^2 I + rho_bar u_t u_t - (rho_bar c_s^2 / s_nu)
    (G + G^T) (the Chapman-Enskog form of the viscous stress), with G from
    central differences of the neighbour velocities, or one-sided ones
    against u_t where a neighbour is missing, as Sec. 2.2 states; and (b)
    f_q / w_q must be a polynomial of degree two in c_q (a second-order
    Hermite form): together these fix all 19 values."""
    n = (20, 20, 20)
    cfg = O.make_config(nx=n[0], ny=n[1], nz=n[2], walls=(0, 0, 1), nu=0.03, max_spheres=1)
    s_nu = O.rates(cfg)[0]
    c, w, _ = O.lattice()
    cf = c.astype(float)
    d = O.RefDomain(cfg)
    x_old = np.array([9.7, 10.2, 10.1])
    sid = d.add_sphere(x_old, 3.3, 2.0)
    d.set_mode(sid, O.MODE_FIXED)
    G = np.array([[2e-3, -1e-3, 5e-4], [1.5e-3, -4e-4, 2e-3], [-7e-4, 1e-3, 1.2e-3]])
    f = _designed_linear_field(n, x_old, np.array([1e-3, -5e-4, 2e-4]), (0.01, -0.005, 0.002), G)
    d.set_pdf(f)
    code0, _ = d.flags()
    x_new = x_old + np.array([0.8, -0.6, 0.5])
    u_s, w_s = np.array([0.004, -0.002, 0.003]), np.array([1e-3, -2e-3, 5e-4])
    d.update_sphere(sid, x=x_new, u=u_s, w=w_s)
    code1, _ = d.flags()
    pdf = d.field("pdf")
    fluid_both = (code0 <= O.SHELL) & (code1 <= O.SHELL)
    rebuilt = np.argwhere((code0 == O.SOLID) & (code1 <= O.SHELL))
    assert len(rebuilt) > 10
    rho_f = f.sum(0)
    j_f = np.einsum("qa,q...->a...", cf, f)
    kinds = set()
    grad_term = 0.0
    # quadratic monomials of c: 1, c_a, c_a c_b (a <= b) -> 10 basis columns
    basis = np.column_stack([np.ones(19)] + [cf[:, a] for a in range(3)] +
                            [cf[:, a] * cf[:, b] for a in range(3) for b in range(a, 3)])
    for k, j, i in rebuilt:
        def nb(di, dj, dk):
            return (k + dk) % n[2], (j + dj) % n[1], (i + di) % n[0]
        valid = [nb(*c[q]) for q in range(1, 19) if fluid_both[nb(*c[q])]]
        rb = np.mean([rho_f[v] for v in valid]) if valid else 1.0
        r = np.array([i + 0.5, j + 0.5, k + 0.5]) - x_new
        ut = u_s + np.cross(w_s, r)
        Gm = np.zeros((3, 3))  # Gm[a, b] = d u_a / d x_b
        for b in range(3):
            e = np.zeros(3, dtype=int)
            e[b] = 1
            p, m = nb(*e), nb(*(-e))
            vp, vm = fluid_both[p], fluid_both[m]
            if vp and vm:
                Gm[:, b] = 0.5 * (j_f[(slice(None),) + p] - j_f[(slice(None),) + m])
                kinds.add("central")
            elif vp:
                Gm[:, b] = j_f[(slice(None),) + p] - ut
                kinds.add("one-sided")
            elif vm:
                Gm[:, b] = ut - j_f[(slice(None),) + m]
                kinds.add("one-sided")
        fr = pdf[:, k, j, i]
        S = Gm + Gm.T
        assert abs(fr.sum() - rb) < 1e-15
        np.testing.assert_allclose(cf.T @ fr, rb * ut, rtol=0, atol=1e-16)
        second = np.einsum("q,qa,qb->ab", fr, cf, cf)
        expect2 = rb / 3.0 * np.eye(3) + rb * np.outer(ut, ut) - rb / (3.0 * s_nu) * S
        np.testing.assert_allclose(second, expect2, rtol=0, atol=2e-16)
        coef, res, *_ = np.linalg.lstsq(basis, fr / w, rcond=None)
        assert np.abs(basis @ coef - fr / w).max() < 1e-13
        grad_term = max(grad_term, np.abs(rb / (3.0 * s_nu) * S).max())
        # the same values, from the formula as the paper prints it
        H = np.einsum("qa,qb->qab", cf, cf) - np.eye(3) / 3.0
        P = rb * np.outer(ut, ut) - rb / (3.0 * s_nu) * S
        direct = w * (rb + 3 * rb * (cf @ ut) + 4.5 * np.einsum("qab,ab->q", H, P))
        np.testing.assert_allclose(fr, direct, rtol=0, atol=5e-16)
    assert kinds == {"central", "one-sided"}
    # the gradient term is exercised (far above rounding)
    assert grad_term > 1e-4


def test_momentum_balance_of_fixed_sphere_in_forced_flow():
    """At steady state the momentum fed by the body force (a per fluid cell and
    step) leaves through the links: F_fp = a * N_fluid."""
    n = 12
    a = 1e-6
    cfg = O.make_config(nx=n, ny=n, nz=n, walls=(0, 0, 0), nu=1 / 6, collision=O.TRT_AB,
                        body_force=(a, 0, 0), max_spheres=1)
    d = O.RefDomain(cfg)
    sid = d.add_sphere((6.2, 5.8, 6.1), 2.6, 2.0)
    d.set_mode(sid, O.MODE_FIXED)
    code, _ = d.flags()
    nf = int((code <= O.SHELL).sum())
    d.step(3000)
    F = d.sphere(sid)["F_raw"]
    assert abs(F[0] / (a * nf) - 1) < 1e-6
    assert abs(F[1]) < 1e-3 * a * nf and abs(F[2]) < 1e-3 * a * nf


def test_settling_sphere_on_symmetry_point_keeps_symmetry():
    cfg = O.make_config(nx=16, ny=16, nz=20, walls=(0, 0, 1), nu=0.05, gravity=(0, 0, -2e-5),
                        max_spheres=1)
    d = O.RefDomain(cfg)
    sid = d.add_sphere((8.0, 8.0, 11.0), 3.0, 2.5)
    d.step(25)
    s = d.sphere(sid)
    # rounding of the summed link forces (each of order 2 w_q) is the bound
    assert abs(s["F_raw"][2]) > 1e-4
    assert abs(s["F_raw"][0]) < 1e-12 and abs(s["F_raw"][1]) < 1e-12
    assert np.abs(s["T_raw"]).max() < 1e-12
    assert abs(s["x"][0] - 8.0) < 1e-12 and abs(s["x"][1] - 8.0) < 1e-12
    assert s["u"][2] < 0


def test_link_value_coefficients_of_cli():
    """Eq. (MEM_CLI) for single links placed by hand: a fluid cell whose link
    along c_q = (1, 0, 0) meets the sphere surface a quarter cell away
    (delta = 1/4, CLI coefficients (1 - 2 delta)/(1 + 2 delta) = 1/3 and
    4/(1 + 2 delta) = 8/3); the same geometry without a second fluid node
    (bounce-back, delta read as 1/2: plain bounce-back plus 6 w_q u.c_q, the
    moving-wall rule); and a rotating sphere, whose wall-point velocity is
    u + w x r_b at r_b = r + delta c_q."""
    c, w, opp = O.lattice()
    q = int(np.nonzero((c == [1, 0, 0]).all(axis=1))[0][0])
    R = 3.0
    r = np.array([-(R + 0.25), 0.0, 0.0])  # |r + delta c| = R at delta = 1/4
    Aq, Aqb, Aqm = 0.061, 0.049, 0.058
    assert abs(O.link_value(q, r, R, [0, 0, 0], [0, 0, 0], Aq, Aqb, Aqm, True) - (Aq + (Aqm - Aqb) / 3)) < 1e-16
    u = np.array([0.01, -0.02, 0.03])
    got = O.link_value(q, r, R, u, [0, 0, 0], Aq, Aqb, Aqm, True)
    assert abs(got - (Aq + (Aqm - Aqb) / 3 - 8.0 / 3.0 * w[q] * 3.0 * u[0])) < 1e-16
    got = O.link_value(q, r, R, u, [0, 0, 0], Aq, Aqb, Aqm, False)
    assert abs(got - (Aq - 6.0 * w[q] * u[0])) < 1e-16
    # rotation about z: the wall point r_b = (-R, 0, 0) moves with w x r_b = (0, -R wz, 0),
    # which has no component along c_q; rotation about y gives (0, 0, R wy) x ... likewise 0;
    # a diagonal link sees it: c = (1, 1, 0)
    q2 = int(np.nonzero((c == [1, 1, 0]).all(axis=1))[0][0])
    r2 = np.array([-(R + 0.25), 0.0, 0.0])
    wz = 0.004
    # delta from |r2 + d c|^2 = R^2: (-(R + 1/4) + d)^2 + d^2 = R^2
    a, b, cc = 2.0, -2.0 * (R + 0.25), (R + 0.25) ** 2 - R * R
    d = (-b - np.sqrt(b * b - 4 * a * cc)) / (2 * a)
    rb = r2 + d * np.array([1.0, 1.0, 0.0])
    ub = np.cross([0.0, 0.0, wz], rb)
    expect = Aq + (1 - 2 * d) / (1 + 2 * d) * (Aqm - Aqb) - 4.0 / (1 + 2 * d) * w[q2] * 3.0 * (ub[0] + ub[1])
    got = O.link_value(q2, r2, R, [0, 0, 0], [0, 0, wz], Aq, Aqb, Aqm, True)
    assert abs(got - expect) < 1e-15, (got, expect)
