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


@pytest.mark.parametrize("seed", range(4))
def test_mapping_matches_exact_integer_classification(seed):
    rng = np.random.default_rng(seed)
    n = (12, 11, 14)
    walls = (0, 0, 1)
    cfg = O.make_config(nx=n[0], ny=n[1], nz=n[2], walls=walls, max_spheres=3)
    d = O.RefDomain(cfg)
    spheres = []
    # includes ties: R and offsets on the 2^-10 grid so d^2 == R^2 happens
    for sid in range(3):
        for _ in range(200):
            R = rng.integers(1 * 1024, 3 * 1024) / 1024.0
            if sid == 0:
                R = 2.5
            x = [rng.integers(0, n[a] * 1024) / 1024.0 for a in range(3)]
            if sid == 0:
                x = [5.0, 5.5, 6.0]  # several cells exactly on the surface
            if d.try_add_sphere(x, R, 2.0) >= 0:
                spheres.append((x, R))
                break
    code, owner = d.flags()
    ecode, eowner = _exact_flags(n, walls, spheres)
    assert np.array_equal(code, ecode)
    sol = ecode == O.SOLID
    assert np.array_equal(owner[sol], eowner[sol])
    # the tie case really happens: cells with d^2 == R^2 exist and are solid
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
