"""Pins of the oracle's fluid solver against closed-form flows.

- shear-wave decay rate nu k^2 with nu from Eq. (Viscosity);
- sound-wave attenuation (k^2/2)(4 nu/3 + nu_b) with nu_b from Eq. (BulkViscosity),
  which checks that TRT+B relaxes rows 5-6 of M with s_b (Eq. TRTbulkmatrix);
- plane Couette flow between half-way bounce-back walls (Eq. MEM_CLI at
  delta = 1/2 with a moving wall, the shear set-up of Sec. 2.5): exact line;
- Poiseuille flow with the magic TRT parameter 3/16 (Sec. 2.1.2): parabola
  with the walls half-way, independent of viscosity; SRT is not;
- exact mass and momentum conservation in periodic boxes, mass with walls.
"""
import numpy as np
import pytest

import oracle as O


def _eq_field(rho, u):
    """f^eq on a whole field: rho (nz,ny,nx), u (3,nz,ny,nx) -> (19,nz,ny,nx)."""
    c, w, _ = O.lattice()
    cu = np.einsum("qa,a...->q...", c.astype(float), u)
    uu = (u * u).sum(0)
    return w[:, None, None, None] * (rho[None] + 3 * cu + 4.5 * cu * cu - 1.5 * uu[None])


def _mode(field, L):
    z = np.arange(L) + 0.5
    k = 2 * np.pi / L
    return (field * np.exp(-1j * k * z)).sum() * 2 / L


@pytest.mark.parametrize("nu,coll", [(0.05, O.TRT), (0.02, O.TRT_AB), (0.1, O.SRT)])
def test_shear_wave_decay_rate(nu, coll):
    L = 64
    cfg = O.make_config(nx=3, ny=3, nz=L, walls=(0, 0, 0), nu=nu, collision=coll, max_spheres=1)
    d = O.RefDomain(cfg)
    z = np.arange(L) + 0.5
    u = np.zeros((3, L, 3, 3))
    u[0] = 1e-4 * np.sin(2 * np.pi * z / L)[:, None, None]
    d.set_pdf(_eq_field(np.ones((L, 3, 3)), u))
    d.step(40)
    a1 = abs(_mode(d.field("vel")[0, :, 1, 1], L))
    d.step(300)
    a2 = abs(_mode(d.field("vel")[0, :, 1, 1], L))
    rate = -np.log(a2 / a1) / 300
    k = 2 * np.pi / L
    assert abs(rate / (nu * k * k) - 1) < 5e-3


@pytest.mark.parametrize("coll,lam_b", [(O.TRT, 1.0), (O.TRT_B, 100.0), (O.TRT_B, 10.0)])
def test_sound_wave_attenuation_gives_bulk_viscosity(coll, lam_b):
    L = 64
    nu = 0.01
    cfg = O.make_config(nx=3, ny=3, nz=L, walls=(0, 0, 0), nu=nu, collision=coll, lambda_b=lam_b,
                        max_spheres=1)
    d = O.RefDomain(cfg)
    z = np.arange(L) + 0.5
    rho = 1 + 1e-5 * np.cos(2 * np.pi * z / L)[:, None, None] * np.ones((L, 3, 3))
    d.set_pdf(_eq_field(rho, np.zeros((3, L, 3, 3))))
    ts, es = [], []
    for t in range(0, 400, 10):
        r = _mode(d.field("rho")[:, 1, 1] - 1, L)
        j = _mode(d.field("vel")[2, :, 1, 1], L)
        ts.append(t)
        es.append(abs(r) ** 2 + 3 * abs(j) ** 2)  # c_s^2 = 1/3
        d.step(10)
    ts, es = np.array(ts[5:]), np.array(es[5:])
    twogamma = -np.polyfit(ts, np.log(es), 1)[0]
    s_nu = 1 / (3 * nu + 0.5)
    s_b = 1 / (0.5 + lam_b * (1 / s_nu - 0.5))
    nu_b = 2 / 9 * (1 / s_b - 0.5)  # Eq. (BulkViscosity)
    k = 2 * np.pi / L
    gamma = 0.5 * k * k * (4 * nu / 3 + nu_b)
    assert abs(0.5 * twogamma / gamma - 1) < 0.03


@pytest.mark.parametrize("coll", [O.TRT_AB, O.TRT, O.SRT])
def test_couette_profile_is_exact(coll):
    nz = 12
    uw = 0.01
    cfg = O.make_config(nx=3, ny=3, nz=nz, walls=(0, 0, 1), wall_u_hi=(uw, 0, 0), nu=1 / 6,
                        collision=coll, max_spheres=1)
    d = O.RefDomain(cfg)
    d.step(6000)
    ux = d.field("vel")[0, 1:-1, 1, 1]
    zc = np.arange(1, nz - 1) + 0.5
    exact = uw * (zc - 1.0) / (nz - 2.0)
    assert np.abs(ux - exact).max() < 1e-12 * uw * 1e1


def _poiseuille(nu, coll, nz=12, a=1e-6, steps=None):
    cfg = O.make_config(nx=3, ny=3, nz=nz, walls=(0, 0, 1), nu=nu, collision=coll,
                        body_force=(a, 0, 0), max_spheres=1)
    d = O.RefDomain(cfg)
    H = nz - 2
    d.step(steps or int(12 * H * H / nu))
    ux = d.field("vel")[0, 1:-1, 1, 1]
    zc = np.arange(1, nz - 1) + 0.5
    exact = a / (2 * nu) * (zc - 1.0) * ((nz - 1.0) - zc)
    return np.abs(ux - exact).max() / exact.max()


@pytest.mark.parametrize("nu", [0.05, 0.3])
def test_poiseuille_trt_magic_is_exact_and_viscosity_independent(nu):
    assert _poiseuille(nu, O.TRT) < 1e-9


def test_poiseuille_srt_wall_location_depends_on_viscosity():
    """SRT's wall position moves with tau (Sec. 2.1.2): large error at large nu."""
    assert _poiseuille(0.5, O.SRT, steps=6000) > 1e-3


def test_mass_and_momentum_conserved_periodic():
    n = 6
    cfg = O.make_config(nx=n, ny=n, nz=n, walls=(0, 0, 0), nu=0.02, collision=O.TRT_B,
                        max_spheres=1)
    d = O.RefDomain(cfg)
    rng = np.random.default_rng(1)
    _, w, _ = O.lattice()
    f = w[:, None, None, None] * (1 + 0.05 * rng.standard_normal((19, n, n, n)))
    d.set_pdf(f)
    m0 = d.field("rho").sum()
    j0 = d.field("vel").reshape(3, -1).sum(1)
    d.step(200)
    assert abs(d.field("rho").sum() / m0 - 1) < 1e-13
    np.testing.assert_allclose(d.field("vel").reshape(3, -1).sum(1), j0, atol=1e-13)


def test_mass_conserved_with_bounce_back_walls():
    n = 6
    cfg = O.make_config(nx=n, ny=n, nz=n + 2, walls=(0, 0, 1), nu=0.02, max_spheres=1)
    d = O.RefDomain(cfg)
    rng = np.random.default_rng(2)
    _, w, _ = O.lattice()
    f = w[:, None, None, None] * (1 + 0.05 * rng.standard_normal((19, n + 2, n, n)))
    d.set_pdf(f)
    m0 = d.field("rho").sum()
    d.step(200)
    assert abs(d.field("rho").sum() / m0 - 1) < 1e-13
