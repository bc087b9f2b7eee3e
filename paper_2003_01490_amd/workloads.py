"""Seeded synthetic workloads (inputs only, none of the method's arithmetic).

Both the GPU path and the test oracle take their inputs from here: lattice
size, fluid and DEM parameters, and sphere positions/velocities drawn with
``numpy.random.default_rng(seed)``.  The paper's experiments use physical
tables (Sec. 4.4, Table sphereWallCollision); the values below convert them to
lattice units where a workload asks for it.

Workloads:
  settling_32     - 32^3, z walls, nu 0.01, D 8, density ratio 2.5, centre
                    (16,16,20) + U[-1/2,1/2]^3, gravity 1e-5, 300 steps, FP64.
  contact_32      - the same domain with the sphere 0.7 above the bottom wall
                    and u_z = -0.01 (contact and lubrication within 300 steps).
  sphere_wall     - 128x128x256, z walls, D 20, Stokes number 100 from a seeded
                    density ratio U[2,8] and viscosity logU[0.005,0.05]
                    (rejecting u_s > 0.1), released from the ramp of
                    Eq. (artificial_acceleration) one diameter above the wall.
  rebound_st27    - the St = 27 case of the sub-cycle study (Table
                    sphereWallCollision_nsub_D20): 12 x 12 x 48 D with D 20,
                    u_s 0.02, T_c and delta_min by the paper's relations, the
                    start 3/2 D below the top wall perturbed by U[-1/2,1/2] in z.
  serve_requests  - a stream of independent sphere-wall requests with Poisson
                    arrivals (edges, diameter, Stokes number, density ratio
                    drawn per request), and serve_workload, the domain of one.
  dense           - cubic lattice with z walls, equal spheres placed by seeded
                    random sequential addition with a surface gap >= 1 to
                    every other sphere and wall (optionally smaller, and with
                    seeded Gaussian velocities so that lubrication and
                    contacts occur within a few hundred steps).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Table sphereWallCollision (Sec. 4.4.2), St = 100 and St = 27 rows: fluid
# density, dynamic viscosity, diameter, particle density, gravity (SI)
_ST100 = dict(rho_f=953.0, mu_f=0.02, D=0.004, rho_p=7800.0, g=9.81)
_ST27 = dict(rho_f=965.0, mu_f=0.1, D=0.006, rho_p=7800.0, g=9.81)


@dataclass
class Workload:
    name: str
    params: dict
    x: np.ndarray
    R: np.ndarray
    rho: np.ndarray
    u: np.ndarray
    w: np.ndarray
    steps: int
    ramp: dict | None = None     # prescribed-velocity protocol of sphere 0
    meta: dict = field(default_factory=dict)


def base_params(**kw) -> dict:
    """Defaults of the paper: Lambda 3/16, Lambda_b 100, delta_aB 2, cut-offs
    2/3, 1/2, 1/2, n_sub 10, T_c and delta_min by its relations; e_dry 0.97
    (Table sphereWallCollision), nu_p 0.23 and mu_p 0.15 (TW1 of Table
    obliqueCollision)."""
    p = dict(nx=32, ny=32, nz=32, walls=(0, 0, 1), wall_u_lo=(0, 0, 0), wall_u_hi=(0, 0, 0),
             nu=0.01, magic_lambda=3.0 / 16.0, lambda_b=100.0, delta_ab=2.0, collision=0,
             boundary=0, n_sub=10, force_averaging=1, gravity=(0.0, 0.0, 0.0), e_dry=0.97,
             poisson_ratio=0.23, friction=0.15, tc=-1.0, dmin=-1.0, cut_n=2.0 / 3.0, cut_tt=0.5,
             cut_tr=0.5, lub_mask=7, max_spheres=1)
    p.update(kw)
    return p


def settling_32(seed: int = 0) -> Workload:
    rng = np.random.default_rng(seed)
    x = np.array([16.0, 16.0, 20.0]) + rng.uniform(-0.5, 0.5, 3)
    p = base_params(nu=0.01, gravity=(0.0, 0.0, -1e-5), max_spheres=1)
    return Workload("settling_32", p, x[None], np.array([4.0]), np.array([2.5]), np.zeros((1, 3)),
                    np.zeros((1, 3)), 300, meta=dict(seed=seed))


def contact_32(seed: int = 0) -> Workload:
    rng = np.random.default_rng(seed)
    x = np.array([16.0, 16.0, 1.0 + 4.0 + 0.7])
    x[:2] += rng.uniform(-0.5, 0.5, 2)
    p = base_params(nu=0.01, gravity=(0.0, 0.0, -1e-5), max_spheres=1)
    return Workload("contact_32", p, x[None], np.array([4.0]), np.array([2.5]),
                    np.array([[0.0, 0.0, -0.01]]), np.zeros((1, 3)), 300, meta=dict(seed=seed))


def sphere_wall(seed: int = 0, nx: int = 128, ny: int = 128, nz: int = 256, D: float = 20.0,
                St: float = 100.0, default_draw: bool = True) -> Workload:
    """Sphere-wall collision at a given Stokes number (Sec. 4.4).  With
    ``default_draw`` the density ratio and viscosity of the paper's St = 100
    row are used (rho_p/rho_f = 7800/953, nu from the lattice speed u_s);
    otherwise they are drawn from the seed."""
    rng = np.random.default_rng(seed)
    if default_draw:
        rho_r = _ST100["rho_p"] / _ST100["rho_f"]
        u_s = 0.028
        nu = u_s * D * rho_r / (9.0 * St)
    else:
        while True:
            rho_r = rng.uniform(2.0, 8.0)
            nu = math.exp(rng.uniform(math.log(0.005), math.log(0.05)))
            u_s = 9.0 * St * nu / (rho_r * D)
            if u_s <= 0.1:
                break
    # gravity from the Froude number g D / u_s^2 of the St = 100 experiment
    nu_phys = _ST100["mu_f"] / _ST100["rho_f"]
    us_phys = 9.0 * St * nu_phys * _ST100["rho_f"] / (_ST100["rho_p"] * _ST100["D"])
    fr = _ST100["g"] * _ST100["D"] / us_phys ** 2
    g = fr * u_s ** 2 / D
    x = np.array([nx / 2.0, ny / 2.0, (nz - 1.0) - 1.5 * D])
    x[:2] += rng.uniform(-0.5, 0.5, 2)
    p = base_params(nx=nx, ny=ny, nz=nz, nu=nu, gravity=(0.0, 0.0, -g), max_spheres=1)
    t_st = rho_r * D * D / (18.0 * nu)
    ramp = dict(u_target=(0.0, 0.0, -u_s), c_acc=10.0, t_st=t_st, release_gap=D)
    return Workload("sphere_wall", p, x[None], np.array([D / 2]), np.array([rho_r]),
                    np.zeros((1, 3)), np.zeros((1, 3)), 20000, ramp=ramp,
                    meta=dict(seed=seed, St=St, u_s=u_s, rho_r=rho_r, nu=nu, g=g, froude=fr))


def dense(seed: int = 0, n: int = 96, count: int = 156, D: float = 12.0, rho_r: float = 2.0,
          nu: float = 0.02, g: float = 2e-6, min_gap: float = 1.0, steps: int = 100,
          nxyz: tuple | None = None, u_rms: float = 0.0) -> Workload:
    """Random sequential addition of equal spheres (periodic x, y; z walls).
    ``u_rms`` > 0 draws N(0, u_rms) velocity components after the placement."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = nxyz if nxyz else (n, n, n)
    R = D / 2.0
    cell = D + min_gap
    gx, gy, gz = int(nx // cell) or 1, int(ny // cell) or 1, int(nz // cell) or 1
    grid: dict = {}
    pts = []
    tries = 0
    lo_z, hi_z = 1.0 + R + min_gap, (nz - 1.0) - R - min_gap
    while len(pts) < count:
        tries += 1
        if tries > 200 * count + 100000:
            raise RuntimeError("could not place the requested number of spheres")
        c = np.array([rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(lo_z, hi_z)])
        key = (int(c[0] / nx * gx) % gx, int(c[1] / ny * gy) % gy, min(int(c[2] / nz * gz), gz - 1))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    kk = ((key[0] + dx) % gx, (key[1] + dy) % gy, key[2] + dz)
                    for j in grid.get(kk, ()):
                        d = c - pts[j]
                        d[0] -= nx * round(d[0] / nx)
                        d[1] -= ny * round(d[1] / ny)
                        if np.linalg.norm(d) < D + min_gap:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            grid.setdefault(key, []).append(len(pts))
            pts.append(c)
    x = np.array(pts)
    u = rng.normal(0.0, u_rms, (count, 3)) if u_rms > 0 else np.zeros((count, 3))
    p = base_params(nx=nx, ny=ny, nz=nz, nu=nu, gravity=(0.0, 0.0, -g), max_spheres=count)
    frac = count * (4.0 / 3.0) * math.pi * R ** 3 / (nx * ny * nz)
    return Workload("dense", p, x, np.full(count, R), np.full(count, rho_r), u,
                    np.zeros((count, 3)), steps,
                    meta=dict(seed=seed, solid_fraction=frac, min_gap=min_gap, u_rms=u_rms))


def serve_requests(seed: int = 0, n: int = 512, rate: float = 50.0, edge_range=(48, 192),
                   D_range=(6.0, 24.0), St_range=(1.0, 1000.0), rho_range=(1.5, 8.0), u_s: float = 0.02,
                   nu_min: float = 1e-3) -> list[dict]:
    """Requests of the serving mix: arrivals of a Poisson process of the given
    rate (per second); edges uniform integers per axis with max/min <= 1.5,
    L_z >= 6 D and min(L_x, L_y) >= 3 D; D uniform; St log-uniform (redrawn
    while nu = u_s D rho_r / (9 St) < nu_min); rho_r uniform."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate))
        while True:
            L = rng.integers(edge_range[0], edge_range[1] + 1, size=3)
            D = float(rng.uniform(*D_range))
            if L.max() / L.min() <= 1.5 and L[2] >= 6 * D and min(L[0], L[1]) >= 3 * D:
                break
        rho_r = float(rng.uniform(*rho_range))
        while True:
            St = math.exp(rng.uniform(math.log(St_range[0]), math.log(St_range[1])))
            nu = u_s * D * rho_r / (9.0 * St)
            if nu >= nu_min:
                break
        jitter = rng.uniform(-0.5, 0.5, 2)
        out.append(dict(id=k, arrival=t, L=tuple(int(v) for v in L), D=D, St=St, rho_r=rho_r, nu=nu,
                        u_s=u_s, jitter=tuple(float(v) for v in jitter)))
    return out


def serve_workload(req: dict) -> Workload:
    """Domain of one request: the sphere-wall protocol (ramp of
    Eq. (artificial_acceleration) to u_s from 1.5 D below the top wall,
    release one diameter above the bottom wall), gravity from the Froude
    number of the St = 100 experiment, FP32-sized parameters."""
    nx, ny, nz = req["L"]
    D, u_s, nu, rho_r = req["D"], req["u_s"], req["nu"], req["rho_r"]
    nu_phys = _ST100["mu_f"] / _ST100["rho_f"]
    us_phys = 9.0 * 100.0 * nu_phys * _ST100["rho_f"] / (_ST100["rho_p"] * _ST100["D"])
    fr = _ST100["g"] * _ST100["D"] / us_phys ** 2
    g = fr * u_s ** 2 / D
    x = np.array([nx / 2.0 + req["jitter"][0], ny / 2.0 + req["jitter"][1], (nz - 1.0) - 1.5 * D])
    p = base_params(nx=nx, ny=ny, nz=nz, nu=nu, gravity=(0.0, 0.0, -g), max_spheres=1)
    t_st = rho_r * D * D / (18.0 * nu)
    ramp = dict(u_target=(0.0, 0.0, -u_s), c_acc=10.0, t_st=t_st, release_gap=D)
    return Workload("serve", p, x[None], np.array([D / 2]), np.array([rho_r]), np.zeros((1, 3)),
                    np.zeros((1, 3)), 0, ramp=ramp, meta=dict(req))


def rebound_st27(seed: int = 0, D: float = 20.0, u_s: float = 0.02, n_sub: int = 10) -> Workload:
    """Sphere-wall collision at St = 27 (Sec. 4.4.2, parameter set SW9/SW10):
    domain 12 x 12 x 48 diameters, density ratio 7800/965, the viscosity from
    St = rho_r u_s D / (9 nu), gravity from the experiment's Froude number
    g D / u_s^2, the sphere horizontally centred, 3/2 D below the top wall
    plane, its height perturbed by U[-1/2, 1/2] (the paper perturbs the start
    by one cell), ramped with c_acc = 10 and released one diameter above the
    bottom wall."""
    rng = np.random.default_rng(seed)
    t = _ST27
    rho_r = t["rho_p"] / t["rho_f"]
    nu_phys = t["mu_f"] / t["rho_f"]
    re = 30.0  # Table sphereWallCollision, St = 27 row
    us_phys = re * nu_phys / t["D"]
    St = rho_r * us_phys * t["D"] / (9.0 * nu_phys)
    nu = rho_r * u_s * D / (9.0 * St)
    fr = t["g"] * t["D"] / us_phys ** 2
    g = fr * u_s ** 2 / D
    n = int(round(12 * D)), int(round(12 * D)), int(round(48 * D))
    x = np.array([n[0] / 2.0, n[1] / 2.0, (n[2] - 1.0) - 1.5 * D + rng.uniform(-0.5, 0.5)])
    p = base_params(nx=n[0], ny=n[1], nz=n[2], nu=nu, n_sub=n_sub, gravity=(0.0, 0.0, -g), max_spheres=1)
    t_st = rho_r * D * D / (18.0 * nu)
    ramp = dict(u_target=(0.0, 0.0, -u_s), c_acc=10.0, t_st=t_st, release_gap=D)
    return Workload("rebound_st27", p, x[None], np.array([D / 2]), np.array([rho_r]),
                    np.zeros((1, 3)), np.zeros((1, 3)), 80000, ramp=ramp,
                    meta=dict(seed=seed, St=St, u_s=u_s, rho_r=rho_r, nu=nu, g=g, froude=fr))
