"""Builds matching oracle and GPU domains from one seeded workload and compares
them.  The oracle is only called here (test infrastructure)."""
from __future__ import annotations

import os

import numpy as np

import oracle as O
from paper_2003_01490_amd import workloads as W

ORACLE_KEYS = set(O.RefConfig._fields_ and [f[0] for f in O.RefConfig._fields_])


def oracle_domain(wl: W.Workload, **over):
    p = dict(wl.params)
    p.update(over)
    p = {k: v for k, v in p.items() if k in ORACLE_KEYS}
    d = O.RefDomain(O.make_config(**p))
    if len(wl.R):
        d.add_spheres(wl.x, wl.R, wl.rho, u=wl.u, w=wl.w)
    if wl.ramp is not None:
        r = wl.ramp
        d.set_mode(0, O.MODE_PRESCRIBED, r["u_target"], r["c_acc"], r["t_st"], r["release_gap"])
    return d


def gpu_domain(wl: W.Workload, storage=0, device="cuda:0", stream=None, **over):
    from paper_2003_01490_amd import lbmdem as L

    p = dict(wl.params)
    p.update(over)
    gkeys = {f[0] for f in L.Config._fields_}
    p = {k: v for k, v in p.items() if k in gkeys}
    p["storage"] = storage
    p["max_radius"] = over.get("max_radius", float(max(wl.R)) if len(wl.R) else 1.0)
    p["max_spheres"] = max(p.get("max_spheres", 1), len(wl.R), 1)
    d = L.Domain(L.default_config(**p), device=device, stream=stream)
    if len(wl.R):
        d.add_spheres(wl.x, wl.R, wl.rho, u=wl.u, w=wl.w)
    if wl.ramp is not None:
        r = wl.ramp
        d.set_mode(0, L.PRESCRIBED, r["u_target"], r["c_acc"], r["t_st"], r["release_gap"])
    return d


def rel_field_err(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


def sphere_errs(sa: dict, sb: dict, D: float, scale: dict | None = None):
    """Errors of one sphere's state against the reference sb.  Positions are
    relative to the diameter D; velocities, angular velocities, forces and
    torques relative to the magnitudes in ``scale`` (keys u, F; defaults to
    the reference's own magnitudes).  Angular velocities are scaled by u/R and
    torques by F R, since a sphere that barely rotates has w at rounding level."""
    R = D / 2
    us = max((scale or {}).get("u", 0.0), np.abs(sb["u"]).max(), 1e-300)
    Fs = max((scale or {}).get("F", 0.0), np.abs(sb["F_tot"]).max(), 1e-300)
    out = {"x": float(np.abs(sa["x"] - sb["x"]).max() / D)}
    out["u"] = float(np.abs(sa["u"] - sb["u"]).max() / us)
    out["w"] = float(np.abs(sa["w"] - sb["w"]).max() * R / us)
    for k in ("F_fp", "F_raw", "F_tot", "F_lub", "F_col"):
        out[k] = float(np.abs(sa[k] - sb[k]).max() / Fs)
    for k in ("T_fp", "T_raw"):
        out[k] = float(np.abs(sa[k] - sb[k]).max() / (Fs * R))
    return out


class Scales:
    """Running maxima of the reference trajectory (velocity and force)."""

    def __init__(self, weight=0.0):
        self.u = 0.0
        self.F = weight

    def update(self, s):
        self.u = max(self.u, float(np.abs(s["u"]).max()))
        self.F = max(self.F, float(np.abs(s["F_tot"]).max()), float(np.abs(s["F_fp"]).max()))
        return {"u": self.u, "F": self.F}


def weight(wl, i=0):
    """Buoyant weight V (rho_p - 1) |g| of sphere i (force scale)."""
    g = np.linalg.norm(np.asarray(wl.params.get("gravity", (0, 0, 0)), dtype=float))
    return 4.0 / 3.0 * np.pi * wl.R[i] ** 3 * abs(wl.rho[i] - 1.0) * g


def random_pdf(n, seed, amp=0.02, u0=(0.0, 0.0, 0.0)):
    """Equilibrium at rho 1 and u0 plus seeded noise (input generator)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    feq = O.equilibrium(1.0, np.asarray(u0, dtype=float))
    f = feq[:, None, None, None] * (1.0 + amp * rng.standard_normal((19, nz, ny, nx)))
    return f


def exact_tie_counts(n, walls, spheres, delta_ab=2.0, scale=1 << 11):
    """Exact counts of cell centres lying on a sphere surface (d^2 == R^2), on a
    shell surface (d^2 == (R + delta_aB)^2), and inside or on two solid balls."""
    on_surface = on_shell = shared = 0
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                ijk = (i, j, k)
                inside = 0
                for x, R in spheres:
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
                    Ri, Rs = int(round(R * scale)), int(round((R + delta_ab) * scale))
                    on_surface += d2 == Ri * Ri
                    on_shell += d2 == Rs * Rs
                    inside += d2 <= Ri * Ri
                shared += inside >= 2
    return on_surface, on_shell, shared


# ---- observed error maxima ---------------------------------------------------
# Every parity bound goes through check(): the largest value seen per test and
# quantity is kept with its bound and printed in the session summary, so a run
# shows how far each bound sits above what the GPU path actually produced.
OBSERVED: dict = {}


def check(quantity: str, value: float, bound: float, where=""):
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    key = (test, quantity)
    old = OBSERVED.get(key, (0.0, bound))
    OBSERVED[key] = (max(old[0], float(value)), max(old[1], bound))
    assert value <= bound, f"{quantity} {value:.3e} above its bound {bound:.1e} {where}"


SPHERE_QUANTITIES = ("x", "u", "w", "F_fp", "F_raw", "F_tot", "F_lub", "F_col", "T_fp", "T_raw")


def fp64_bounds(**over):
    """Bounds on the sphere errors of sphere_errs() for FP64 storage: 1e-12
    for every quantity unless a test sets another (each such bound sits 3 to
    10 times above the maximum the test has shown)."""
    b = {k: 1e-12 for k in SPHERE_QUANTITIES}
    b.update(over)
    return b


def check_all(errs: dict, bounds: dict, where=""):
    for k, b in bounds.items():
        check(k, errs[k], b, where)


def oracle_fingerprint() -> str:
    """SHA-256 over the oracle's arithmetic (its C source and header): a
    stored oracle result is valid only for the oracle that wrote it."""
    import hashlib

    h = hashlib.sha256()
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
    for name in ("lbmdem_ref.c", "lbmdem_ref.h"):
        with open(os.path.join(root, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def workload_key(wl: W.Workload) -> dict:
    """What a stored trajectory depends on: the workload's parameters, its
    initial sphere state and the prescribed-motion ramp."""
    def plain(v):
        if isinstance(v, (tuple, list, np.ndarray)):
            return [plain(u) for u in np.asarray(v).tolist()] if isinstance(v, np.ndarray) else [plain(u) for u in v]
        if isinstance(v, (np.floating, np.integer)):
            return v.item()
        return v

    return {"params": {k: plain(v) for k, v in sorted(wl.params.items())},
            "x": plain(wl.x), "R": plain(wl.R), "rho": plain(wl.rho), "u": plain(wl.u), "w": plain(wl.w),
            "ramp": {k: plain(v) for k, v in sorted((wl.ramp or {}).items())}}
