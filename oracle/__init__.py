"""Oracle of the four-way coupled LBM-DEM scheme (Rettinger & Ruede).

TEST INFRASTRUCTURE ONLY.  A plain single-threaded FP64 C implementation of the
paper's method (``lbmdem_ref.c``), the same oracle behind the argument lists of
the GPU library's C interface (``lbmdem_ref_abi.c``: ``lbmdem_ref_*``), plus
this ctypes wrapper.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may load it;
the GPU library never imports, links or calls anything here.

Parity pins: see ``tests/test_oracle_*.py``.  Functions without a pin are
called "parity unpinned" in their docstrings here and in the design notes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblbmdem_ref.so")
_SRC = os.path.join(_HERE, "lbmdem_ref.c")
_SRCS = [_SRC, os.path.join(_HERE, "lbmdem_ref_abi.c")]
_HDRS = [os.path.join(_HERE, "lbmdem_ref.h"), os.path.join(_HERE, "lbmdem_ref_abi.h")]

NQ = 19
SPHERE_OUT = 42

FLUID, SHELL, SOLID, WALL = 0, 1, 2, 3
MODE_FREE, MODE_PRESCRIBED, MODE_FIXED = 0, 1, 2
TRT_AB, TRT_B, TRT, SRT = 0, 1, 2, 3


BUILD_FLAGS = ["-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, plain -O2) into a new
    file that then replaces the library (a process that has the old one
    loaded keeps it intact)."""
    if force or not os.path.exists(_SO):
        tmp = f"{_SO}.{os.getpid()}.tmp"
        cmd = ["gcc"] + BUILD_FLAGS + ["-o", tmp] + _SRCS + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


class RefConfig(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("walls", C.c_int32 * 3),
        ("wall_u_lo", C.c_double * 3), ("wall_u_hi", C.c_double * 3),
        ("nu", C.c_double), ("magic_lambda", C.c_double), ("lambda_b", C.c_double),
        ("delta_ab", C.c_double),
        ("collision", C.c_int32), ("boundary", C.c_int32),
        ("n_sub", C.c_int32), ("force_averaging", C.c_int32),
        ("gravity", C.c_double * 3),
        ("e_dry", C.c_double), ("poisson_ratio", C.c_double), ("friction", C.c_double),
        ("tc", C.c_double), ("dmin", C.c_double),
        ("cut_n", C.c_double), ("cut_tt", C.c_double), ("cut_tr", C.c_double),
        ("lub_mask", C.c_int32), ("max_spheres", C.c_int32),
        ("body_force", C.c_double * 3),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        stale = (not os.path.exists(_SO) or
                 os.path.getmtime(_SO) < max(os.path.getmtime(f) for f in _SRCS + _HDRS))
        if stale:
            build(force=True)
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        L.ref_create.restype = C.c_void_p
        L.ref_create.argtypes = [C.POINTER(RefConfig)]
        L.ref_destroy.argtypes = [C.c_void_p]
        L.ref_add_sphere.restype = C.c_int32
        L.ref_add_sphere.argtypes = [C.c_void_p, dp, dp, dp, C.c_double, C.c_double]
        L.ref_add_spheres.argtypes = [C.c_void_p, C.c_int32, dp, dp, dp, dp, dp]
        L.ref_add_spheres.restype = C.c_int32
        L.ref_set_mode.restype = C.c_int32
        L.ref_set_mode.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp, C.c_double,
                                   C.c_double, C.c_double]
        L.ref_update_sphere.restype = C.c_int32
        L.ref_update_sphere.argtypes = [C.c_void_p, C.c_int32, dp, dp, dp, C.c_int32]
        L.ref_step.restype = C.c_int32
        L.ref_step.argtypes = [C.c_void_p, C.c_int32]
        L.ref_dem_step.restype = C.c_int32
        L.ref_dem_step.argtypes = [C.c_void_p, dp]
        L.ref_get_sphere.restype = C.c_int32
        L.ref_get_sphere.argtypes = [C.c_void_p, C.c_int32, dp]
        L.ref_num_spheres.restype = C.c_int32
        L.ref_num_spheres.argtypes = [C.c_void_p]
        L.ref_get_field.restype = C.c_int32
        L.ref_get_field.argtypes = [C.c_void_p, C.c_int32, dp]
        L.ref_get_flags.restype = C.c_int32
        L.ref_get_flags.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.ref_set_pdf.restype = C.c_int32
        L.ref_set_pdf.argtypes = [C.c_void_p, dp]
        L.ref_step_count.restype = C.c_int64
        L.ref_step_count.argtypes = [C.c_void_p]
        L.ref_lattice.argtypes = [C.c_void_p, dp, C.c_void_p]
        L.ref_moment_matrix.argtypes = [dp]
        L.ref_moment_inverse.restype = C.c_int
        L.ref_moment_inverse.argtypes = [dp]
        L.ref_rates.argtypes = [C.POINTER(RefConfig), dp, dp, dp]
        L.ref_equilibrium.argtypes = [C.c_double, dp, dp]
        L.ref_collide.argtypes = [C.POINTER(RefConfig), dp, C.c_int32, dp, dp]
        L.ref_link_value.restype = C.c_double
        L.ref_link_value.argtypes = [C.c_int32, dp, C.c_double, dp, dp, C.c_double, C.c_double, C.c_double,
                                     C.c_int32]
        L.ref_lubrication.argtypes = [C.POINTER(RefConfig), dp, dp, dp, C.c_double, dp, dp,
                                      dp, C.c_double, C.c_int32, dp, dp]
        L.ref_collision_time.restype = C.c_double
        L.ref_collision_time.argtypes = [C.POINTER(RefConfig), C.c_double]
        L.ref_min_gap.restype = C.c_double
        L.ref_min_gap.argtypes = [C.POINTER(RefConfig), C.c_double]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(v, n=3):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n))


def make_config(**kw) -> RefConfig:
    """Config with the paper's defaults (Lambda = 3/16, Lambda_b = 100,
    delta_aB = 2, cut-offs 2/3, 1/2, 1/2, n_sub = 10) overridden by ``kw``."""
    d = dict(nx=16, ny=16, nz=16, walls=(0, 0, 1), wall_u_lo=(0, 0, 0), wall_u_hi=(0, 0, 0),
             nu=0.01, magic_lambda=3.0 / 16.0, lambda_b=100.0, delta_ab=2.0,
             collision=TRT_AB, boundary=0, n_sub=10, force_averaging=1,
             gravity=(0, 0, 0), e_dry=0.97, poisson_ratio=0.23, friction=0.15,
             tc=-1.0, dmin=-1.0, cut_n=2.0 / 3.0, cut_tt=0.5, cut_tr=0.5,
             lub_mask=7, max_spheres=4, body_force=(0, 0, 0))
    d.update(kw)
    c = RefConfig()
    for k, v in d.items():
        if isinstance(v, (tuple, list, np.ndarray)):
            arr = getattr(c, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(c, k, v)
    return c


def lattice():
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().ref_lattice(c.ctypes.data, _dp(w), opp.ctypes.data)
    return c, w, opp


def moment_matrix():
    M = np.zeros((19, 19))
    lib().ref_moment_matrix(_dp(M))
    return M


def moment_inverse():
    M = np.zeros((19, 19))
    lib().ref_moment_inverse(_dp(M))
    return M


def rates(cfg: RefConfig):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().ref_rates(C.byref(cfg), C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def collision_time(cfg: RefConfig, D: float) -> float:
    return lib().ref_collision_time(C.byref(cfg), float(D))


def min_gap(cfg: RefConfig, R: float) -> float:
    return lib().ref_min_gap(C.byref(cfg), float(R))


def equilibrium(rho, u):
    out = np.zeros(19)
    lib().ref_equilibrium(float(rho), _dp(_vec(u)), _dp(out))
    return out


def link_value(q, r, R, u, w, Aq, Aqb, Aqm, cli):
    """Eq. (MEM_CLI): the boundary value of one particle link, from the
    oracle's own link arithmetic (r = x - x_p of the fluid cell, the sphere's
    R, u, w; Aq = f~_q(x), Aqb = f~_qbar(x), Aqm = f~_q(x - c_q) with CLI)."""
    return lib().ref_link_value(int(q), _dp(_vec(r)), float(R), _dp(_vec(u)), _dp(_vec(w)), float(Aq), float(Aqb),
                                float(Aqm), int(bool(cli)))


def collide(cfg: RefConfig, f, shell=False, force=None):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(19)
    fp = _dp(_vec(force)) if force is not None else None
    lib().ref_collide(C.byref(cfg), _dp(f), int(bool(shell)), fp, _dp(out))
    return out


def lubrication(cfg: RefConfig, xi, ui, wi, Ri, xj=(0, 0, 0), uj=(0, 0, 0), wj=(0, 0, 0),
                Rj=1.0, wall=-1):
    F = np.zeros(3)
    T = np.zeros(3)
    lib().ref_lubrication(C.byref(cfg), _dp(_vec(xi)), _dp(_vec(ui)), _dp(_vec(wi)), float(Ri),
                          _dp(_vec(xj)), _dp(_vec(uj)), _dp(_vec(wj)), float(Rj), int(wall),
                          _dp(F), _dp(T))
    return F, T


class RefDomain:
    """Stateful oracle domain (one lattice, its spheres, Alg. 1 time steps)."""

    def __init__(self, cfg: RefConfig):
        self.cfg = cfg
        self.n = (cfg.nx, cfg.ny, cfg.nz)
        self.N = cfg.nx * cfg.ny * cfg.nz
        self.h = lib().ref_create(C.byref(cfg))
        if not self.h:
            raise ValueError("oracle: invalid configuration")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ref_destroy(h)
            self.h = None

    def add_sphere(self, x, R, rho, u=(0, 0, 0), w=(0, 0, 0)) -> int:
        rc = lib().ref_add_sphere(self.h, _dp(_vec(x)), _dp(_vec(u)), _dp(_vec(w)),
                                  float(R), float(rho))
        if rc < 0:
            raise ValueError(f"oracle add_sphere failed: {rc}")
        return rc

    def add_spheres(self, x, R, rho, u=None, w=None):
        """n spheres at once (arrays (n, 3), (n,), (n,)), mapped once."""
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))
        n = len(x)
        R = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(n))
        rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(n))
        uu = np.ascontiguousarray(np.zeros((n, 3)) if u is None else np.asarray(u, dtype=np.float64).reshape(n, 3))
        ww = np.ascontiguousarray(np.zeros((n, 3)) if w is None else np.asarray(w, dtype=np.float64).reshape(n, 3))
        rc = lib().ref_add_spheres(self.h, n, _dp(x), _dp(uu), _dp(ww), _dp(R), _dp(rho))
        if rc < 0:
            raise ValueError(f"oracle add_spheres failed: {rc}")

    def try_add_sphere(self, x, R, rho, u=(0, 0, 0), w=(0, 0, 0)) -> int:
        return lib().ref_add_sphere(self.h, _dp(_vec(x)), _dp(_vec(u)), _dp(_vec(w)),
                                    float(R), float(rho))

    def set_mode(self, sid, mode, u_target=(0, 0, 0), c_acc=10.0, t_st=1.0, release_gap=0.0):
        rc = lib().ref_set_mode(self.h, sid, mode, _dp(_vec(u_target)), float(c_acc),
                                float(t_st), float(release_gap))
        if rc < 0:
            raise ValueError("oracle set_mode failed")

    def update_sphere(self, sid, x=None, u=None, w=None):
        mask = (1 if x is not None else 0) | (2 if u is not None else 0) | (4 if w is not None else 0)
        z = np.zeros(3)
        rc = lib().ref_update_sphere(self.h, sid, _dp(_vec(x) if x is not None else z),
                                     _dp(_vec(u) if u is not None else z),
                                     _dp(_vec(w) if w is not None else z), mask)
        if rc < 0:
            raise ValueError("oracle update_sphere failed")

    def step(self, n=1):
        if lib().ref_step(self.h, int(n)) != 0:
            raise RuntimeError("oracle step failed")

    def dem_step(self, fext=None):
        P = self.num_spheres()
        arr = None
        if fext is not None:
            arr = np.ascontiguousarray(np.asarray(fext, dtype=np.float64).reshape(P * 6))
        lib().ref_dem_step(self.h, _dp(arr) if arr is not None else None)

    def num_spheres(self) -> int:
        return lib().ref_num_spheres(self.h)

    def sphere(self, sid) -> dict:
        out = np.zeros(SPHERE_OUT)
        lib().ref_get_sphere(self.h, sid, _dp(out))
        return dict(x=out[0:3].copy(), u=out[3:6].copy(), w=out[6:9].copy(),
                    F_fp=out[9:12].copy(), T_fp=out[12:15].copy(),
                    F_tot=out[15:18].copy(), T_tot=out[18:21].copy(),
                    F_lub=out[21:24].copy(), T_lub=out[24:27].copy(),
                    F_col=out[27:30].copy(), T_col=out[30:33].copy(),
                    mode=int(out[33]), R=out[34], rho=out[35],
                    F_raw=out[36:39].copy(), T_raw=out[39:42].copy())

    def field(self, which: str) -> np.ndarray:
        nx, ny, nz = self.n
        if which == "rho":
            out = np.zeros(self.N)
            lib().ref_get_field(self.h, 0, _dp(out))
            return out.reshape(nz, ny, nx)
        if which == "vel":
            out = np.zeros(3 * self.N)
            lib().ref_get_field(self.h, 1, _dp(out))
            return out.reshape(3, nz, ny, nx)
        if which == "pdf":
            out = np.zeros(19 * self.N)
            lib().ref_get_field(self.h, 2, _dp(out))
            return out.reshape(19, nz, ny, nx)
        raise ValueError(which)

    def flags(self):
        nx, ny, nz = self.n
        code = np.zeros(self.N, dtype=np.uint8)
        owner = np.zeros(self.N, dtype=np.int32)
        lib().ref_get_flags(self.h, code.ctypes.data, owner.ctypes.data)
        return code.reshape(nz, ny, nx), owner.reshape(nz, ny, nx)

    def set_pdf(self, f):
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(19 * self.N))
        lib().ref_set_pdf(self.h, _dp(f))
