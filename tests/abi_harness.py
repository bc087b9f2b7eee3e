"""One ctypes harness for both C interfaces: the GPU library's lbmdem_* calls
and the oracle's lbmdem_ref_* mirror take the same arguments, so the same code
below drives either (test infrastructure)."""
from __future__ import annotations

import ctypes as C

import numpy as np


class AbiConfig(C.Structure):
    """The configuration layout both interfaces share."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("walls", C.c_int32 * 3),
        ("wall_u_lo", C.c_double * 3), ("wall_u_hi", C.c_double * 3),
        ("nu", C.c_double), ("magic_lambda", C.c_double), ("lambda_b", C.c_double), ("delta_ab", C.c_double),
        ("collision", C.c_int32), ("boundary", C.c_int32), ("storage", C.c_int32),
        ("n_sub", C.c_int32), ("force_averaging", C.c_int32),
        ("gravity", C.c_double * 3),
        ("e_dry", C.c_double), ("poisson_ratio", C.c_double), ("friction", C.c_double),
        ("tc", C.c_double), ("dmin", C.c_double),
        ("cut_n", C.c_double), ("cut_tt", C.c_double), ("cut_tr", C.c_double),
        ("lub_mask", C.c_int32), ("max_spheres", C.c_int32), ("max_radius", C.c_double),
        ("dem_kernel", C.c_int32), ("map_kernel", C.c_int32), ("overlap", C.c_int32),
        ("body_force", C.c_double * 3),
    ]


FIELDS = {"rho": (0, np.float64, 1), "vel": (1, np.float64, 3), "pdf": (2, np.float64, 19),
          "flags": (3, np.uint8, 1), "owner": (4, np.int32, 1)}
STATE = {"x": 0, "u": 3, "w": 6, "F_fp": 9, "T_fp": 12, "F_tot": 15, "T_tot": 18, "F_lub": 21, "T_lub": 24,
         "F_col": 27, "T_col": 30, "F_raw": 36, "T_raw": 39}


_PRIVATE: dict = {}


def _own(lib):
    """A CDLL instance of the same library for the harness alone: ctypes keeps
    prototypes per instance, so the harness's prototypes do not replace those
    of the library's own binding."""
    if lib._name not in _PRIVATE:
        _PRIVATE[lib._name] = C.CDLL(lib._name)
    return _PRIVATE[lib._name]


def _fn(lib, prefix, name, restype, argtypes):
    f = getattr(lib, prefix + name)
    f.restype = restype
    f.argtypes = argtypes
    return f


class AbiDomain:
    """A domain of either interface: `lib` a loaded CDLL, `prefix` "lbmdem_"
    (GPU library) or "lbmdem_ref_" (oracle)."""

    def __init__(self, lib, prefix: str, cfg: AbiConfig):
        lib = _own(lib)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        self.f = {
            "create": _fn(lib, prefix, "create", C.c_int32, [C.POINTER(AbiConfig), vp, C.c_size_t, vp,
                                                             C.POINTER(vp)]),
            "destroy": _fn(lib, prefix, "destroy", C.c_int32, [vp]),
            "add_spheres": _fn(lib, prefix, "add_spheres", C.c_int32, [vp, C.c_int32, dp, dp, dp, dp, dp, ip]),
            "update_spheres": _fn(lib, prefix, "update_spheres", C.c_int32, [vp, C.c_int32, ip, dp, dp, dp,
                                                                             C.c_int32]),
            "set_sphere_mode": _fn(lib, prefix, "set_sphere_mode", C.c_int32, [vp, C.c_int32, C.c_int32, dp,
                                                                               C.c_double, C.c_double, C.c_double]),
            "step": _fn(lib, prefix, "step", C.c_int32, [vp, C.c_int32]),
            "sync": _fn(lib, prefix, "sync", C.c_int32, [vp]),
            "num_spheres": _fn(lib, prefix, "num_spheres", C.c_int32, [vp]),
            "get_sphere_state": _fn(lib, prefix, "get_sphere_state", C.c_int32, [vp, C.c_int32, dp]),
            "get_field": _fn(lib, prefix, "get_field", C.c_int32, [vp, C.c_int32, vp, C.c_size_t, C.c_int32]),
            "set_pdf": _fn(lib, prefix, "set_pdf", C.c_int32, [vp, dp]),
            "last_error": _fn(lib, prefix, "last_error", C.c_char_p, [vp]),
        }
        self.cfg = cfg
        self.N = cfg.nx * cfg.ny * cfg.nz
        h = vp()
        self._ok(self.f["create"](C.byref(cfg), None, 0, None, C.byref(h)), None)
        self.h = h

    def _ok(self, rc, h=...):
        if rc != 0:
            msg = self.f["last_error"](self.h if h is ... else h)
            raise RuntimeError(f"status {rc}: {msg.decode() if msg else ''}")

    @staticmethod
    def _d(a):
        return a.ctypes.data_as(C.POINTER(C.c_double))

    def add_spheres(self, x, R, rho, u=None, w=None):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        n = len(x)
        u = np.zeros((n, 3)) if u is None else np.ascontiguousarray(u, dtype=np.float64)
        w = np.zeros((n, 3)) if w is None else np.ascontiguousarray(w, dtype=np.float64)
        R = np.ascontiguousarray(np.broadcast_to(R, (n,)), dtype=np.float64)
        rho = np.ascontiguousarray(np.broadcast_to(rho, (n,)), dtype=np.float64)
        self._ok(self.f["add_spheres"](self.h, n, self._d(x), self._d(u), self._d(w), self._d(R), self._d(rho),
                                       None))

    def set_mode(self, i, mode, u_target=(0.0, 0.0, 0.0), c_acc=0.0, t_st=1.0, release_gap=0.0):
        ut = np.asarray(u_target, dtype=np.float64)
        self._ok(self.f["set_sphere_mode"](self.h, i, mode, self._d(ut), c_acc, t_st, release_gap))

    def step(self, n=1):
        self._ok(self.f["step"](self.h, n))
        self._ok(self.f["sync"](self.h))

    def sphere(self, i):
        out = np.zeros(42)
        self._ok(self.f["get_sphere_state"](self.h, i, self._d(out)))
        s = {k: out[a:a + 3].copy() for k, a in STATE.items()}
        s["mode"] = int(out[33])
        return s

    def field(self, name):
        code, dt, comps = FIELDS[name]
        a = np.zeros(comps * self.N, dtype=dt)
        self._ok(self.f["get_field"](self.h, code, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))
        shape = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        return a.reshape((comps,) + shape) if comps > 1 else a.reshape(shape)

    def set_pdf(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._ok(self.f["set_pdf"](self.h, self._d(f)))

    def close(self):
        if self.h:
            self.f["destroy"](self.h)
            self.h = None


def config_from(params: dict, lib, prefix: str, **over) -> AbiConfig:
    """The interface's defaults (its config_init call) overridden by the
    workload parameters it has fields for, then by `over`."""
    c = AbiConfig()
    init = getattr(_own(lib), prefix + "config_init")
    init.restype = C.c_int32
    init.argtypes = [C.POINTER(AbiConfig)]
    assert init(C.byref(c)) == 0
    names = {f[0] for f in AbiConfig._fields_}
    for k, v in {**params, **over}.items():
        if k not in names:
            continue
        if isinstance(v, (tuple, list, np.ndarray)):
            arr = getattr(c, k)
            for i, e in enumerate(v):
                arr[i] = e
        else:
            setattr(c, k, v)
    return c
