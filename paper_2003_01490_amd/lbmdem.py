"""Python binding of the lbmdem C-ABI (``include/lbmdem.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
``liblbmdem.so``.  PyTorch provides the device region (a uint8 tensor the
domain lives in) and the stream.  There is no fallback: if the library is
missing this module raises at import of ``lib()``.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import re
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "liblbmdem.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lbmdem.h")

OK, EINVAL, ENOMEM, EDEVICE, EOVERLAP, EUNSTABLE, ECAPACITY, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
TRT_AB, TRT_B, TRT, SRT = 0, 1, 2, 3
BC_CLI, BC_BOUNCE_BACK = 0, 1
STORE_F64, STORE_F32, STORE_F16 = 0, 1, 2
FREE, PRESCRIBED, FIXED = 0, 1, 2
STOP_NONE, STOP_REBOUND = 0, 1
FIELD_RHO, FIELD_VEL, FIELD_PDF, FIELD_FLAGS, FIELD_OWNER, FIELD_PDF_RAW = 0, 1, 2, 3, 4, 5
SPHERE_STATE = 42


class LbmdemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbmdem error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("walls", C.c_int32 * 3),
        ("wall_u_lo", C.c_double * 3), ("wall_u_hi", C.c_double * 3),
        ("nu", C.c_double), ("magic_lambda", C.c_double), ("lambda_b", C.c_double),
        ("delta_ab", C.c_double),
        ("collision", C.c_int32), ("boundary", C.c_int32), ("storage", C.c_int32),
        ("n_sub", C.c_int32), ("force_averaging", C.c_int32),
        ("gravity", C.c_double * 3),
        ("e_dry", C.c_double), ("poisson_ratio", C.c_double), ("friction", C.c_double),
        ("tc", C.c_double), ("dmin", C.c_double),
        ("cut_n", C.c_double), ("cut_tt", C.c_double), ("cut_tr", C.c_double),
        ("lub_mask", C.c_int32), ("max_spheres", C.c_int32),
        ("max_radius", C.c_double),
        ("dem_kernel", C.c_int32),
        ("map_kernel", C.c_int32),
        ("overlap", C.c_int32),
        ("body_force", C.c_double * 3),
    ]


_lib = None

# Domains and batches still open.  They are closed by an exit handler, which
# runs before the HIP runtime tears down (a handle destroyed from a finaliser
# during interpreter shutdown could reach a runtime that is already gone), and
# a finaliser that runs during shutdown leaves the handle alone.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def lib():
    """Load ``liblbmdem.so`` (built by ``paper_2003_01490_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime under the same soname; importing it
    # first makes this library bind to that runtime, so device pointers and
    # streams from torch are valid here.
    import torch  # noqa: F401

    if not os.path.exists(SO_PATH):
        raise ImportError(f"{SO_PATH} is not built; run `python -m paper_2003_01490_amd.build`")
    L = C.CDLL(SO_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    sig = {
        "lbmdem_config_init": (C.c_int32, [C.POINTER(Config)]),
        "lbmdem_footprint_bytes": (C.c_size_t, [C.POINTER(Config)]),
        "lbmdem_create": (C.c_int32, [C.POINTER(Config), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "lbmdem_destroy": (C.c_int32, [vp]),
        "lbmdem_add_spheres": (C.c_int32, [vp, C.c_int32, dp, dp, dp, dp, dp, ip]),
        "lbmdem_update_spheres": (C.c_int32, [vp, C.c_int32, ip, dp, dp, dp, C.c_int32]),
        "lbmdem_set_sphere_mode": (C.c_int32, [vp, C.c_int32, C.c_int32, dp, C.c_double,
                                               C.c_double, C.c_double]),
        "lbmdem_step": (C.c_int32, [vp, C.c_int32]),
        "lbmdem_sync": (C.c_int32, [vp]),
        "lbmdem_num_spheres": (C.c_int32, [vp]),
        "lbmdem_get_sphere_state": (C.c_int32, [vp, C.c_int32, dp]),
        "lbmdem_get_spheres": (C.c_int32, [vp, C.c_int32, ip, dp, dp, dp, dp, dp, dp, dp]),
        "lbmdem_get_field": (C.c_int32, [vp, C.c_int32, vp, C.c_size_t, C.c_int32]),
        "lbmdem_set_pdf": (C.c_int32, [vp, dp]),
        "lbmdem_save": (C.c_int32, [vp, vp, C.POINTER(C.c_size_t)]),
        "lbmdem_restore": (C.c_int32, [vp, vp, C.c_size_t]),
        "lbmdem_set_stop_rule": (C.c_int32, [vp, C.c_int32, C.c_int64]),
        "lbmdem_get_progress": (C.c_int32, [vp, C.POINTER(C.c_int64), ip]),
        "lbmdem_batch_create": (C.c_int32, [vp, C.c_size_t, C.POINTER(vp)]),
        "lbmdem_batch_destroy": (C.c_int32, [vp]),
        "lbmdem_batch_set_graph": (C.c_int32, [vp, C.c_int32]),
        "lbmdem_batch_admit": (C.c_int32, [vp, vp, ip]),
        "lbmdem_batch_retire": (C.c_int32, [vp, vp]),
        "lbmdem_batch_step": (C.c_int32, [vp, C.c_int32]),
        "lbmdem_batch_status": (C.c_int32, [vp, ip, C.POINTER(C.c_int64), ip, ip]),
        "lbmdem_batch_done": (C.c_int32, [vp, ip, ip]),
        "lbmdem_batch_last_error": (C.c_char_p, [vp]),
        "lbmdem_set_profiling": (C.c_int32, [vp, C.c_int32]),
        "lbmdem_set_graph": (C.c_int32, [vp, C.c_int32]),
        "lbmdem_get_profile": (C.c_int32, [vp, C.c_int32, dp, C.POINTER(C.c_int64)]),
        "lbmdem_sweep_bytes": (C.c_double, [vp]),
        "lbmdem_probe_density": (C.c_int32, [vp, C.c_int32, dp, dp]),
        "lbmdem_probe_density_static": (C.c_int32, [vp, C.c_int32, vp, vp]),
        "lbmdem_device_copy": (C.c_int32, [vp, vp, C.c_size_t, vp]),
        "lbmdem_last_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions ``include/lbmdem.h`` declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(lbmdem_[a-z0-9_]+)\s*\(", text)))


def default_config(**kw) -> Config:
    c = Config()
    lib().lbmdem_config_init(C.byref(c))
    for k, v in kw.items():
        if isinstance(v, (tuple, list, np.ndarray)):
            arr = getattr(c, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(c, k, v)
    return c


def footprint_bytes(cfg: Config) -> int:
    return int(lib().lbmdem_footprint_bytes(C.byref(cfg)))


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(v, n):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n))


class Domain:
    """One simulation domain resident on a GPU.

    The device region is a torch uint8 tensor owned by this object; all work
    runs on ``stream`` (default: torch's current stream of ``device``)."""

    def __init__(self, cfg: Config, device="cuda:0", stream=None, region=None):
        import torch

        self.cfg = cfg
        self.n = (cfg.nx, cfg.ny, cfg.nz)
        self.N = cfg.nx * cfg.ny * cfg.nz
        self.nbytes = footprint_bytes(cfg)
        if self.nbytes == 0:
            raise LbmdemError(EINVAL, "invalid configuration")
        if region is None:
            region = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        self.region = region
        base = region.data_ptr()
        ptr = (base + 255) & ~255
        if ptr + self.nbytes > base + region.numel():
            raise LbmdemError(ENOMEM, "region too small")
        self.stream = stream if stream is not None else torch.cuda.current_stream(region.device)
        h = C.c_void_p()
        rc = lib().lbmdem_create(C.byref(cfg), C.c_void_p(ptr), self.nbytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise LbmdemError(rc, lib().lbmdem_last_error(None).decode())
        self.h = h
        _live.add(self)

    def _check(self, rc):
        if rc != OK:
            raise LbmdemError(rc, lib().lbmdem_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().lbmdem_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # --- spheres ----------------------------------------------------------
    def add_spheres(self, x, R, rho, u=None, w=None):
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        n = x.shape[0]
        x = _arr(x, 3 * n)
        u = _arr(np.zeros((n, 3)) if u is None else u, 3 * n)
        w = _arr(np.zeros((n, 3)) if w is None else w, 3 * n)
        R = _arr(np.broadcast_to(np.asarray(R, dtype=np.float64), (n,)), n)
        rho = _arr(np.broadcast_to(np.asarray(rho, dtype=np.float64), (n,)), n)
        ids = np.zeros(n, dtype=np.int32)
        self._check(lib().lbmdem_add_spheres(self.h, n, _dp(x), _dp(u), _dp(w), _dp(R), _dp(rho),
                                             ids.ctypes.data_as(C.POINTER(C.c_int32))))
        return ids

    def try_add_spheres(self, x, R, rho, u=None, w=None) -> int:
        try:
            self.add_spheres(x, R, rho, u, w)
            return OK
        except LbmdemError as e:
            return e.code

    def update_spheres(self, ids, x=None, u=None, w=None):
        ids = np.ascontiguousarray(np.atleast_1d(ids), dtype=np.int32)
        n = len(ids)
        mask = (1 if x is not None else 0) | (2 if u is not None else 0) | (4 if w is not None else 0)
        z = np.zeros(3 * n)
        xa = _arr(x, 3 * n) if x is not None else z
        ua = _arr(u, 3 * n) if u is not None else z
        wa = _arr(w, 3 * n) if w is not None else z
        self._check(lib().lbmdem_update_spheres(self.h, n, ids.ctypes.data_as(C.POINTER(C.c_int32)),
                                                _dp(xa), _dp(ua), _dp(wa), mask))

    def set_mode(self, sid, mode, u_target=(0, 0, 0), c_acc=10.0, t_st=1.0, release_gap=0.0):
        ut = _arr(u_target, 3)
        self._check(lib().lbmdem_set_sphere_mode(self.h, int(sid), int(mode), _dp(ut), float(c_acc),
                                                 float(t_st), float(release_gap)))

    def num_spheres(self) -> int:
        return int(lib().lbmdem_num_spheres(self.h))

    def sphere(self, sid) -> dict:
        out = np.zeros(SPHERE_STATE)
        self._check(lib().lbmdem_get_sphere_state(self.h, int(sid), _dp(out)))
        return dict(x=out[0:3].copy(), u=out[3:6].copy(), w=out[6:9].copy(),
                    F_fp=out[9:12].copy(), T_fp=out[12:15].copy(),
                    F_tot=out[15:18].copy(), T_tot=out[18:21].copy(),
                    F_lub=out[21:24].copy(), T_lub=out[24:27].copy(),
                    F_col=out[27:30].copy(), T_col=out[30:33].copy(),
                    mode=int(out[33]), R=out[34], rho=out[35],
                    F_raw=out[36:39].copy(), T_raw=out[39:42].copy())

    def spheres(self, ids=None) -> dict:
        """States of many spheres at once (all when ids is None): arrays of
        shape (n, 3) for x, u, w, F_fp, T_fp, F_tot, T_tot."""
        if ids is None:
            n, idp = self.num_spheres(), None
        else:
            ids = np.ascontiguousarray(ids, dtype=np.int32)
            n, idp = len(ids), ids.ctypes.data_as(C.POINTER(C.c_int32))
        keys = ("x", "u", "w", "F_fp", "T_fp", "F_tot", "T_tot")
        out = {k: np.zeros((n, 3)) for k in keys}
        self._check(lib().lbmdem_get_spheres(self.h, n, idp, *[_dp(out[k]) for k in keys]))
        return out

    # --- checkpoint ---------------------------------------------------------
    def save(self) -> bytes:
        """Bitwise checkpoint (host bytes)."""
        n = C.c_size_t(0)
        self._check(lib().lbmdem_save(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(lib().lbmdem_save(self.h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def restore(self, blob: bytes):
        self._check(lib().lbmdem_restore(self.h, blob, len(blob)))

    # --- stop rule --------------------------------------------------------
    def set_stop_rule(self, rule=STOP_NONE, max_steps=0):
        self._check(lib().lbmdem_set_stop_rule(self.h, int(rule), int(max_steps)))

    def progress(self):
        """(steps done, stopped)"""
        n, st = C.c_int64(0), C.c_int32(0)
        self._check(lib().lbmdem_get_progress(self.h, C.byref(n), C.byref(st)))
        return n.value, bool(st.value)

    # --- time stepping ----------------------------------------------------
    def step(self, n=1):
        self._check(lib().lbmdem_step(self.h, int(n)))

    def sync(self):
        self._check(lib().lbmdem_sync(self.h))

    # --- fields -------------------------------------------------------------
    def field(self, which: str) -> np.ndarray:
        nx, ny, nz = self.n
        if which == "rho":
            out = np.zeros(self.N)
            shape, fid = (nz, ny, nx), FIELD_RHO
        elif which == "vel":
            out = np.zeros(3 * self.N)
            shape, fid = (3, nz, ny, nx), FIELD_VEL
        elif which == "pdf":
            out = np.zeros(19 * self.N)
            shape, fid = (19, nz, ny, nx), FIELD_PDF
        elif which == "flags":
            out = np.zeros(self.N, dtype=np.uint8)
            shape, fid = (nz, ny, nx), FIELD_FLAGS
        elif which == "owner":
            out = np.zeros(self.N, dtype=np.int32)
            shape, fid = (nz, ny, nx), FIELD_OWNER
        elif which == "pdf_raw":
            out = np.zeros(19 * self.N)
            shape, fid = (19, nz, ny, nx), FIELD_PDF_RAW
        else:
            raise ValueError(which)
        self._check(lib().lbmdem_get_field(self.h, fid, C.c_void_p(out.ctypes.data), out.nbytes, 0))
        return out.reshape(shape)

    def field_into(self, which: str, out) -> None:
        """Synchronising copy of a whole-lattice field into the device tensor
        `out` (float64 rho (N), vel (3N), pdf or pdf_raw (19N); uint8 flags;
        int32 owner), for fields too large to bring to the host."""
        fid = {"rho": FIELD_RHO, "vel": FIELD_VEL, "pdf": FIELD_PDF, "flags": FIELD_FLAGS,
               "owner": FIELD_OWNER, "pdf_raw": FIELD_PDF_RAW}[which]
        self._check(lib().lbmdem_get_field(self.h, fid, C.c_void_p(out.data_ptr()),
                                           out.numel() * out.element_size(), 1))

    def flags(self):
        return self.field("flags"), self.field("owner")

    def probe_density(self, xyz) -> np.ndarray:
        """Densities at points (n, 3) by trilinear interpolation (NaN where a
        surrounding cell is not fluid)."""
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        out = np.empty(len(xyz))
        self._check(lib().lbmdem_probe_density(self.h, len(xyz), _dp(xyz), _dp(out)))
        return out

    def probe_density_static(self, xyz, out):
        """lbmdem_probe_density_static: ``xyz`` (n, 3) and ``out`` (n,) are
        float64 device tensors; enqueued on the domain's stream, no wait."""
        n = int(out.numel())
        assert xyz.dtype == out.dtype and str(out.dtype) == "torch.float64" and xyz.numel() == 3 * n
        assert xyz.is_cuda and out.is_cuda and xyz.is_contiguous() and out.is_contiguous()
        self._check(lib().lbmdem_probe_density_static(self.h, n, C.c_void_p(xyz.data_ptr()),
                                                      C.c_void_p(out.data_ptr())))

    def set_pdf(self, f):
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(19 * self.N))
        self._check(lib().lbmdem_set_pdf(self.h, _dp(f)))

    def set_graph(self, on: bool = True):
        """Replay one captured step graph per step (needs a non-null stream)."""
        self._check(lib().lbmdem_set_graph(self.h, 1 if on else 0))

    # --- profiling --------------------------------------------------------
    def set_profiling(self, level: int):
        """0 off, 1 time the sweep only, 2 time every kernel group."""
        self._check(lib().lbmdem_set_profiling(self.h, int(level)))

    def profile(self, kernel: int):
        ms = C.c_double()
        cnt = C.c_int64()
        self._check(lib().lbmdem_get_profile(self.h, int(kernel), C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def sweep_bytes(self) -> float:
        return float(lib().lbmdem_sweep_bytes(self.h))


class Batch:
    """Many domains stepped together (one launch per kernel kind for all of
    them, replayed from a captured HIP graph).  Domains must be created on
    ``stream``."""

    def __init__(self, stream, pool_bytes: int, use_graph: bool = True):
        h = C.c_void_p()
        rc = lib().lbmdem_batch_create(C.c_void_p(stream.cuda_stream), int(pool_bytes), C.byref(h))
        if rc != OK:
            raise LbmdemError(rc, "batch creation failed")
        self.h = h
        _live.add(self)
        self.stream = stream
        self.members = {}
        if not use_graph:
            self._check(lib().lbmdem_batch_set_graph(self.h, 0))

    def _check(self, rc):
        if rc != OK:
            raise LbmdemError(rc, lib().lbmdem_batch_last_error(self.h).decode())
        return rc

    def try_admit(self, dom) -> int | None:
        """Slot id, or None when the pool budget is exhausted."""
        slot = C.c_int32(-1)
        rc = lib().lbmdem_batch_admit(self.h, dom.h, C.byref(slot))
        if rc == ENOMEM:
            return None
        self._check(rc)
        self.members[slot.value] = dom
        return slot.value

    def admit(self, dom) -> int:
        slot = self.try_admit(dom)
        if slot is None:
            raise LbmdemError(ENOMEM, "pool budget exceeded")
        return slot

    def retire(self, slot: int):
        dom = self.members.pop(slot)
        self._check(lib().lbmdem_batch_retire(self.h, dom.h))
        return dom

    def step(self, n=1):
        self._check(lib().lbmdem_batch_step(self.h, int(n)))

    def status(self):
        """{slot: (steps, stopped)} of the admitted domains."""
        n = C.c_int32(max(len(self.members), 1))
        sl = np.zeros(n.value, np.int32)
        st = np.zeros(n.value, np.int64)
        sp = np.zeros(n.value, np.int32)
        self._check(lib().lbmdem_batch_status(self.h, sl.ctypes.data_as(C.POINTER(C.c_int32)),
                                              st.ctypes.data_as(C.POINTER(C.c_int64)),
                                              sp.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
        return {int(sl[k]): (int(st[k]), bool(sp[k])) for k in range(n.value)}

    def done(self) -> list[int]:
        n = C.c_int32(max(len(self.members), 1))
        sl = np.zeros(n.value, np.int32)
        self._check(lib().lbmdem_batch_done(self.h, sl.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
        return [int(v) for v in sl[: n.value]]

    def close(self):
        if getattr(self, "h", None):
            lib().lbmdem_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def device_copy(dst_tensor, src_tensor, nbytes, stream):
    rc = lib().lbmdem_device_copy(C.c_void_p(dst_tensor.data_ptr()), C.c_void_p(src_tensor.data_ptr()),
                                  int(nbytes), C.c_void_p(stream.cuda_stream))
    if rc != OK:
        raise LbmdemError(rc, "device copy failed")
