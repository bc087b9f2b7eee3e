"""The oracle behind the GPU library's argument lists (lbmdem_ref_*): the
configuration layout and defaults equal those of the GPU interface (lbmdem_*,
whose pure calls run without a GPU), and driving the oracle through the
mirror with the shared harness reproduces the oracle's own wrapper bit for
bit (the mirror adds no arithmetic)."""
import ctypes as C

import numpy as np

import oracle as O
from paper_2003_01490_amd import workloads as W

from abi_harness import AbiConfig, AbiDomain, config_from
from harness import oracle_domain, random_pdf


def test_config_layout_and_defaults_equal_the_gpu_interface():
    from paper_2003_01490_amd import lbmdem as L

    ref = O.lib()
    ref.lbmdem_ref_config_bytes.restype = C.c_size_t
    assert ref.lbmdem_ref_config_bytes() == C.sizeof(AbiConfig) == C.sizeof(L.Config)
    assert [f[0] for f in AbiConfig._fields_] == [f[0] for f in L.Config._fields_]
    g = config_from({}, L.lib(), "lbmdem_")
    r = config_from({}, ref, "lbmdem_ref_")
    assert bytes(g) == bytes(r)


def test_mirror_reproduces_the_oracle_wrapper():
    wl = W.settling_32(0)
    wl.params.update(nx=16, ny=16, nz=24)
    wl.x = np.array([[8.2, 7.9, 12.3]])
    m = AbiDomain(O.lib(), "lbmdem_ref_", config_from(wl.params, O.lib(), "lbmdem_ref_", max_spheres=2))
    m.add_spheres(wl.x, wl.R, wl.rho)
    o = oracle_domain(wl)
    f = random_pdf((16, 16, 24), seed=2, amp=0.01)
    m.set_pdf(f)
    o.set_pdf(f)
    for dom in (m, o):
        dom.step(12)
    sm, so = m.sphere(0), o.sphere(0)
    for k in ("x", "u", "w", "F_fp", "T_fp", "F_tot", "F_raw"):
        assert np.array_equal(sm[k], so[k]), k
    assert np.array_equal(m.field("pdf"), o.field("pdf"))
    code, owner = o.flags()
    assert np.array_equal(m.field("flags"), code) and np.array_equal(m.field("owner"), owner)
    m.close()


def test_mirror_reports_errors_like_the_gpu_interface():
    ref = O.lib()
    m = AbiDomain(ref, "lbmdem_ref_", config_from({}, ref, "lbmdem_ref_", max_spheres=1, max_radius=3.0))
    try:
        m.add_spheres([[4.0, 4.0, 4.0]], 5.0, 2.0)  # R above max_radius
        raise AssertionError("no error")
    except RuntimeError as e:
        assert "status -1" in str(e)
    try:
        m.add_spheres([[4.0, 4.0, 1.5]], 2.0, 2.0)  # crosses the wall plane at z = 1
        raise AssertionError("no error")
    except RuntimeError as e:
        assert "status -4" in str(e)
    m.close()
