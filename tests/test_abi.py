"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and its pure functions (defaults, footprint) behave."""
import ctypes as C

import pytest

from paper_2003_01490_amd import lbmdem as L


def test_library_exports_every_header_function():
    lib = L.lib()
    names = L.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_config_defaults_are_the_papers():
    c = L.default_config()
    assert c.magic_lambda == 3 / 16 and c.lambda_b == 100 and c.delta_ab == 2
    assert c.cut_n == 2 / 3 and c.cut_tt == 0.5 and c.cut_tr == 0.5 and c.n_sub == 10
    assert c.collision == L.TRT_AB and c.boundary == L.BC_CLI


def test_footprint_is_pure_and_scales_with_storage():
    f64 = L.footprint_bytes(L.default_config(nx=64, ny=64, nz=64, storage=L.STORE_F64))
    f32 = L.footprint_bytes(L.default_config(nx=64, ny=64, nz=64, storage=L.STORE_F32))
    f16 = L.footprint_bytes(L.default_config(nx=64, ny=64, nz=64, storage=L.STORE_F16))
    N = 64 ** 3
    assert f64 - f32 == pytest.approx(2 * 19 * 4 * N, abs=1024)
    assert f32 - f16 == pytest.approx(2 * 19 * 2 * N, abs=1024)
    assert f64 % 256 == 0


@pytest.mark.parametrize("bad", [dict(nx=2), dict(nu=0.0), dict(storage=5), dict(n_sub=0),
                                 dict(collision=9), dict(e_dry=0.0), dict(max_spheres=3, max_radius=0.0)])
def test_invalid_config_has_zero_footprint(bad):
    assert L.footprint_bytes(L.default_config(**bad)) == 0


def test_create_rejects_small_region_without_touching_device():
    c = L.default_config(nx=16, ny=16, nz=16)
    h = C.c_void_p()
    rc = L.lib().lbmdem_create(C.byref(c), C.c_void_p(256), 16, None, C.byref(h))
    assert rc == L.ENOMEM and not h.value
    assert b"smaller" in L.lib().lbmdem_last_error(None)


def test_ball_pass_domains_hold_cell_words_not_claims():
    """The slab pass keeps a 64-bit claim word and a 32-bit shell stamp per
    cell; the one-block-per-sphere pass (geometric mapping update) keeps a
    32-bit cell word and the mapping bins instead: 8 bytes per cell less,
    minus the bins (at most 4 x 10^6 bins of 17 ints)."""
    kw = dict(nx=128, ny=128, nz=128, storage=L.STORE_F32, max_spheres=500, max_radius=6.0)
    slab = L.footprint_bytes(L.default_config(map_kernel=1, **kw))
    ball = L.footprint_bytes(L.default_config(map_kernel=2, **kw))
    N = 128 ** 3
    bins = 8 * N - (slab - ball)
    assert slab > 0 and ball > 0
    assert 0 < bins <= 4 * 17 * (128 // 9) ** 3 + 4 * 256
