"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, agrees with the binding on the config layout, and validates
configurations on the host before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1206_6152_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _built():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1206_6152_amd import build
        build.build()
    return _lib.lib()


def _declared():
    text = open(os.path.join(ROOT, "include", "vp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _built()
    for name in _declared():
        assert hasattr(L, name), name


def test_config_layout_matches():
    L = _built()
    assert L.vp_config_size() == ctypes.sizeof(_lib.vp_config)


def _good():
    return _lib.make_config((8, 8, 8), (16, 16, 16), (1, 1, 1), (-1, -1, -1), (1, 1, 1))


def test_validate_accepts_good_config():
    _built()
    assert _lib.vp_config_validate(_good()) == _lib.VP_OK
    c = _good()
    c.bc = _lib.VP_BC_ISOLATED
    c.dtype = _lib.VP_F64
    assert _lib.vp_config_validate(c) == _lib.VP_OK


@pytest.mark.parametrize("field,value,code", [
    ("n", (0, 8, 8), _lib.VP_EINVAL),
    ("nv", (16, -1, 16), _lib.VP_EINVAL),
    ("n", (10, 8, 8), _lib.VP_EUNSUPPORTED),
    ("nv", (16, 16, 20), _lib.VP_EUNSUPPORTED),
    ("L", (1, 0, 1), _lib.VP_EINVAL),
    ("L", (1, float("nan"), 1), _lib.VP_EINVAL),
    ("vmax", (1, -1, 1), _lib.VP_EINVAL),
    ("G", -1.0, _lib.VP_EINVAL),
    ("bc", 7, _lib.VP_EINVAL),
    ("dtype", 2, _lib.VP_EINVAL),
    ("flags", 1, _lib.VP_EINVAL),
])
def test_validate_rejects(field, value, code):
    _built()
    c = _good()
    if isinstance(value, tuple):
        arr = getattr(c, field)
        for i, v in enumerate(value):
            arr[i] = v
    else:
        setattr(c, field, value)
    assert _lib.vp_config_validate(c) == code
    assert _lib.vp_last_error() != ""


def test_isolated_needs_equal_spacing():
    _built()
    c = _good()
    c.bc = _lib.VP_BC_ISOLATED
    c.L[1] = 2.0
    assert _lib.vp_config_validate(c) == _lib.VP_EUNSUPPORTED


def test_init_rejects_null_pointers_before_device_work():
    L = _built()
    c = _good()
    ctx = ctypes.c_void_p()
    assert L.vp_init(ctypes.byref(c), None, None, ctypes.byref(ctx)) == _lib.VP_EINVAL
    assert ctx.value is None
    assert L.vp_init(ctypes.byref(c), ctypes.c_void_p(1), None, None) == _lib.VP_EINVAL
    assert L.vp_init(None, ctypes.c_void_p(1), None, ctypes.byref(ctx)) == _lib.VP_EINVAL


def test_calls_reject_null_context():
    L = _built()
    assert L.vp_step(None, 0.1) == _lib.VP_EINVAL
    assert L.vp_sweep(None, 0, 0.1) == _lib.VP_EINVAL
    assert L.vp_free(None) == _lib.VP_OK
    with pytest.raises(_lib.VPError):
        _lib.vp_step(None, 0.1)


@pytest.mark.parametrize("src,dst,nbytes,why", [
    (0, 4096, 64, "null"), (4096, 0, 64, "null"),
    (4096, 8192, 24, "multiple of 16"), (4096, 8192, -16, "multiple of 16"),
    (4104, 8192, 64, "aligned"), (4096, 8200, 64, "aligned"),
    (4096, 4112, 64, "overlap"), (4112, 4096, 64, "overlap"), (4096, 4096, 16, "overlap")])
def test_stream_copy_rejects_bad_arguments_before_device_work(src, dst, nbytes, why):
    # the addresses are never dereferenced: every case fails host validation
    _built()
    with pytest.raises(_lib.VPError) as e:
        _lib.vp_stream_copy(src, dst, nbytes, 0)
    assert e.value.code == _lib.VP_EINVAL and why in str(e.value)


@pytest.mark.parametrize("d", [(1.0, 1.0, 1.0), (0.75, 0.75, 0.75), (1.0, 2.0, 0.5), (0.3, 1.7, 1.1), (1e-3, 1.0, 1.0)])
def test_cell_self_integral_matches_the_oracles_closed_form(orc, d):
    # Two independent derivations of the isolated kernel's self term (Sec. 2.2):
    # the library's divergence-theorem quadrature (host code, no device) and
    # the oracle's closed form for a box seen from a corner.
    _built()
    got = _lib.vp_cell_self_integral(*d)
    np.testing.assert_allclose(got, orc.cell_self_integral(*d), rtol=1e-13)
    # scaling: the integral of 1/|r| over a volume scales as length^2
    np.testing.assert_allclose(_lib.vp_cell_self_integral(*(3 * x for x in d)), 9 * got, rtol=1e-13)


def test_cell_self_integral_rejects_bad_widths():
    _built()
    for d in [(0.0, 1.0, 1.0), (1.0, -1.0, 1.0), (1.0, 1.0, float("nan")), (float("inf"), 1.0, 1.0)]:
        assert np.isnan(_lib.vp_cell_self_integral(*d))
        assert "widths" in _lib.vp_last_error()
    assert np.isfinite(_lib.vp_cell_self_integral(1.0, 1.0, 1.0)) and _lib.vp_last_error() == ""
