"""C ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2309_00651_amd import hfx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hfx.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hfx_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hfx.LIB_PATH):
        pytest.skip("libhfx.so not built")
    return hfx.load_library()


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("hfx_plan_create", "hfx_plan_destroy", "hfx_workspace_size",
              "hfx_exchange_energy", "hfx_apply_exchange", "hfx_exchange_matrix",
              "hfx_exchange_matrix_kpsi", "hfx_exchange_gradient", "hfx_orthonormalize", "hfx_ace_build",
              "hfx_ace_apply", "hfx_screen", "hfx_scdm", "hfx_schedule_info", "hfx_plan_describe",
              "hfx_status_string",
              "hfx_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s
        assert ctypes.cast(getattr(lib, s), ctypes.c_void_p).value


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        hfx.load_library(str(tmp_path / "libhfx.so"))


def _create(lib, systems, prec=hfx.FP32, opts=None):
    arr = (hfx.System * max(len(systems), 1))(*[s.to_c() for s in systems])
    h = ctypes.c_void_p()
    st = lib.hfx_plan_create(ctypes.byref(h), arr if systems else None, len(systems), prec,
                             opts)
    return st, h, lib.hfx_last_error().decode()


GOOD = hfx.SystemSpec(24, (10.0, 10.0, 10.0), 8, hfx.TRUNCATED, 0.0)


@pytest.mark.parametrize("spec,code,msg", [
    (hfx.SystemSpec(0, (10.0, 10.0, 10.0), 8), 1, "grid size"),
    (hfx.SystemSpec(24, (0.0, 10.0, 10.0), 8), 1, "box length"),
    (hfx.SystemSpec(24, (10.0, -1.0, 10.0), 8), 1, "box length"),
    (hfx.SystemSpec(24, (10.0, 10.0, 10.0), 0), 1, "n_orb"),
    (hfx.SystemSpec(24, (10.0, 10.0, 10.0), 8, 7), 1, "kernel"),
    (hfx.SystemSpec(24, (10.0, 10.0, 10.0), 8, hfx.ERFC, 0.0), 1, "w > 0"),
    (hfx.SystemSpec(98, (10.0, 10.0, 10.0), 8), 2, "not supported"),
    (hfx.SystemSpec(25, (10.0, 10.0, 10.0), 8), 2, "not supported"),
])
def test_plan_validation(lib, spec, code, msg):
    st, h, err = _create(lib, [spec])
    assert st == code and msg in err and not h.value


def test_unsupported_grid_shapes(lib):
    """n_x != n_y, and an n x n x n_z slab grid without a compiled variant,
    are rejected before any device call."""
    s = GOOD.to_c()
    s.n[2] = 32
    arr = (hfx.System * 1)(s)
    h = ctypes.c_void_p()
    assert lib.hfx_plan_create(ctypes.byref(h), arr, 1, 0, None) == 2
    assert "not supported" in lib.hfx_last_error().decode()
    s = GOOD.to_c()
    s.n[1] = s.n[0] + 8
    arr = (hfx.System * 1)(s)
    assert lib.hfx_plan_create(ctypes.byref(h), arr, 1, 0, None) == 2
    assert "n_x == n_y" in lib.hfx_last_error().decode()


def test_bad_precision_and_counts(lib):
    assert _create(lib, [GOOD], prec=5)[0] == 1
    assert _create(lib, [])[0] == 1
    h = ctypes.c_void_p()
    assert lib.hfx_plan_create(None, None, 1, 0, None) == 1
    assert lib.hfx_plan_create(ctypes.byref(h), None, 1, 0, None) == 1


def test_workspace_cap_rejected_before_device(lib, monkeypatch):
    st, h, err = _create(lib, [GOOD], opts=b"maxws=1024")
    assert st == 3 and "exceeds" in err and not h.value
    monkeypatch.setenv("HFX_MAX_WORKSPACE_BYTES", "4096")
    st, h, err = _create(lib, [GOOD])
    assert st == 3 and "exceeds" in err


def test_null_plan_calls(lib):
    vp = ctypes.c_void_p
    assert lib.hfx_plan_destroy(vp(0)) == 1
    assert lib.hfx_workspace_size(vp(0), ctypes.byref(ctypes.c_size_t())) == 1
    assert lib.hfx_exchange_energy(vp(0), vp(8), vp(8), vp(256), 0, vp(0)) == 1
    assert lib.hfx_apply_exchange(vp(0), vp(8), vp(8), vp(0), vp(256), 0, vp(0)) == 1
    assert lib.hfx_exchange_matrix(vp(0), vp(8), vp(8), vp(0), vp(256), 0, vp(0)) == 1
    assert lib.hfx_exchange_matrix_kpsi(vp(0), vp(8), vp(8), vp(8), vp(256), 0, vp(0)) == 1
    assert lib.hfx_exchange_gradient(vp(0), vp(8), vp(0), vp(8), vp(256), 0, vp(0)) == 1
    assert lib.hfx_orthonormalize(vp(0), vp(8), 0, vp(256), 0, vp(0)) == 1
    assert lib.hfx_ace_build(vp(0), vp(8), vp(8), vp(8), vp(256), 0, vp(0)) == 1
    assert lib.hfx_ace_apply(vp(0), vp(8), vp(8), vp(16), vp(256), 0, vp(0)) == 1
    assert lib.hfx_screen(vp(0), vp(8), 1e-3, None, vp(256), 0, vp(0)) == 1
    assert lib.hfx_schedule_info(vp(0), 0, None) == 1
    assert lib.hfx_plan_describe(vp(0), 0) is None
    assert lib.hfx_scdm(vp(0), vp(8), vp(8), None, vp(256), 0, vp(0)) == 1


def test_status_strings(lib):
    for code in range(5):
        assert lib.hfx_status_string(code).decode().startswith("HFX_")


@pytest.mark.parametrize("opts", [b"shard=2/2", b"shard=1", b"shard=-1/3", b"shard=0/0",
                                  b"streams=3", b"mix=0", b"mix=1.5", b"mix=abc",
                                  b"mix=0.25x", b"mix=nan", b"tiles=abc", b"tiles=-2",
                                  b"tiles=", b"maxws=1e9", b"streams=", b"tilez=3",
                                  b"tiles", b"tiles=2;bogus=1", b"rows=12", b"rows=40",
                                  b"rows=-8", b"rows=abc", b"rows=", b"ecut=0", b"ecut=-5",
                                  b"ecut=abc", b"ecut=nan", b"ecut=", b"ecut=5Ha", b"mix=",
                                  b"tune_cache=", b"rows=8,16", b"tiles=1,2", b"variant=a,b",
                                  b"variant=nope", b"check=2", b"check=x", b"check="])
def test_bad_plan_options_rejected_before_device(lib, opts):
    st, h, err = _create(lib, [GOOD], opts=opts)
    assert st == 1 and not h.value and err


def test_autotune_argument_errors_before_device(lib):
    vp = ctypes.c_void_p
    arr = (hfx.System * 1)(GOOD.to_c())
    buf = ctypes.create_string_buffer(64)
    assert lib.hfx_autotune(None, 1, 0, None, vp(8), 1, None, buf, 64, vp(0)) == 1
    assert lib.hfx_autotune(arr, 0, 0, None, vp(8), 1, None, buf, 64, vp(0)) == 1
    assert lib.hfx_autotune(arr, 1, 0, None, vp(0), 1, None, buf, 64, vp(0)) == 1
    assert lib.hfx_autotune(arr, 1, 7, None, vp(8), 1, None, buf, 64, vp(0)) == 1
    assert lib.hfx_autotune(arr, 1, 0, b"rows=8", vp(8), 1, None, buf, 64, vp(0)) == 1
    assert "chooses" in lib.hfx_last_error().decode()
