"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/rf3.h, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rf3.h")


@pytest.fixture(scope="module")
def rf3():
    from paper_1404_5756_amd import rf3 as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1404_5756_amd import build
        build.build()
    m.lib()
    return m


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rf\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("rf_coeffs_bytes", "rf_coeffs", "rf3_apply_xy", "rf3_adjoint_xy", "rf3_apply_dir", "rf1_apply_xy",
              "rf3_batch_plan_bytes", "rf3_batch_plan", "rf3_apply_batch", "rf_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol(rf3):
    L = rf3.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_strerror(rf3):
    for s in (0, -1, -2, -3, -4, -5):
        assert len(rf3.rf_strerror(s)) > 5
    assert rf3.rf_strerror(-99) == "unknown status"


def test_coeffs_bytes_validates_grid(rf3):
    L = rf3.lib()
    g = rf3.make_grid(100, 50, 10)
    n = L.rf_coeffs_bytes(ctypes.byref(g))
    assert n > 100 * 50 * (16 * 3 + 32 + 16) * 2
    assert n % 256 == 0
    for bad in (rf3.make_grid(0, 5, 1), rf3.make_grid(5, 5, 0), rf3.make_grid(5, 5, 3, mask_nlev=2),
                rf3.make_grid(5, 5, 3, sigma_nlev=4), rf3.make_grid(5, 5, 1, n_img=-1),
                rf3.make_grid(5, 5, 1, n_img=65), rf3.make_grid(5, 5, 1, qmode=3),
                rf3.make_grid(5, 5, 1, k1=0), rf3.make_grid(70000, 5, 1)):
        assert L.rf_coeffs_bytes(ctypes.byref(bad)) == 0
    assert L.rf_coeffs_bytes(None) == 0
    # 3-D sigma and mask make the tables per level
    g3 = rf3.make_grid(100, 50, 10, mask_nlev=10, sigma_nlev=10)
    assert L.rf_coeffs_bytes(ctypes.byref(g3)) > 10 * 100 * 50 * (16 * 3 + 32 + 16) * 2


FAKE = 0x7f0000000000  # never dereferenced: every call below fails its host-side checks


def test_apply_argument_errors(rf3):
    L = rf3.lib()
    g = rf3.make_grid(64, 32, 4)
    gp = ctypes.byref(g)
    E_ARG, E_SHAPE = rf3.RF_E_ARG, rf3.RF_E_SHAPE
    for fn in (L.rf3_apply_xy, L.rf3_adjoint_xy):
        assert fn(None, FAKE, 0, FAKE, FAKE + 10 ** 7, 4, 1, None) == E_ARG
        assert fn(gp, None, 0, FAKE, FAKE + 10 ** 7, 4, 1, None) == E_ARG
        assert fn(gp, FAKE, 0, None, FAKE + 10 ** 7, 4, 1, None) == E_ARG
        assert fn(gp, FAKE, 0, FAKE, None, 4, 1, None) == E_ARG
        assert fn(gp, FAKE, 2, FAKE, FAKE + 10 ** 7, 4, 1, None) == E_ARG          # bad precision
        assert fn(gp, FAKE, 0, FAKE, FAKE + 10 ** 7, 5, 1, None) == E_SHAPE        # nlev > g.nlev
        assert fn(gp, FAKE, 0, FAKE, FAKE + 10 ** 7, 0, 1, None) == E_SHAPE
        assert fn(gp, FAKE, 0, FAKE, FAKE + 10 ** 7, 4, 0, None) == E_SHAPE
        assert fn(gp, FAKE + 8, 0, FAKE, FAKE + 10 ** 7, 4, 1, None) == E_ARG      # coef not 256-aligned
        assert fn(gp, FAKE, 0, FAKE + 2, FAKE + 10 ** 7, 4, 1, None) == E_ARG      # misaligned field
        # partial overlap of in and out (FP32 field of 64*32*4*4 bytes)
        assert fn(gp, FAKE, 0, FAKE, FAKE + 4 * 100, 4, 1, None) == E_ARG
        assert fn(gp, FAKE, 1, FAKE, FAKE + 64 * 32 * 4 * 4, 4, 1, None) == E_ARG  # FP64 is twice as long
    bad = rf3.make_grid(64, 32, 4, qmode=7)
    assert L.rf3_apply_xy(ctypes.byref(bad), FAKE, 0, FAKE, FAKE, 4, 1, None) == E_SHAPE


def test_apply_dir_argument_errors(rf3):
    L = rf3.lib()
    g = rf3.make_grid(64, 32, 4)
    gp = ctypes.byref(g)
    assert L.rf3_apply_dir(gp, FAKE, 0, 2, 0, FAKE, FAKE + 10 ** 7, 4, 1, None) == rf3.RF_E_ARG
    assert L.rf3_apply_dir(gp, FAKE, 0, -1, 0, FAKE, FAKE + 10 ** 7, 4, 1, None) == rf3.RF_E_ARG
    assert L.rf3_apply_dir(gp, FAKE, 0, 0, 0, FAKE, FAKE + 8, 4, 1, None) == rf3.RF_E_ARG


def test_rf1_argument_errors(rf3):
    L = rf3.lib()
    g = rf3.make_grid(64, 32, 4, k1=5)
    gp = ctypes.byref(g)
    assert L.rf1_apply_xy(gp, FAKE, 1, 4, FAKE, FAKE + 10 ** 7, 4, 1, None) == rf3.RF_E_ARG    # K != k1
    assert L.rf1_apply_xy(gp, FAKE, 0, 5, FAKE, FAKE + 10 ** 7, 4, 1, None) == rf3.RF_E_UNSUPPORTED
    assert L.rf1_apply_xy(None, FAKE, 1, 5, FAKE, FAKE + 10 ** 7, 4, 1, None) == rf3.RF_E_ARG


def test_coeffs_argument_errors(rf3):
    L = rf3.lib()
    g = rf3.make_grid(64, 32, 4)
    gp = ctypes.byref(g)
    assert L.rf_coeffs(None, FAKE, FAKE, FAKE, FAKE, None) == rf3.RF_E_ARG
    assert L.rf_coeffs(gp, None, FAKE, FAKE, FAKE, None) == rf3.RF_E_ARG
    assert L.rf_coeffs(gp, FAKE, FAKE, FAKE, FAKE + 16, None) == rf3.RF_E_ARG
    bad = rf3.make_grid(64, 32, 4, n_img=100)
    assert L.rf_coeffs(ctypes.byref(bad), FAKE, FAKE, FAKE, FAKE, None) == rf3.RF_E_SHAPE


def test_harness_argument_errors(rf3):
    L = rf3.lib()
    # null plan / output, bad precision: refused before any launch
    assert L.rf_obs_innovation(None, 10, 10, 100, rf3.RF_FP32, None, None, None, 1.0, None, None, None) == rf3.RF_E_ARG
    assert L.rf_obs_innovation(ctypes.c_void_p(1 << 40), 10, 10, 100, 7, None, None, None, 1.0, None,
                               ctypes.c_void_p(1 << 40), None) == rf3.RF_E_ARG
    assert L.rf_obs_innovation(ctypes.c_void_p((1 << 40) + 16), 10, 10, 100, rf3.RF_FP32, None, None, None, 1.0,
                               None, ctypes.c_void_p(1 << 40), None) == rf3.RF_E_ARG   # misaligned plan
    assert L.rf_axpy(rf3.RF_FP32, 0, 1.0, ctypes.c_void_p(1 << 40), ctypes.c_void_p(1 << 40), None) == rf3.RF_E_ARG
    assert L.rf_axpy(rf3.RF_FP32, 10, 1.0, None, ctypes.c_void_p(1 << 40), None) == rf3.RF_E_ARG
    assert L.rf_axpy(5, 10, 1.0, ctypes.c_void_p(1 << 40), ctypes.c_void_p(1 << 40), None) == rf3.RF_E_ARG
