"""Host-side batch work list (rf3_batch_plan): sizes, header, unit counts, errors.

Runs without a GPU: the plan is built from the grids and the block layout
only, so fake (aligned) device addresses are enough.
"""
import ctypes
import struct

import pytest

from paper_1404_5756_amd import rf3

FAKE = 1 << 40   # aligned fake device addresses, never dereferenced


def _item(k, nx, ny, nlev, nfields=1, mask_nlev=1, sigma_nlev=1, in_place=False):
    g = rf3.make_grid(nx, ny, nlev, mask_nlev, sigma_nlev, 4, "fit", 5)
    coef = FAKE + k * (1 << 32)
    inp = FAKE + (1 << 36) + k * (1 << 32)
    out = inp if in_place else inp + (1 << 31)
    return (g, coef, inp, out, nfields)


def _x_groups(ny, nplanes, gmax=8, cus=256):
    """Workgroups per x row (the library's rule; without a GPU the library assumes 256 CUs)."""
    groups = 1
    while groups * 2 <= gmax and ((ny + 7) // 8) * 8 * groups < 2 * cus and groups * 4 * 2 <= nplanes:
        groups *= 2
    return groups


def _tile_lx(nx):
    return ((nx + 63) // 64) | 1


def _tile_ly(ny):
    need = (ny + 15) // 16
    return next(o for o in (1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 28, 32, 36, 40, 45, 48, 56, 64) if o >= need)


def _expected_units(items):
    """Units per (direction, tile size) group before the per-XCD padding."""
    groups = {}
    for g, _c, _i, _o, nf in items:
        if g.mask_nlev != 1 or g.sigma_nlev != 1:
            continue
        nplanes = g.nlev * nf
        groups.setdefault((0, _tile_lx(g.nx)), 0)
        groups[(0, _tile_lx(g.nx))] += g.ny * _x_groups(g.ny, nplanes)
        ly = _tile_ly(g.ny)
        groups.setdefault((1, ly), 0)
        groups[(1, ly)] += -(-g.nx // 64) * -(-nplanes // 8)   # units of up to 8 planes
    return groups


def test_plan_header_and_unit_count():
    items = [_item(0, 300, 200, 7), _item(1, 1440, 720, 50), _item(2, 130, 130, 1, nfields=2, in_place=True),
             _item(3, 200, 100, 3, mask_nlev=3)]
    nb = rf3.rf3_batch_plan_bytes(items)
    assert nb > 0 and nb % 256 == 0
    buf = rf3.rf3_batch_plan(items)
    magic, version, n_items, n_units, off_e, off_u, total = struct.unpack_from("<IIiiQQQ", buf, 0)
    assert magic == 0x50424652 and version == 3
    assert n_items == len(items) and total == nb == len(buf)
    exp = _expected_units(items)
    lo = sum(exp.values())
    # each group is padded with idle units to whole rounds of 8 (one unit per XCD)
    assert n_units >= lo and n_units % 8 == 0
    assert off_e == 64 and off_u % 256 == 0 and off_u + 16 * n_units <= total
    # entry 1 (1440 x 720 x 50): pointers and sizes as given
    # in, out, T[2], KY, LM[2], PHI[2], PER, END[2], sizes
    e = struct.unpack_from("<QQ10Qiiii", buf, off_e + 1 * 112)
    assert e[0] == items[1][2] and e[1] == items[1][3]
    assert e[12:15] == (1440, 720, 50)
    # the 3-D-mask item runs the sequential path: no units reference it
    units = [struct.unpack_from("<iiii", buf, off_u + 16 * k) for k in range(n_units)]
    assert all(u[0] != 3 for u in units)
    real = [u for u in units if u[0] >= 0]
    assert len(real) == lo


def test_units_cover_every_row_and_plane_once():
    items = [_item(0, 257, 131, 5), _item(1, 70, 801, 3), _item(2, 1100, 40, 1, nfields=3)]
    buf = rf3.rf3_batch_plan(items)
    _m, _v, _n, n_units, _oe, off_u, _t = struct.unpack_from("<IIiiQQQ", buf, 0)
    units = [struct.unpack_from("<iiii", buf, off_u + 16 * k) for k in range(n_units)]
    real = [u for u in units if u[0] >= 0]
    # all x units precede all y units
    nx_units = sum(g.ny * _x_groups(g.ny, g.nlev * nf) for g, _c, _i, _o, nf in items)
    xu, yu = real[:nx_units], real[nx_units:]
    for k, (g, _c, _i, _o, nf) in enumerate(items):
        groups = _x_groups(g.ny, g.nlev * nf)
        rows = sorted((u[1], u[2]) for u in xu if u[0] == k)
        assert rows == [(r, q) for r in range(g.ny) for q in range(groups)]
        assert all(u[3] == groups for u in xu if u[0] == k)
        # y units: {item, column block, first plane, end plane}
        cover = sorted((u[1], q) for u in yu if u[0] == k for q in range(u[2], u[3]))
        assert cover == [(b, q) for b in range(-(-g.nx // 64)) for q in range(g.nlev * nf)]
    # largest tiles first in each direction: a launch's short units come last and fill its final round
    lxs = [_tile_lx(items[u[0]][0].nx) for u in xu]
    lys = [_tile_ly(items[u[0]][0].ny) for u in yu]
    assert lxs == sorted(lxs, reverse=True) and len(set(lxs)) == 3
    assert lys == sorted(lys, reverse=True) and len(set(lys)) == 3


def test_plan_errors():
    assert rf3.rf3_batch_plan_bytes([]) == 0
    bad = rf3.make_grid(0, 10, 1)
    assert rf3.rf3_batch_plan_bytes([(bad, FAKE, FAKE, FAKE + (1 << 30), 1)]) == 0
    # misaligned coefficient block
    g = rf3.make_grid(64, 64, 1)
    assert rf3.rf3_batch_plan_bytes([(g, FAKE + 16, FAKE, FAKE + (1 << 30), 1)]) == 0
    # overlapping in/out
    assert rf3.rf3_batch_plan_bytes([(g, FAKE, FAKE + (1 << 34), FAKE + (1 << 34) + 4, 1)]) == 0
    items = [_item(0, 100, 100, 2)]
    nb = rf3.rf3_batch_plan_bytes(items)
    arr, _keep = rf3._items(items)
    small = ctypes.create_string_buffer(nb - 256)
    assert rf3.lib().rf3_batch_plan(arr, 1, small, nb - 256) == rf3.RF_E_ARG
    # wrong plan size at apply: refused before anything is enqueued
    assert rf3.lib().rf3_apply_batch(arr, 1, rf3.RF_FP32, 0, ctypes.c_void_p(FAKE), nb + 256, None) == rf3.RF_E_ARG
    with pytest.raises(rf3.RFError):
        rf3.rf3_batch_plan([])


def test_tuning_shapes_the_work_list():
    g = rf3.make_grid(300, 200, 7)
    items = [(g, FAKE, FAKE + (1 << 36), FAKE + (1 << 36) + (1 << 31), 3)]   # 21 planes
    nplanes = 21
    for xg, yp in ((1, 1), (2, 5), (4, 21), (16, 64), (3, 8)):
        buf = rf3.rf3_batch_plan(items, (xg, yp))
        _m, _v, _n, n_units, _oe, off_u, _t = struct.unpack_from("<IIiiQQQ", buf, 0)
        units = [struct.unpack_from("<iiii", buf, off_u + 16 * k) for k in range(n_units)]
        real = [u for u in units if u[0] >= 0]
        cap = 1 << (xg.bit_length() - 1)     # the largest power of two not above x_groups_max
        groups = _x_groups(200, nplanes, cap)
        xu = [u for u in real[:200 * groups]]
        assert sorted((u[1], u[2]) for u in xu) == [(r, q) for r in range(200) for q in range(groups)]
        yu = real[200 * groups:]
        nblk = -(-300 // 64)
        assert len(yu) == nblk * -(-nplanes // yp)
        assert all(u[3] - u[2] <= yp for u in yu)
        cover = sorted((u[1], q) for u in yu for q in range(u[2], u[3]))
        assert cover == [(b, q) for b in range(nblk) for q in range(nplanes)]


def test_tuning_out_of_range_is_refused():
    g = rf3.make_grid(64, 64, 2)
    items = [(g, FAKE, FAKE + (1 << 36), FAKE + (1 << 36) + (1 << 31), 1)]
    for t in ((-1, 0), (0, -1), (65, 0), (0, 4097), (0, 0, 2), (0, 0, -1)):
        assert rf3.rf3_batch_plan_bytes(items, t) == 0
        with pytest.raises(rf3.RFError):
            rf3.rf3_batch_plan(items, t)
    assert rf3.rf3_batch_plan_bytes(items, (0, 0)) == rf3.rf3_batch_plan_bytes(items)
    # one x launch changes the launches, not the work list
    assert rf3.rf3_batch_plan(items, (0, 0, 1)) == rf3.rf3_batch_plan(items)
    arr, _keep = rf3._items(items)
    bad = rf3.rf_batch_tuning(0, -3)
    assert rf3.lib().rf3_apply_batch_ex(arr, 1, ctypes.byref(bad), rf3.RF_FP32, 0, ctypes.c_void_p(FAKE), 256,
                                        None) == rf3.RF_E_ARG


def test_tuning_struct_matches_the_header():
    """rf_batch_tuning is three int32 fields (x_groups_max, y_planes, x_one_launch) in
    include/rf3.h; the binding's struct must have the same size and order, and a
    (x_groups_max, y_planes) pair means x_one_launch = 0."""
    import re
    from pathlib import Path
    hdr = (Path(__file__).resolve().parents[1] / "include" / "rf3.h").read_text()
    body = hdr[:hdr.index("} rf_batch_tuning;")]
    body = body[body.rindex("typedef struct {"):]
    fields = re.findall(r"int32_t\s+(\w+);", body)
    assert fields == [f for f, _ in rf3.rf_batch_tuning._fields_]
    assert ctypes.sizeof(rf3.rf_batch_tuning) == 4 * len(fields)
    t = rf3._tuning((4, 6))
    assert (t.x_groups_max, t.y_planes, t.x_one_launch) == (4, 6, 0)
    t = rf3._tuning((1, 2, 1))
    assert (t.x_groups_max, t.y_planes, t.x_one_launch) == (1, 2, 1)
