"""GPU parity of the options beyond the paper's scheme: zonally periodic rows
(RF_PERIODIC_X) and exact end conditions (RF_EXACT_ENDS), against the FP64
oracle with the same flags.

Periodic grids have all-sea rows (cyclic lines, solved by one fixed point per
line), rows whose sea runs wrap from x = nx-1 to x = 0, and row lengths that
fill the x tile exactly or leave padding in the last chunk.  Every path is
checked: the tiled FP32 kernels (field-wide relative L2 1e-5 and line by line;
2-D and per-level tables), the line-sequential FP32 kernels (RF3_SEQUENTIAL=1), FP64
(1e-12), the 1st-RF (FP64), forward and adjoint, in place.
"""
import os

import numpy as np
import pytest
import torch

from paper_1404_5756_amd import synth
from paper_1404_5756_amd.operator import HorizontalCovariance
from parity_util import assert_lines

pytestmark = pytest.mark.gpu
TOL32, TOL64 = 1e-5, 1e-12


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def periodic_case(seed, ny, nx, nlev, mask_3d=False, sigma=(1.5, 12.0)):
    w = synth.random_case(seed, ny, nx, nlev, 0.3, 4, sigma, 3.0, "fit", mask_3d, False)
    m = w.mask.copy()
    m[:, 1::7, :] = 1                       # all-sea rows: cyclic lines
    m[:, 3::5, :3] = 1                      # sea at both ends of the row: runs that wrap
    m[:, 3::5, -3:] = 1
    m[:, 4::9, :] = 0                       # all-land rows
    w.mask = m
    return w


PCASES = [
    # seed, ny, nx, nlev, 3-D mask: x tiles of 23 (1440 = 64*22.5: padding), 23 (1472 = 64*23: none),
    # 1 (nx = 50), 33 (2100), and per-level masks (per-level tables: x tiles of 5 and 23)
    (41, 40, 1440, 2, False),
    (42, 33, 1472, 2, False),
    (43, 30, 50, 3, False),
    (44, 21, 2100, 1, False),
    (45, 35, 300, 3, True),
    (46, 48, 1440, 3, True),
]


@pytest.fixture(scope="module", params=PCASES, ids=lambda c: f"per_s{c[0]}_{c[2]}x{c[1]}x{c[3]}")
def pcase(request, orc):
    seed, ny, nx, nlev, m3 = request.param
    w = periodic_case(seed, ny, nx, nlev, m3)
    P = orc.Problem(w.mask, w.sigma_x, w.sigma_y, n_img=w.n_img, qmode=orc.QMODES[w.qmode], k1=5,
                    flags=orc.PERIODIC_X)
    op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, k1=5,
                              periodic_x=True)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((2, nlev, ny, nx))
    print(f"periodic case {w.name}", flush=True)
    return w, P, op, x


def test_periodic_fp32(pcase):
    w, P, op, x = pcase
    x32 = x.astype(np.float32)
    for name, fn, ref in (("forward", op.apply, P.rf3), ("adjoint", op.adjoint, P.rf3_adjoint)):
        r = ref(x32.astype(np.float64))
        got = fn(torch.from_numpy(x32).cuda()).cpu().numpy()
        e = rel(got, r)
        lr = assert_lines(got, r, f"{w.name} periodic fp32 {name}")
        print(f"  fp32 {name}: rel {e:.2e}, worst line {lr:.3f}", flush=True)
        assert e <= TOL32


def test_periodic_fp32_sequential_kernels(pcase, monkeypatch):
    w, P, op, x = pcase
    monkeypatch.setenv("RF3_SEQUENTIAL", "1")
    x32 = x.astype(np.float32)
    for fn, ref in ((op.apply, P.rf3), (op.adjoint, P.rf3_adjoint)):
        r = ref(x32.astype(np.float64))
        got = fn(torch.from_numpy(x32).cuda()).cpu().numpy()
        assert rel(got, r) <= TOL32
        assert_lines(got, r, f"{w.name} periodic fp32 sequential")


def test_periodic_fp64_and_rf1(pcase):
    w, P, op, x = pcase
    xd = torch.from_numpy(x).cuda()
    assert rel(op.apply(xd).cpu().numpy(), P.rf3(x)) <= TOL64
    assert rel(op.adjoint(xd).cpu().numpy(), P.rf3_adjoint(x)) <= TOL64
    assert rel(op.rf1(xd, K=5).cpu().numpy(), P.rf1(x, K=5)) <= TOL64


def test_periodic_in_place_and_y_unchanged(pcase):
    w, P, op, x = pcase
    x32 = torch.from_numpy(x.astype(np.float32)).cuda()
    ref = op.apply(x32)
    y = x32.clone()
    op.apply(y, out=y)
    assert torch.equal(y, ref)
    # columns are not periodic: G_y is the same with or without the flag
    op0 = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, k1=5)
    assert torch.equal(op.apply_dir(x32, "y"), op0.apply_dir(x32, "y"))
    # and rows are: the x direction differs where a run wraps or a row has no land
    assert not torch.equal(op.apply_dir(x32, "x"), op0.apply_dir(x32, "x"))


def test_periodic_constant_field_all_sea_uniform_sigma(orc):
    """All sea, uniform sigma, periodic rows: a constant field's x pass is c sqrt(2 pi) sigma at every
    point (no ends), to FP32 and FP64 precision."""
    ny, nx, s = 8, 1440, 6.0
    mask = np.ones((1, ny, nx), np.uint8)
    sig = np.full((1, ny, nx), s)
    op = HorizontalCovariance(mask, sig, sig, 1, n_img=0, qmode="fit", periodic_x=True)
    for dt, tol in ((torch.float32, 2e-6), (torch.float64, 1e-12)):
        c = torch.full((1, ny, nx), 1.25, dtype=dt, device="cuda")
        out = op.apply_dir(c, "x").double().cpu().numpy()
        np.testing.assert_allclose(out, 1.25 * np.sqrt(2 * np.pi) * s, rtol=tol)


# ---------------------------------------------------------------- exact end conditions
# Per-line FP32 bound with exact ends.  The end correction injects the infinite
# line's tail, which for large sigma dominates a short segment's output and is a
# strongly cancelling combination of the end state: an FP32 emulation of the
# kernels' arithmetic against the oracle gives 1-D errors up to 6.6e-6 on
# segments of 4-14 points at sigma <= 12 (2.8e-6 on longer ones).  Two such
# passes (x, y) per line: 3e-5 per line; the field-wide bound stays 1e-5.
TOL_LINE_END = 3e-5
# FP64 with exact ends: the oracle and the FP64 kernels both run the printed
# (direct) recurrence, whose rounding at sigma = 12 is already ~1e-13 without end
# conditions; the injected tail on segments of a few points adds about one more
# digit (measured 1.9e-12 between the two on a 50 x 14 grid).  Bound: 1e-11.
TOL64_END = 1e-11

ECASES = [
    # seed, ny, nx, nlev, 3-D mask, periodic: tiles x 23 / y 45 (two planes per lane), x 33 / y 56 (one
    # plane), x 1 / y 1 (one point per lane, one row per wave), a per-level mask (per-level tables), and
    # periodic rows with exact ends (sequential FP32)
    (51, 720, 1440, 3, False, False),
    (52, 801, 2112, 1, False, False),
    (53, 14, 50, 2, False, False),
    (54, 97, 131, 3, False, False),
    (55, 60, 300, 3, True, False),
    (56, 40, 500, 2, False, True),
]


@pytest.fixture(scope="module", params=ECASES, ids=lambda c: f"end_s{c[0]}_{c[2]}x{c[1]}x{c[3]}")
def ecase(request, orc):
    seed, ny, nx, nlev, m3, per = request.param
    w = synth.random_case(seed, ny, nx, nlev, 0.3, 4, (1.5, 12.0), 3.0, "fit", m3, False)
    if per:
        w = periodic_case(seed, ny, nx, nlev, m3)
    flags = orc.EXACT_ENDS | (orc.PERIODIC_X if per else 0)
    P = orc.Problem(w.mask, w.sigma_x, w.sigma_y, n_img=w.n_img, qmode=orc.QMODES[w.qmode], k1=5, flags=flags)
    op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, k1=5,
                              exact_ends=True, periodic_x=per)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((1, nlev, ny, nx))
    print(f"exact-ends case {w.name} periodic={per}", flush=True)
    return w, P, op, x


def test_exact_ends_fp32(ecase, monkeypatch):
    """Tiled and line-sequential FP32 paths against the oracle (field-wide 1e-5, per line
    TOL_LINE_END), and against each other line by line (two independent implementations
    of the end correction: a slip in either shows as a line far outside rounding)."""
    w, P, op, x = ecase
    x32 = x.astype(np.float32)
    for name, fn, ref in (("forward", op.apply, P.rf3), ("adjoint", op.adjoint, P.rf3_adjoint)):
        r = ref(x32.astype(np.float64), threads=16)
        monkeypatch.delenv("RF3_SEQUENTIAL", raising=False)
        got = fn(torch.from_numpy(x32).cuda()).cpu().numpy()
        monkeypatch.setenv("RF3_SEQUENTIAL", "1")
        seq = fn(torch.from_numpy(x32).cuda()).cpu().numpy()
        monkeypatch.delenv("RF3_SEQUENTIAL")
        e, es = rel(got, r), rel(seq, r)
        lr = assert_lines(got, r, f"{w.name} exact ends fp32 {name}", TOL_LINE_END)
        ls = assert_lines(seq, r, f"{w.name} exact ends fp32 sequential {name}", TOL_LINE_END)
        lt = assert_lines(got, seq, f"{w.name} exact ends tiled vs sequential {name}", TOL_LINE_END)
        print(f"  fp32 {name}: rel {e:.2e} (sequential {es:.2e}); worst line {lr:.3f} / {ls:.3f} "
              f"(tiled vs sequential {lt:.3f}) of allowance", flush=True)
        assert e <= TOL32 and es <= TOL32


def test_exact_ends_fp64(ecase):
    w, P, op, x = ecase
    xd = torch.from_numpy(x).cuda()
    ef = rel(op.apply(xd).cpu().numpy(), P.rf3(x, threads=16))
    ea = rel(op.adjoint(xd).cpu().numpy(), P.rf3_adjoint(x, threads=16))
    print(f"  fp64: forward {ef:.2e}, adjoint {ea:.2e}", flush=True)
    assert ef <= TOL64_END and ea <= TOL64_END


def test_exact_ends_leave_rf1_and_differ_from_zero_ends(ecase):
    w, P, op, x = ecase
    per = bool(P.flags & 1)
    op0 = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, k1=5,
                               periodic_x=per)
    xd = torch.from_numpy(x).cuda()
    assert torch.equal(op.rf1(xd, K=5), op0.rf1(xd, K=5))
    x32 = xd.float()
    assert not torch.equal(op.apply(x32), op0.apply(x32))


def test_exact_ends_uniform_sigma_diagonal_is_flat_on_the_gpu():
    """Uniform sigma, one all-sea row: with exact ends the x operator's diagonal is the same at
    both ends of the row as inside it (FP64 path)."""
    nx, s = 61, 4.0
    mask = np.ones((1, 1, nx), np.uint8)
    sig = np.full((1, 1, nx), s)
    op = HorizontalCovariance(mask, sig, sig, 1, n_img=0, qmode="fit", exact_ends=True)
    E = torch.eye(nx, dtype=torch.float64, device="cuda").reshape(nx, 1, 1, nx)
    G = op.apply_dir(E, "x").reshape(nx, nx).cpu().numpy().T
    d = np.diag(G)
    assert np.ptp(d) <= 1e-12 * d.max()
    np.testing.assert_allclose(G, G.T, atol=1e-12 * d.max())
