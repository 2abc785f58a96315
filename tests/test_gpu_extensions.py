"""GPU parity of the options beyond the paper's scheme: zonally periodic rows
(RF_PERIODIC_X) and exact end conditions (RF_EXACT_ENDS), against the FP64
oracle with the same flags.

Periodic grids have all-sea rows (cyclic lines, solved by one fixed point per
line), rows whose sea runs wrap from x = nx-1 to x = 0, and row lengths that
fill the x tile exactly or leave padding in the last chunk.  Every path is
checked: the tiled FP32 kernels (field-wide relative L2 1e-5 and line by line),
the line-sequential FP32 kernels (RF3_SEQUENTIAL=1, and per-level masks), FP64
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
    # 1 (nx = 50), 33 (2100), and a per-level mask (sequential FP32 path)
    (41, 40, 1440, 2, False),
    (42, 33, 1472, 2, False),
    (43, 30, 50, 3, False),
    (44, 21, 2100, 1, False),
    (45, 35, 300, 3, True),
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
