"""Parity at the full workload sizes, in the launch configuration bench.py times.

C3 (1440 x 720 x 50, forward and adjoint), C2 (871 x 253 x 72, T and S,
forward and adjoint) and the C4 batch (64 grids, autotuned work list, hipGraph replay)
against the FP64 C oracle.  C3 and C2 are compared at every output point (the
oracle runs them in seconds with OpenMP), as one field-wide relative L2 and
line by line (every x-row and y-column of every plane, parity_util); the C4
batch is compared with the per-item calls bitwise for all 64 grids and with the
oracle on a spread of eight of them.  Tolerance: relative L2 1e-5 (FP32 path).
"""
import os

import numpy as np
import pytest
import torch

from paper_1404_5756_amd import synth
from paper_1404_5756_amd.operator import Batch, HorizontalCovariance
from parity_util import assert_lines

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
THREADS = min(16, os.cpu_count() or 1)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _op(w, dev):
    return HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, device=dev)


def _problem(orc, w):
    return orc.Problem(w.mask, w.sigma_x, w.sigma_y, n_img=w.n_img, qmode=orc.QMODES[w.qmode], k1=5)


def test_c3_forward_and_adjoint_full(orc):
    dev = torch.device("cuda:0")
    w = synth.c3_global()
    xh = w.field(np.float32)                       # the bench's input
    x = torch.from_numpy(xh).to(dev)
    op = _op(w, dev)
    f = op.apply(x)
    a = op.adjoint(x)
    torch.cuda.synchronize()
    P = _problem(orc, w)
    x64 = xh.astype(np.float64)
    fr, ar = P.rf3(x64, threads=THREADS), P.rf3_adjoint(x64, threads=THREADS)
    fg, ag = f.double().cpu().numpy(), a.double().cpu().numpy()
    ef, ea = rel(fg, fr), rel(ag, ar)
    lf, la = assert_lines(fg, fr, "C3 forward"), assert_lines(ag, ar, "C3 adjoint")
    print(f"C3 full: fwd rel L2 {ef:.3e}, adj rel L2 {ea:.3e}; worst line {lf:.3f} / {la:.3f} of allowance",
          flush=True)
    assert ef < TOL32 and ea < TOL32


@pytest.mark.parametrize("variant", ["anisotropic", "periodic_x", "exact_ends", "depth"])
def test_c3_variants_full(orc, variant):
    """C3 with anisotropic, inhomogeneous length scales (zonal twice meridional at the equator),
    with zonally periodic rows, with exact end conditions, and with a depth-dependent mask and
    sigma (one plane per level: the line-sequential FP32 kernels): forward and adjoint at every
    point, field-wide and line by line (exact ends: its stated per-line bound)."""
    dev = torch.device("cuda:0")
    w = {"anisotropic": synth.c3_anisotropic, "depth": synth.c3_depth}.get(variant, synth.c3_global)()
    kw = {"periodic_x": variant == "periodic_x", "exact_ends": variant == "exact_ends"}
    flags = (orc.PERIODIC_X if kw["periodic_x"] else 0) | (orc.EXACT_ENDS if kw["exact_ends"] else 0)
    xh = w.field(np.float32)
    x = torch.from_numpy(xh).to(dev)
    op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, device=dev, **kw)
    f = op.apply(x)
    a = op.adjoint(x)
    torch.cuda.synchronize()
    P = orc.Problem(w.mask, w.sigma_x, w.sigma_y, n_img=w.n_img, qmode=orc.QMODES[w.qmode], k1=5, flags=flags)
    x64 = xh.astype(np.float64)
    fr, ar = P.rf3(x64, threads=THREADS), P.rf3_adjoint(x64, threads=THREADS)
    fg, ag = f.double().cpu().numpy(), a.double().cpu().numpy()
    ef, ea = rel(fg, fr), rel(ag, ar)
    tl = 3e-5 if variant == "exact_ends" else 1e-5
    lf, la = assert_lines(fg, fr, f"C3 {variant} forward", tl), assert_lines(ag, ar, f"C3 {variant} adjoint", tl)
    print(f"C3 {variant}: fwd rel L2 {ef:.3e}, adj rel L2 {ea:.3e}; worst line {lf:.3f} / {la:.3f} of allowance",
          flush=True)
    assert ef < TOL32 and ea < TOL32


def test_c2_forward_and_adjoint_full(orc):
    dev = torch.device("cuda:0")
    w = synth.c2_regional()
    xh = w.field(np.float32)                       # [2][72][253][871]
    x = torch.from_numpy(xh).to(dev)
    op = _op(w, dev)
    f = op.apply(x)
    a = op.adjoint(x)
    torch.cuda.synchronize()
    P = _problem(orc, w)
    x64 = xh.astype(np.float64)
    fr, ar = P.rf3(x64, threads=THREADS), P.rf3_adjoint(x64, threads=THREADS)
    fg, ag = f.double().cpu().numpy(), a.double().cpu().numpy()
    ef, ea = rel(fg, fr), rel(ag, ar)
    lf, la = assert_lines(fg, fr, "C2 forward"), assert_lines(ag, ar, "C2 adjoint")
    print(f"C2 full: fwd rel L2 {ef:.3e}, adj rel L2 {ea:.3e}; worst line {lf:.3f} / {la:.3f} of allowance",
          flush=True)
    assert ef < TOL32 and ea < TOL32


def test_c2_depth_full(orc):
    """C2 (T and S, 72 levels) with a depth-dependent mask and sigma: the per-level tiled
    kernels with both fields of a level in one y unit; every point, field-wide and line by line."""
    dev = torch.device("cuda:0")
    w = synth.c2_depth()
    xh = w.field(np.float32)
    x = torch.from_numpy(xh).to(dev)
    op = _op(w, dev)
    f = op.apply(x)
    a = op.adjoint(x)
    torch.cuda.synchronize()
    P = _problem(orc, w)
    x64 = xh.astype(np.float64)
    fr, ar = P.rf3(x64, threads=THREADS), P.rf3_adjoint(x64, threads=THREADS)
    fg, ag = f.double().cpu().numpy(), a.double().cpu().numpy()
    ef, ea = rel(fg, fr), rel(ag, ar)
    lf, la = assert_lines(fg, fr, "C2 depth forward"), assert_lines(ag, ar, "C2 depth adjoint")
    print(f"C2 depth: fwd rel L2 {ef:.3e}, adj rel L2 {ea:.3e}; worst line {lf:.3f} / {la:.3f} of allowance",
          flush=True)
    assert ef < TOL32 and ea < TOL32


def test_c4_batch_full(orc):
    dev = torch.device("cuda:0")
    ws = synth.c4_batch()
    gen = torch.Generator(device=dev).manual_seed(synth.SEEDS["c4"])
    ops = [_op(w, dev) for w in ws]
    xs = [torch.randn((1, w.nlev, w.ny, w.nx), generator=gen, device=dev) for w in ws]
    ys = [torch.empty_like(x) for x in xs]
    b = Batch([(op, x, y) for op, x, y in zip(ops, xs, ys)])
    b.autotune(reps=1)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.apply(False)
    for rep in range(2):
        for y in ys:
            y.fill_(float("nan"))                  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        for k, (op, x, y) in enumerate(zip(ops, xs, ys)):
            assert torch.equal(y, op.apply(x)), f"replay {rep}, item {k} (tuning {b.tuning})"
    for k in range(0, len(ws), 8):
        w = ws[k]
        ref = _problem(orc, w).rf3(xs[k].double().cpu().numpy(), threads=THREADS)
        e = rel(ys[k].double().cpu().numpy(), ref)
        assert e < TOL32, f"item {k} ({w.name}): {e:.3e}"
        assert_lines(ys[k].double().cpu().numpy(), ref, f"item {k} ({w.name})")
    b.apply(True)
    torch.cuda.synchronize()
    for k in range(4, len(ws), 8):
        w = ws[k]
        ref = _problem(orc, w).rf3_adjoint(xs[k].double().cpu().numpy(), threads=THREADS)
        e = rel(ys[k].double().cpu().numpy(), ref)
        assert e < TOL32, f"adjoint item {k} ({w.name}): {e:.3e}"
        assert_lines(ys[k].double().cpu().numpy(), ref, f"adjoint item {k} ({w.name})")
