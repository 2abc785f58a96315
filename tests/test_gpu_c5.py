"""The 3D-VAR gradient workload at its full size: V = G_y G_x on the 1440 x 720 x 50
quarter-degree-shaped grid behind the autograd function, 200,000 bilinear point
observations at random sea positions, R = diag(0.25), y = H V v_true + N(0, 0.5^2),
50 CG iterations (the minimiser of Sec. 2.1, cost eq. "functional2", system eq. "eight").

Checked here, in the launch configuration bench.py times (the tiled FP32 kernels):
  - H and H^T at 200k observations against the FP64 reference (oracle/var3d.py);
  - the FP64 gradient against central differences (eps = 1e-2 |v|/|d|; J is
    quadratic, so the difference has no truncation error, relative tolerance 1e-6);
  - the FP32 gradient against the FP64 gradient (relative L2 1e-5);
  - the first CG iterates (FP64) against the reference CG built from the C oracle;
  - 50 FP32 CG iterations with J never increasing.
"""
import os

import numpy as np
import pytest
import torch

from oracle import var3d as ov
from paper_1404_5756_amd import synth
from paper_1404_5756_amd.operator import HorizontalCovariance
from paper_1404_5756_amd.var3d import Var3D, rf3xy, synthetic_problem

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
NOBS = 200_000
THREADS = min(16, os.cpu_count() or 1)


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c5():
    w = synth.c3_global()
    op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, device=DEV)
    p64, vt = synthetic_problem(w, NOBS, DEV, torch.float64, op=op)
    p32 = Var3D(op, p64.obs, p64.y.float(), p64.rinv)
    lev, xs, ys = synth.c5_observations(w, NOBS)
    print(f"C5: {w.nx}x{w.ny}x{w.nlev}, {NOBS} observations", flush=True)
    return w, op, p64, p32, (lev, xs, ys)


def test_c5_observation_operator_full(c5):
    w, op, p64, p32, (lev, xs, ys) = c5
    idx, wt = ov.obs_weights(w.nx, w.ny, lev, xs, ys)
    rng = np.random.default_rng(12)
    f = rng.standard_normal((w.nlev, w.ny, w.nx))
    d = rng.standard_normal(NOBS)
    for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 1e-6)):
        got = p64.obs.apply(torch.from_numpy(f).to(DEV, dtype)).double().cpu().numpy()
        assert rel(got, ov.obs_apply(f, idx, wt)) < tol
        gt = p64.obs.adjoint(torch.from_numpy(d).to(DEV, dtype)).double().cpu().numpy()
        assert rel(gt, ov.obs_adjoint(d, idx, wt, f.size)) < tol


def test_c5_gradient_central_differences_fp64(c5):
    w, op, p64, p32, _ = c5
    gen = torch.Generator(device=DEV).manual_seed(21)
    v = torch.randn(p64.obs.shape, generator=gen, device=DEV, dtype=torch.float64)
    d = torch.randn(p64.obs.shape, generator=gen, device=DEV, dtype=torch.float64)
    _, g = p64.cost_grad(v)
    eps = 1e-2 * float(v.norm() / d.norm())
    fd = (p64.cost_grad(v + eps * d)[0] - p64.cost_grad(v - eps * d)[0]) / (2 * eps)
    gd = float((g * d).sum())
    print(f"C5 FD: directional derivative {gd:.10e}, central difference {fd:.10e}", flush=True)
    assert abs(fd - gd) <= 1e-6 * abs(gd)


def test_c5_fp32_gradient_matches_fp64(c5):
    w, op, p64, p32, _ = c5
    gen = torch.Generator(device=DEV).manual_seed(22)
    v = torch.randn(p64.obs.shape, generator=gen, device=DEV, dtype=torch.float64)
    _, g64 = p64.cost_grad(v)
    _, g32 = p32.cost_grad(v.float())
    e = rel(g32.cpu().numpy(), g64.cpu().numpy())
    print(f"C5 FP32 gradient vs FP64: rel L2 {e:.3e}", flush=True)
    assert e < 1e-5


def test_c5_autograd_backward_is_the_adjoint(c5):
    w, op, *_ = c5
    gen = torch.Generator(device=DEV).manual_seed(23)
    x = torch.randn(w.nlev, w.ny, w.nx, generator=gen, device=DEV, requires_grad=True)
    g = torch.randn(w.nlev, w.ny, w.nx, generator=gen, device=DEV)
    (rf3xy(x, op) * g).sum().backward()
    assert torch.equal(x.grad, op.adjoint(g))


def test_c5_first_cg_iterates_match_reference(c5, orc):
    w, op, p64, p32, (lev, xs, ys) = c5
    iters = 2
    v64, _ = p64.cg(iters, track_cost=False)
    P = orc.Problem(w.mask, w.sigma_x, w.sigma_y, n_img=w.n_img, qmode=orc.QMODES[w.qmode])
    shape = (1, w.nlev, w.ny, w.nx)
    idx, wt = ov.obs_weights(w.nx, w.ny, lev, xs, ys)
    its = ov.cg(lambda v: P.rf3(v.reshape(shape), threads=THREADS).ravel(),
                lambda v: P.rf3_adjoint(v.reshape(shape), threads=THREADS).ravel(),
                idx, wt, p64.y.cpu().numpy(), p64.rinv, int(np.prod(shape)), iters)
    e = rel(v64.cpu().numpy(), its[-1])
    print(f"C5 CG: {iters} FP64 iterates vs reference rel L2 {e:.3e}", flush=True)
    assert e < 1e-8


def test_c5_fifty_cg_iterations_fp32_monotone(c5):
    w, op, p64, p32, _ = c5
    v, costs = p32.cg(50)
    print(f"C5 CG FP32: J {costs[0]:.6e} -> {costs[-1]:.6e} in 50 iterations", flush=True)
    assert len(costs) == 51
    assert all(c1 <= c0 * (1 + 1e-6) for c0, c1 in zip(costs, costs[1:]))
    assert costs[-1] < 0.1 * costs[0]
    _, g = p32.cost_grad(v)
    _, g0 = p32.cost_grad(torch.zeros_like(v))
    print(f"C5 CG FP32: |grad J| {float(g0.norm()):.4e} -> {float(g.norm()):.4e}", flush=True)
    assert float(g.norm()) < float(g0.norm())
