"""Pins of the FP64 3D-VAR reference (oracle/var3d.py) against mathematics.

Bilinear interpolation reproduces bilinear fields exactly; the weights are a
partition of unity; H^T is the transpose of H; the gradient matches central
differences (J is quadratic, so exactly up to rounding); CG reaches the dense
solution of the normal equations and J never increases along it.
"""
import numpy as np
import pytest

from oracle import var3d as ov


def _obs(rng, nx, ny, nlev, n):
    lev = rng.integers(0, nlev, n)
    x = rng.uniform(0, nx - 1, n)
    y = rng.uniform(0, ny - 1, n)
    # include the last row and column exactly
    x[:3] = nx - 1
    y[3:6] = ny - 1
    return lev, x, y


def test_bilinear_fields_are_reproduced_exactly():
    rng = np.random.default_rng(1)
    nx, ny, nlev = 13, 9, 3
    a, b, c, d = (rng.standard_normal(nlev) for _ in range(4))
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    f = np.stack([a[k] + b[k] * ii + c[k] * jj + d[k] * ii * jj for k in range(nlev)])
    lev, x, y = _obs(rng, nx, ny, nlev, 200)
    idx, w = ov.obs_weights(nx, ny, lev, x, y)
    got = ov.obs_apply(f, idx, w)
    exact = a[lev] + b[lev] * x + c[lev] * y + d[lev] * x * y
    assert np.max(np.abs(got - exact)) < 1e-11


def test_weights_are_a_partition_of_unity():
    rng = np.random.default_rng(2)
    lev, x, y = _obs(rng, 20, 15, 2, 300)
    idx, w = ov.obs_weights(20, 15, lev, x, y)
    assert np.all(w >= 0)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-15)
    assert np.all((idx >= 0) & (idx < 20 * 15 * 2))
    assert np.all(idx // (20 * 15) == lev[:, None])


def test_adjoint_is_transpose():
    rng = np.random.default_rng(3)
    nx, ny, nlev = 11, 7, 2
    lev, x, y = _obs(rng, nx, ny, nlev, 50)
    idx, w = ov.obs_weights(nx, ny, lev, x, y)
    f = rng.standard_normal(nx * ny * nlev)
    d = rng.standard_normal(50)
    lhs = ov.obs_apply(f, idx, w) @ d
    rhs = f @ ov.obs_adjoint(d, idx, w, nx * ny * nlev)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.fixture(scope="module")
def small(orc):
    rng = np.random.default_rng(4)
    nx, ny, nlev = 12, 9, 2
    mask = np.ones((1, ny, nx), np.uint8)
    mask[0, 3:5, 4:8] = 0
    sig = rng.uniform(1.5, 3.0, (1, ny, nx))
    P = orc.Problem(mask, sig, sig.copy(), n_img=1, qmode=orc.FIT)
    shape = (1, nlev, ny, nx)

    def V(v):
        return P.rf3(v.reshape(shape)).ravel()

    def Vt(v):
        return P.rf3_adjoint(v.reshape(shape)).ravel()

    lev, x, y = _obs(rng, nx, ny, nlev, 40)
    idx, w = ov.obs_weights(nx, ny, lev, x, y)
    yobs = rng.standard_normal(40)
    return V, Vt, idx, w, yobs, 4.0, nx * ny * nlev


def test_gradient_matches_central_differences(small):
    V, Vt, idx, w, yobs, rinv, n = small
    rng = np.random.default_rng(5)
    v = rng.standard_normal(n)
    d = rng.standard_normal(n)
    J, g = ov.cost(v, V, Vt, idx, w, yobs, rinv)
    eps = 1e-2 * np.linalg.norm(v) / np.linalg.norm(d)
    fd = (ov.cost(v + eps * d, V, Vt, idx, w, yobs, rinv)[0] - ov.cost(v - eps * d, V, Vt, idx, w, yobs, rinv)[0]) / (
        2 * eps)
    assert abs(fd - g @ d) <= 1e-8 * abs(g @ d)


def test_cg_reaches_dense_solution_monotonically(small):
    V, Vt, idx, w, yobs, rinv, n = small
    # dense normal matrix from unit vectors
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = e + Vt(ov.obs_adjoint(rinv * ov.obs_apply(V(e), idx, w), idx, w, n))
    b = Vt(ov.obs_adjoint(rinv * yobs, idx, w, n))
    vstar = np.linalg.solve(A, b)
    its = ov.cg(V, Vt, idx, w, yobs, rinv, n, 60)
    costs = [ov.cost(v, V, Vt, idx, w, yobs, rinv)[0] for v in its]
    assert all(c1 <= c0 + 1e-12 * abs(c0) for c0, c1 in zip(costs, costs[1:]))
    assert np.linalg.norm(its[-1] - vstar) <= 1e-8 * np.linalg.norm(vstar)
