"""Pins of the oracle's two options beyond the paper's scheme.

Exact end conditions (EXACT_ENDS): the anti-causal 3rd-RF sweep starts from the
values the infinite-line filter would carry back from past the segment end
(input zero outside the segment, the last point's coefficients continued).
Periodic rows (PERIODIC_X): zonally periodic lines, sea runs and imaginary
points found around the cycle, a row without land solved as a cyclic recurrence.

Each option is pinned against something other than the oracle's own formula:
dense brute-force solves on a long embedding line or on the cyclic matrices,
exact invariants (Toeplitz / circulant structure, constant preservation), the
dense transpose, and reduction to the paper's case.
"""
import numpy as np
import pytest

from test_oracle_pins import brute_rf3_segment, brute_segments, dense_operator, impulse


def line(orc, sigma, mask=None, n_img=0, qmode=2, flags=0, K=5):
    sigma = np.atleast_1d(np.asarray(sigma, float))
    mask = np.ones(sigma.size) if mask is None else np.asarray(mask)
    return orc.Problem(mask[None], sigma[None], sigma[None], n_img=n_img, qmode=qmode, k1=K, flags=flags)


# ---------------------------------------------------------------- exact end conditions
def long_line_block(orc, sig, qmode, W):
    """Printed zero-state filter on the segment followed by W points with the last point's
    coefficients and zero input, restricted to the segment (brute force, dense solves)."""
    m = sig.size
    ext = np.concatenate([sig, np.full(W, sig[-1])])
    al = orc.coef3(ext, qmode)
    return brute_rf3_segment(al[:3], al[3])[:m, :m]


@pytest.mark.parametrize("qmode", [0, 2])
def test_exact_ends_equal_the_long_line_restricted(orc, qmode):
    rng = np.random.default_rng(60 + qmode)
    m = 41
    mask = np.ones(m, np.uint8)
    mask[[9, 10, 25]] = 0
    sig = rng.uniform(1.5, 7.0, m)
    n_img = 2
    P = line(orc, sig, mask, n_img, qmode, flags=orc.EXACT_ENDS)
    G = dense_operator(orc, P)
    B = np.zeros((m, m))
    for a, e in brute_segments(list(mask), n_img):
        B[a:e + 1, a:e + 1] = long_line_block(orc, sig[a:e + 1], qmode, 900)
    sea = np.diag(mask.astype(float))
    np.testing.assert_allclose(G, sea @ B @ sea, rtol=1e-11, atol=1e-12 * np.abs(B).max())
    # and they differ from the paper's zero ends
    G0 = dense_operator(orc, line(orc, sig, mask, n_img, qmode))
    assert np.abs(G - G0).max() > 1e-3


@pytest.mark.parametrize("sigma", [2.0, 4.0, 8.0])
def test_exact_ends_uniform_sigma_is_toeplitz_with_a_flat_diagonal(orc, sigma):
    """Uniform sigma: the segment operator is the infinite-line convolution restricted, so
    G[i, j] = g(i - j): symmetric, constant along every diagonal (the diagonal is as flat
    at both ends as inside; the zero ends damp one end to ~1e-2 of it)."""
    m = 60
    G = dense_operator(orc, line(orc, np.full(m, sigma), flags=orc.EXACT_ENDS))
    scale = np.abs(G).max()
    np.testing.assert_allclose(G[1:, 1:], G[:-1, :-1], atol=1e-12 * scale)
    np.testing.assert_allclose(G, G.T, atol=1e-12 * scale)
    d = np.diag(G)
    assert np.ptp(d) <= 1e-12 * scale
    # the diagonal is the peak of the infinite-line impulse response
    n = int(80 * sigma) | 1
    h = impulse(orc, n, sigma, qmode=2)
    np.testing.assert_allclose(G[:, 0], h[n // 2:n // 2 + m], rtol=1e-10, atol=1e-12 * scale)


@pytest.mark.parametrize("qmode", [0, 1, 2])
def test_exact_ends_adjoint_is_the_dense_transpose(orc, qmode):
    rng = np.random.default_rng(70 + qmode)
    m = 37
    mask = (rng.uniform(size=m) > 0.2).astype(np.uint8)
    mask[[3, 4]] = 1, 0          # one-point segment at 3
    sig = rng.uniform(1.2, 6.0, m)
    P = line(orc, sig, mask, 2, qmode, flags=orc.EXACT_ENDS)
    G = dense_operator(orc, P, "rf3")
    Gt = dense_operator(orc, P, "rf3_adj")
    np.testing.assert_allclose(Gt, G.T, rtol=1e-11, atol=1e-12 * np.abs(G).max())


def test_exact_ends_change_only_the_segment_end_region(orc):
    """The end condition enters at the segment end and decays backwards through the
    anti-causal recurrence: far from the end the two operators agree."""
    m, sigma = 200, 3.0
    G = dense_operator(orc, line(orc, np.full(m, sigma), flags=orc.EXACT_ENDS))
    G0 = dense_operator(orc, line(orc, np.full(m, sigma)))
    far = slice(0, m - 120)
    np.testing.assert_allclose(G[far, far], G0[far, far], atol=1e-12 * np.abs(G).max())
    assert np.abs(G[-1, -1] - G0[-1, -1]) > 0.1 * G[-1, -1]


def test_exact_ends_leave_the_1st_rf_unchanged(orc):
    rng = np.random.default_rng(73)
    m = 30
    sig = rng.uniform(1.5, 5.0, m)
    mask = np.ones(m, np.uint8)
    mask[12] = 0
    G = dense_operator(orc, line(orc, sig, mask, 1, flags=orc.EXACT_ENDS), "rf1", K=3)
    G0 = dense_operator(orc, line(orc, sig, mask, 1), "rf1", K=3)
    np.testing.assert_array_equal(G, G0)


# ---------------------------------------------------------------- periodic rows
def brute_segments_cyclic(mask, n_img):
    """Cyclic sea runs, and each land point within n_img (around the cycle) of a run joins the
    nearest run; at equal distance the run before the point wins."""
    n = len(mask)
    if all(mask):
        return [], True
    if not any(mask):
        return [], False
    runs = []
    for i in range(n):
        if mask[i] and not mask[i - 1]:
            j = i
            while mask[(j + 1) % n]:
                j = (j + 1) % n
            runs.append((i, j))
    owner = {}
    for r, (a, e) in enumerate(runs):
        t = a
        while True:
            owner[t] = r
            if t == e:
                break
            t = (t + 1) % n
    trailing = {}
    for i in range(n):
        if mask[i]:
            continue
        cands = []
        for r, (a, e) in enumerate(runs):
            db, da = (i - e) % n, (a - i) % n
            cands.append((min(db, da), 0 if db <= da else 1, r))
        d, side, r = min(cands)
        if d <= n_img:
            owner[i] = r
            trailing[i] = side == 0
    segs = []
    for r, (a, e) in enumerate(runs):
        # leading imaginary points, the run, trailing imaginary points
        while owner.get((a - 1) % n) == r and trailing.get((a - 1) % n) is False:
            a = (a - 1) % n
        while owner.get((e + 1) % n) == r and trailing.get((e + 1) % n) is True:
            e = (e + 1) % n
        segs.append((a, e))
    return sorted(segs), False


def test_cyclic_single_run_with_covered_gap(orc):
    """One run whose land gap is all imaginary points: the segment starts at the first
    leading point (the gap's second half) and ends at the last trailing one (its first half)."""
    mask = np.array([1, 1, 1, 0, 0, 0, 0, 1, 1], np.uint8)     # gap 3..6
    _, kind, segs, whole = orc.segments_cyclic(mask, 2)
    assert not whole and segs == [(5, 4)]                      # 3, 4 trail the run; 5, 6 lead it
    assert list(kind) == [1, 1, 1, 2, 2, 2, 2, 1, 1]


@pytest.mark.parametrize("n_img", [0, 1, 3])
def test_cyclic_segments_match_brute_force(orc, n_img):
    rng = np.random.default_rng(80 + n_img)
    for _ in range(60):
        n = int(rng.integers(1, 30))
        mask = (rng.uniform(size=n) > rng.uniform(0.1, 0.8)).astype(np.uint8)
        _, kind, segs, whole = orc.segments_cyclic(mask, n_img)
        exp, exp_whole = brute_segments_cyclic(list(mask), n_img)
        assert whole == exp_whole
        assert sorted(segs) == exp, (mask, n_img)
        assert np.all((kind == 1) == (mask == 1))


def brute_cyclic_operator(al, be):
    """U_cyc^-1 D_beta L_cyc^-1 D_beta with every index taken mod n (dense solve)."""
    n = be.size
    L = np.eye(n)
    U = np.eye(n)
    for i in range(n):
        for k in (1, 2, 3):
            L[i, (i - k) % n] -= al[k - 1, i]
            U[i, (i + k) % n] -= al[k - 1, i]
    Db = np.diag(be)
    return np.linalg.solve(U, Db @ np.linalg.solve(L, Db))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 48])
@pytest.mark.parametrize("qmode", [0, 2])
def test_periodic_all_sea_row_is_the_cyclic_system(orc, n, qmode):
    rng = np.random.default_rng(90 + n)
    sig = rng.uniform(1.2, 6.0, n)
    P = line(orc, sig, qmode=qmode, flags=orc.PERIODIC_X)
    G = dense_operator(orc, P)
    al = orc.coef3(sig, qmode)
    np.testing.assert_allclose(G, brute_cyclic_operator(al[:3], al[3]), rtol=1e-11,
                               atol=1e-12 * np.abs(G).max())
    Gt = dense_operator(orc, P, "rf3_adj")
    np.testing.assert_allclose(Gt, G.T, rtol=1e-11, atol=1e-12 * np.abs(G).max())


@pytest.mark.parametrize("sigma", [2.0, 5.0, 11.0])
def test_periodic_uniform_sigma_keeps_constants_and_folds_the_impulse_response(orc, sigma):
    """A cycle has no ends: a constant field comes out as c sqrt(2 pi) sigma at every point,
    the operator is circulant and symmetric, and its column is the infinite-line impulse
    response folded around the cycle."""
    n = 40
    P = line(orc, np.full(n, sigma), flags=orc.PERIODIC_X)
    out = P.apply_dir(np.full((1, n), 1.5), "x")[0]
    np.testing.assert_allclose(out, 1.5 * np.sqrt(2 * np.pi) * sigma, rtol=1e-11)
    G = dense_operator(orc, P)
    scale = np.abs(G).max()
    np.testing.assert_allclose(G, np.roll(np.roll(G, 1, 0), 1, 1), atol=1e-12 * scale)
    np.testing.assert_allclose(G, G.T, atol=1e-12 * scale)
    m = (int(200 * sigma) // n) * n + 1
    h = impulse(orc, m, sigma, qmode=2)
    c = m // 2
    folded = np.zeros(n)
    for t in range(m):
        folded[(t - c) % n] += h[t]
    np.testing.assert_allclose(G[:, 0], folded, rtol=1e-10, atol=1e-12 * scale)


@pytest.mark.parametrize("n_img", [0, 2])
def test_periodic_row_with_land_is_block_diagonal_over_cyclic_segments(orc, n_img):
    rng = np.random.default_rng(95 + n_img)
    n = 34
    mask = np.ones(n, np.uint8)
    mask[[8, 9, 20]] = 0          # runs 10..19 and a wrapped run 21..33, 0..7
    sig = rng.uniform(1.5, 6.0, n)
    P = line(orc, sig, mask, n_img, flags=orc.PERIODIC_X)
    G = dense_operator(orc, P)
    segs, whole = brute_segments_cyclic(list(mask), n_img)
    assert not whole and any(a > e for a, e in segs)
    al = orc.coef3(sig, 2)
    B = np.zeros((n, n))
    for a, e in segs:
        idx = [(a + t) % n for t in range((e - a) % n + 1)]
        B[np.ix_(idx, idx)] = brute_rf3_segment(al[:3, idx], al[3, idx])
    sea = np.diag(mask.astype(float))
    np.testing.assert_allclose(G, sea @ B @ sea, rtol=1e-11, atol=1e-13 * np.abs(B).max())
    for flags in (orc.PERIODIC_X, orc.PERIODIC_X | orc.EXACT_ENDS):
        Q = line(orc, sig, mask, n_img, flags=flags)
        np.testing.assert_allclose(dense_operator(orc, Q, "rf3_adj"), dense_operator(orc, Q).T, rtol=1e-11,
                                   atol=1e-12 * np.abs(G).max())


def test_periodic_with_land_at_the_seam_is_the_paper_case(orc):
    """Land at i = 0 and no imaginary points: no run wraps, so periodic = non-periodic."""
    rng = np.random.default_rng(97)
    n = 30
    mask = (rng.uniform(size=n) > 0.25).astype(np.uint8)
    mask[0] = 0
    sig = rng.uniform(1.5, 6.0, n)
    for op in ("rf3", "rf3_adj", "rf1"):
        G = dense_operator(orc, line(orc, sig, mask, 0, flags=orc.PERIODIC_X), op, K=3)
        G0 = dense_operator(orc, line(orc, sig, mask, 0), op, K=3)
        np.testing.assert_array_equal(G, G0)


@pytest.mark.parametrize("K", [1, 3, 5])
def test_periodic_1st_rf(orc, K):
    rng = np.random.default_rng(98 + K)
    n = 23
    sig = rng.uniform(1.5, 5.0, n)
    P = line(orc, sig, flags=orc.PERIODIC_X, K=K)
    G = dense_operator(orc, P, "rf1", K=K)
    al, be = orc.coef1(sig, K)
    L = np.eye(n)
    U = np.eye(n)
    for i in range(n):
        L[i, (i - 1) % n] -= al[i]
        U[i, (i + 1) % n] -= al[i]
    one = np.linalg.solve(U, np.diag(be) @ np.linalg.solve(L, np.diag(be)))
    np.testing.assert_allclose(G, np.linalg.matrix_power(one, K), rtol=1e-11, atol=1e-14)
    Pu = line(orc, np.full(n, 3.0), flags=orc.PERIODIC_X, K=K)
    np.testing.assert_allclose(Pu.apply_dir(np.full((1, n), 2.0), "x", op="rf1", K=K)[0], 2.0, rtol=1e-12)


def test_periodic_is_x_only_and_2d_is_rows_then_columns(orc):
    rng = np.random.default_rng(99)
    ny, nx = 6, 9
    mask = (rng.uniform(size=(1, ny, nx)) > 0.2).astype(np.uint8)
    mask[0, 2, :] = 1             # one all-sea (cyclic) row
    sx = rng.uniform(1.0, 5.0, (1, ny, nx))
    sy = rng.uniform(1.0, 5.0, (1, ny, nx))
    P = orc.Problem(mask, sx, sy, n_img=1, qmode=2, flags=orc.PERIODIC_X)
    P0 = orc.Problem(mask, sx, sy, n_img=1, qmode=2)
    N = ny * nx
    E = np.eye(N).reshape(N, ny, nx)
    Gx = np.stack([P.apply_dir(E[k], "x").ravel() for k in range(N)], axis=1)
    Gy = np.stack([P.apply_dir(E[k], "y").ravel() for k in range(N)], axis=1)
    Gy0 = np.stack([P0.apply_dir(E[k], "y").ravel() for k in range(N)], axis=1)
    np.testing.assert_array_equal(Gy, Gy0)
    V = np.stack([P.rf3(E[k]).ravel() for k in range(N)], axis=1)
    np.testing.assert_allclose(V, Gy @ Gx, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- anisotropic, inhomogeneous scales
@pytest.mark.parametrize("sx,sy", [(2.0, 5.0), (7.0, 3.0)])
def test_anisotropic_impulse_moments(orc, sx, sy):
    """sigma_x != sigma_y (VARMATCH): the 2-D impulse response is separable with second moments
    exactly sigma_x^2 along x and sigma_y^2 along y, no cross moment, mass 2 pi sigma_x sigma_y."""
    ny, nx = int(48 * sy) | 1, int(48 * sx) | 1
    P = orc.Problem(np.ones((ny, nx)), np.full((ny, nx), sx), np.full((ny, nx), sy), qmode=orc.VARMATCH)
    imp = np.zeros((ny, nx))
    imp[ny // 2, nx // 2] = 1.0
    h = P.rf3(imp)
    yy, xx = np.mgrid[0:ny, 0:nx]
    yy, xx = yy - ny // 2, xx - nx // 2
    m = h.sum()
    assert m == pytest.approx(2 * np.pi * sx * sy, rel=1e-7)
    assert (h * xx * xx).sum() / m == pytest.approx(sx * sx, rel=1e-6)
    assert (h * yy * yy).sum() / m == pytest.approx(sy * sy, rel=1e-6)
    assert abs((h * xx * yy).sum() / m) < 1e-9 * sx * sy
    # separable: the response is the outer product of the two 1-D responses
    np.testing.assert_allclose(h, np.outer(h[:, nx // 2], h[ny // 2, :]) / h[ny // 2, nx // 2], rtol=1e-10,
                               atol=1e-14 * h.max())


def test_inhomogeneous_anisotropic_covariance_is_symmetric_psd(orc):
    """Spatially varying sigma_x != sigma_y with land: V is not symmetric, but the covariance
    B = V V^T it models is symmetric positive semi-definite (dense, tiny grid)."""
    rng = np.random.default_rng(110)
    ny, nx = 9, 11
    mask = (rng.uniform(size=(ny, nx)) > 0.2).astype(np.uint8)
    sx = rng.uniform(1.5, 6.0, (ny, nx))
    sy = 0.5 * sx + rng.uniform(0.5, 1.0, (ny, nx))
    P = orc.Problem(mask, sx, sy, n_img=2, qmode=orc.FIT)
    N = ny * nx
    E = np.eye(N).reshape(N, ny, nx)
    V = np.stack([P.rf3(E[k]).ravel() for k in range(N)], axis=1)
    Vt = np.stack([P.rf3_adjoint(E[k]).ravel() for k in range(N)], axis=1)
    np.testing.assert_allclose(Vt, V.T, rtol=1e-12, atol=1e-13 * np.abs(V).max())
    assert np.abs(V - V.T).max() > 1e-3
    B = V @ Vt
    np.testing.assert_allclose(B, B.T, rtol=1e-12, atol=1e-12 * np.abs(B).max())
    assert np.linalg.eigvalsh(B).min() > -1e-10 * np.abs(B).max()


def test_inhomogeneous_local_width_follows_the_local_scale(orc):
    """Slowly varying sigma_x along a line (VARMATCH): the impulse response at a point has a
    second moment close to the local sigma^2 (a 1.2% per grid point gradient moves it by a few %)."""
    n = 1201
    i = np.arange(n)
    sig = 6.0 * np.exp(0.012 * (i - n // 2) / 6.0)          # +-20% over +-100 points
    P = orc.Problem(np.ones((1, n)), sig[None], sig[None], qmode=orc.VARMATCH)
    for c in (450, 600, 750):
        x = np.zeros((1, n))
        x[0, c] = 1.0
        h = P.apply_dir(x, "x")[0]
        k = i - c
        var = (h * k * k).sum() / h.sum()
        assert var == pytest.approx(sig[c] ** 2, rel=0.05)
