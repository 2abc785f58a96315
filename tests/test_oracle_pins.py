"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numbers the
paper prints (tests/golden/paper_constants.json), closed forms, invariants, and
brute force with dense matrices on tiny inputs.  A plausible slip in the oracle
(a dropped term, a wrong sign or index, a transposed operand, a wrong constant)
fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


# ---------------------------------------------------------------- helpers
def line_problem(orc, sigma, mask=None, n_img=0, qmode=0):
    sigma = np.atleast_1d(np.asarray(sigma, float))
    m = sigma.size
    mask = np.ones(m) if mask is None else np.asarray(mask)
    return orc.Problem(mask[None], sigma[None], sigma[None], n_img=n_img, qmode=qmode)


def dense_operator(orc, P, op="rf3", K=None):
    """Column-by-column matrix of the oracle's 1-D x-operator on a single row."""
    m = P.nx
    E = np.eye(m)
    return np.stack([P.apply_dir(E[j][None], "x", op=op, K=K)[0] for j in range(m)], axis=1)


def brute_rf3_segment(al, be):
    """G = U^-1 D_beta L^-1 D_beta with (L)_{i,i-k} = -alpha_{i,k}, (U)_{i,i+k} = -alpha_{i,k}:
    eqs. 'fort'/'bact' with zero state outside the segment, as dense solves."""
    m = be.size
    L = np.eye(m)
    U = np.eye(m)
    for i in range(m):
        for k in (1, 2, 3):
            if i - k >= 0:
                L[i, i - k] = -al[k - 1, i]
            if i + k < m:
                U[i, i + k] = -al[k - 1, i]
    Db = np.diag(be)
    return np.linalg.solve(U, Db @ np.linalg.solve(L, Db))


def brute_segments(mask, n_img):
    """Extended segments by brute force: distance of every land point to every sea run."""
    m = len(mask)
    runs = []
    i = 0
    while i < m:
        if mask[i]:
            j = i
            while j + 1 < m and mask[j + 1]:
                j += 1
            runs.append([i, j])
            i = j + 1
        else:
            i += 1
    owner = [None] * m
    for r, (a, e) in enumerate(runs):
        for i in range(a, e + 1):
            owner[i] = r
    for i in range(m):
        if mask[i]:
            continue
        d = [(a - i if i < a else i - e, r) for r, (a, e) in enumerate(runs)]
        d = [x for x in d if x[0] <= n_img]
        if d:
            owner[i] = min(d)[1]  # smallest distance, then smallest run index
    segs = []
    for r in range(len(runs)):
        idx = [i for i in range(m) if owner[i] == r]
        segs.append((min(idx), max(idx)))
    return segs


def gaussian(m, sigma):
    i = np.arange(m) - m // 2
    return np.exp(-i * i / (2.0 * sigma * sigma))


def shape_error(h, g):
    hn, gn = h / h.sum(), g / g.sum()
    return np.linalg.norm(hn - gn) / np.linalg.norm(gn)


def impulse(orc, m, sigma, qmode=0, op="rf3", K=None):
    P = line_problem(orc, np.full(m, sigma), qmode=qmode)
    x = np.zeros((1, m))
    x[0, m // 2] = 1.0
    return P.apply_dir(x, "x", op=op, K=K)[0]


# ---------------------------------------------------------------- constants
def test_theorem_polynomials_match_the_factorised_denominator(orc):
    """1 - sum_k alpha_k w^k must equal D(1-w)/D(1) with D from eq. 'indietro' (s = 1 - z^-1)."""
    lin = GOLD["causal_factors"]["linear"]
    quad = GOLD["causal_factors"]["quadratic"]
    rng = np.random.default_rng(11)
    for q in [0.3, 1.0, 2.0, 4.7, 12.0, 25.0]:
        al1, al2, al3, _ = orc.coef3(np.array([q]), 0)[:, 0]
        for w in rng.uniform(-1.5, 1.5, 5):
            s = 1.0 - w
            D = lambda s_: (lin[0] + lin[1] * q * s_) * (quad[0] + quad[1] * q * s_ + quad[2] * (q * s_) ** 2)
            lhs = 1.0 - al1 * w - al2 * w * w - al3 * w ** 3
            assert lhs == pytest.approx(D(s) / D(1.0), rel=2e-6, abs=2e-7)


def test_theorem_polynomials_are_the_golden_numbers(orc):
    """alpha_k = a_k/a_0 with the a_k printed in Theorem 3.1."""
    g = GOLD["theorem_a_poly"]
    for q in [0.5, 2.0, 7.0]:
        pw = np.array([1, q, q * q, q ** 3])
        a = [np.dot(g[k], pw) for k in ("a0", "a1", "a2", "a3")]
        al = orc.coef3(np.array([q]), 0)[:3, 0]
        np.testing.assert_allclose(al, np.array(a[1:]) / a[0], rtol=1e-14)


def test_abramowitz_stegun_polynomial_roots_and_factors():
    """The printed real root +-1.16680481 and the two printed factors reproduce the A&S polynomial."""
    g = GOLD["abramowitz_stegun"]
    poly = np.array([-g["b6"], 0, g["b4"], 0, -g["b2"], 0, g["b0"]])  # in u = sigma*s, highest first
    roots = np.roots(poly)
    real = np.sort(roots[np.abs(roots.imag) < 1e-9].real)
    np.testing.assert_allclose(real, [-GOLD["real_root"]["value"], GOLD["real_root"]["value"]], rtol=1e-7)
    lin = GOLD["causal_factors"]["linear"]
    quad = GOLD["causal_factors"]["quadratic"]
    f = np.polymul([lin[1], lin[0]], [quad[2], quad[1], quad[0]])            # causal factor in u
    b = np.polymul([-lin[1], lin[0]], [quad[2], -quad[1], quad[0]])          # anti-causal factor
    prod = np.polymul(f, b)
    np.testing.assert_allclose(prod / prod[-1], poly / poly[-1], rtol=3e-5, atol=3e-6)
    # and the rational approximation itself honours the printed bound
    t = np.linspace(-6, 6, 2001)
    approx = 1.0 / (g["b0"] + g["b2"] * t ** 2 + g["b4"] * t ** 4 + g["b6"] * t ** 6)
    assert np.max(np.abs(np.exp(-t * t / 2) / np.sqrt(2 * np.pi) - approx)) < g["eps_bound"]


# ---------------------------------------------------------------- 1-D 3rd-RF
@pytest.mark.parametrize("qmode", [0, 1, 2])
def test_rf3_matches_dense_brute_force(orc, qmode):
    rng = np.random.default_rng(3 + qmode)
    m = 37
    sig = rng.uniform(1.2, 9.0, m)
    P = line_problem(orc, sig, qmode=qmode)
    G = dense_operator(orc, P)
    al = orc.coef3(sig, qmode)
    Gb = brute_rf3_segment(al[:3], al[3])
    np.testing.assert_allclose(G, Gb, rtol=1e-12, atol=1e-13 * np.abs(Gb).max())


@pytest.mark.parametrize("qmode", [0, 1, 2])
def test_rf3_adjoint_is_the_dense_transpose(orc, qmode):
    rng = np.random.default_rng(5)
    m = 29
    sig = rng.uniform(1.0, 7.0, m)
    mask = (rng.uniform(size=m) > 0.25).astype(np.uint8)
    P = line_problem(orc, sig, mask=mask, n_img=2, qmode=qmode)
    G = dense_operator(orc, P, "rf3")
    Gt = dense_operator(orc, P, "rf3_adj")
    np.testing.assert_allclose(Gt, G.T, rtol=1e-12, atol=1e-13 * np.abs(G).max())
    # varying sigma: the operator is not symmetric (the adjoint is a different operator)
    assert np.abs(G - G.T).max() > 1e-3


def test_rf3_uniform_sigma_is_symmetric(orc):
    P = line_problem(orc, np.full(40, 3.3))
    G = dense_operator(orc, P)
    np.testing.assert_allclose(G, G.T, atol=1e-13 * np.abs(G).max())


@pytest.mark.parametrize("sigma", [2.0, 4.0, 8.0, 12.0])
@pytest.mark.parametrize("qmode", [0, 1, 2])
def test_rf3_dc_gain_is_sqrt_2pi_sigma(orc, sigma, qmode):
    """Gain constraint of Appendix A (eqs. 'avanti3','avanti4'): the fwd+bwd pair has H(omega=0) = sqrt(2 pi) sigma."""
    m = int(80 * sigma) | 1
    h = impulse(orc, m, sigma, qmode)
    assert h.sum() == pytest.approx(np.sqrt(2 * np.pi) * sigma, rel=1e-10)
    i = np.arange(m) - m // 2
    assert abs((h * i).sum() / h.sum()) < 1e-9   # zero mean shift


@pytest.mark.parametrize("q", [1.0, 2.0, 4.0, 8.0])
def test_rf3_literal_variance_closed_form(orc, q):
    """Variance of the pair = 2[(c1/c0) q + ((c1/c0)^2 - 2 c2/c0) q^2], from the generating function
    of 1/(a0 - a1 z^-1 - a2 z^-2 - a3 z^-3) with the Theorem's constants."""
    c0, c1, c2 = GOLD["theorem_a_poly"]["a0"][:3]
    m = int(120 * q) | 1
    h = impulse(orc, m, q, 0)
    i = np.arange(m) - m // 2
    var = (h * i * i).sum() / h.sum()
    r = c1 / c0
    assert var == pytest.approx(2 * (r * q + (r * r - 2 * c2 / c0) * q * q), rel=1e-9)


@pytest.mark.parametrize("sigma", [2.0, 5.0, 11.0])
def test_rf3_varmatch_has_variance_sigma_squared(orc, sigma):
    m = int(120 * sigma) | 1
    h = impulse(orc, m, sigma, 1)
    i = np.arange(m) - m // 2
    assert (h * i * i).sum() / h.sum() == pytest.approx(sigma * sigma, rel=1e-9)


def test_fit_q_is_near_the_shape_error_minimiser(orc):
    from scipy.optimize import minimize_scalar
    for sigma in (2.0, 6.0, 12.0):
        m = int(60 * sigma) | 1
        g = gaussian(m, sigma)
        r = minimize_scalar(lambda q: shape_error(impulse(orc, m, q, 0), g),
                            bounds=(0.3 * sigma, 1.2 * sigma), method="bounded")
        assert abs(orc.qmap(2, sigma) - r.x) < 0.02
        # and the FIT impulse response is a better Gaussian than LITERAL's
        assert shape_error(impulse(orc, m, sigma, 2), g) < shape_error(impulse(orc, m, sigma, 0), g)


# ---------------------------------------------------------------- 1st-RF
@pytest.mark.parametrize("K", [1, 2, 3, 5, 10])
@pytest.mark.parametrize("sigma", [2.0, 6.0])
def test_rf1_mass_one_and_variance_sigma_squared(orc, K, sigma):
    """Hayden relation eq. 'crucial': K fwd+bwd passes of the 1st-order filter have variance R^2/dx^2."""
    m = int(60 * sigma) | 1
    h = impulse(orc, m, sigma, op="rf1", K=K)
    i = np.arange(m) - m // 2
    assert h.sum() == pytest.approx(1.0, rel=1e-10)
    assert (h * i * i).sum() / h.sum() == pytest.approx(sigma * sigma, rel=1e-8)


def test_rf1_matches_dense_brute_force(orc):
    rng = np.random.default_rng(7)
    m, K = 23, 3
    sig = rng.uniform(1.0, 5.0, m)
    P = line_problem(orc, sig)
    G = dense_operator(orc, P, "rf1", K=K)
    al, be = orc.coef1(sig, K)
    L = np.eye(m) - np.diag(al[1:], -1)
    U = np.eye(m) - np.diag(al[:-1], 1)
    one = np.linalg.solve(U, np.diag(be) @ np.linalg.solve(L, np.diag(be)))   # eqs. proc1-1, proc1-2
    np.testing.assert_allclose(G, np.linalg.matrix_power(one, K), rtol=1e-11, atol=1e-14)


def test_fig1_setting_rf1_converges_and_rf3_fit_beats_k5(orc):
    """Fig. 1 setting: m = 300, sigma = R/dx = 2. 1st-RF error decreases with K; 3rd-RF (one pass) is
    competitive with many 1st-RF iterations."""
    f = GOLD["fig1_setting"]
    m, sigma = f["m"], f["R"] / f["dx"]
    g = gaussian(m + 1, sigma)
    errs = [shape_error(impulse(orc, m + 1, sigma, op="rf1", K=K), g) for K in (1, 2, 3, 5, 10, 20)]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.06
    e_fit = shape_error(impulse(orc, m + 1, sigma, 2), g)
    assert e_fit < errs[3]          # better than K = 5


@pytest.mark.parametrize("sigma", [1.5, 2.0, 4.0, 8.0, 12.0])
def test_rf3_fit_beats_rf1_k5_over_the_sigma_range(orc, sigma):
    m = int(60 * sigma) | 1
    g = gaussian(m, sigma)
    assert shape_error(impulse(orc, m, sigma, 2), g) < shape_error(impulse(orc, m, sigma, op="rf1", K=5), g)


def brute_rf1_iteration(al, be):
    """One 1st-RF iteration on a segment from zero state at both ends (eqs. 'proc1-1', 'proc1-2'),
    as dense solves: U^-1 D_beta L^-1 D_beta with (L)_{i,i-1} = -alpha_i, (U)_{i,i+1} = -alpha_i."""
    m = be.size
    L = np.eye(m) - np.diag(al[1:], -1)
    U = np.eye(m) - np.diag(al[:-1], 1)
    return np.linalg.solve(U, np.diag(be) @ np.linalg.solve(L, np.diag(be)))


@pytest.mark.parametrize("n_img", [0, 1, 3])
@pytest.mark.parametrize("K", [1, 3, 5])
def test_rf1_masked_line_with_imaginary_points_is_brute_force(orc, n_img, K):
    """1st-RF on a line with coasts: imaginary points take zero input in the first iteration, keep
    their values between iterations and are zeroed in the output, so the line operator is
    P_sea (block-diagonal over the extended segments of one-iteration operators)^K P_sea."""
    rng = np.random.default_rng(40 + 7 * n_img + K)
    for trial in range(6):
        m = int(rng.integers(12, 48))
        mask = (rng.uniform(size=m) > rng.uniform(0.15, 0.5)).astype(np.uint8)
        mask[int(rng.integers(0, m))] = 1
        sig = rng.uniform(1.2, 6.0, m)
        P = line_problem(orc, sig, mask=mask, n_img=n_img)
        G = dense_operator(orc, P, "rf1", K=K)
        al, be = orc.coef1(sig, K)
        B = np.zeros((m, m))
        for a, e in brute_segments(list(mask), n_img):
            B[a:e + 1, a:e + 1] = np.linalg.matrix_power(brute_rf1_iteration(al[a:e + 1], be[a:e + 1]), K)
        sea = np.diag(mask.astype(float))
        np.testing.assert_allclose(G, sea @ B @ sea, rtol=1e-12, atol=1e-14)
        # the imaginary points matter once K > 1 or a trailing extension exists
        if n_img > 0 and K > 1 and trial == 0:
            B0 = np.zeros((m, m))
            for a, e in brute_segments(list(mask), 0):
                B0[a:e + 1, a:e + 1] = np.linalg.matrix_power(brute_rf1_iteration(al[a:e + 1], be[a:e + 1]), K)
            assert np.abs(sea @ B0 @ sea - G).max() > 1e-6
            # zeroing the imaginary points between iterations is a different operator
            Bz = np.zeros((m, m))
            for a, e in brute_segments(list(mask), n_img):
                one = brute_rf1_iteration(al[a:e + 1], be[a:e + 1])
                keep = np.diag(mask[a:e + 1].astype(float))
                Bz[a:e + 1, a:e + 1] = np.linalg.matrix_power(keep @ one, K)
            if np.any(mask == 0):
                assert np.abs(sea @ Bz @ sea - G).max() > 1e-6


# ---------------------------------------------------------------- coasts
@pytest.mark.parametrize("n_img", [0, 1, 2, 4])
def test_segments_match_brute_force(orc, n_img):
    rng = np.random.default_rng(100 + n_img)
    for _ in range(40):
        m = int(rng.integers(1, 40))
        mask = (rng.uniform(size=m) > rng.uniform(0.1, 0.7)).astype(np.uint8)
        seg, kind, segs = orc.segments(mask, n_img)
        assert segs == brute_segments(list(mask), n_img)
        assert np.all((kind == 1) == (mask == 1))


@pytest.mark.parametrize("n_img", [0, 3])
def test_masked_line_is_block_diagonal_over_segments(orc, n_img):
    rng = np.random.default_rng(21)
    m = 45
    mask = np.ones(m, np.uint8)
    mask[[7, 8, 9, 20, 31, 32]] = 0
    sig = rng.uniform(1.5, 4.0, m)
    P = line_problem(orc, sig, mask=mask, n_img=n_img)
    G = dense_operator(orc, P)
    al = orc.coef3(sig, 0)
    Gb = np.zeros((m, m))
    for a, e in brute_segments(list(mask), n_img):
        Gb[a:e + 1, a:e + 1] = brute_rf3_segment(al[:3, a:e + 1], al[3, a:e + 1])
    sea = np.diag(mask.astype(float))
    np.testing.assert_allclose(G, sea @ Gb @ sea, rtol=1e-12, atol=1e-14)


def test_land_blocks_information(orc):
    m = 60
    mask = np.ones(m, np.uint8)
    mask[30] = 0
    P = line_problem(orc, np.full(m, 5.0), mask=mask)
    x = np.zeros((1, m))
    x[0, 10] = 1.0
    y = P.apply_dir(x, "x")[0]
    assert np.all(y[30:] == 0.0) and y[10] > 0


def test_leading_imaginary_points_do_not_change_rf3_sea_output(orc):
    """Zero input and zero state before the run: the extension before a run has no effect on one 3rd-RF pass."""
    m = 50
    mask = np.zeros(m, np.uint8)
    mask[10:35] = 1
    rng = np.random.default_rng(4)
    sig = rng.uniform(2, 5, m)
    x = rng.standard_normal((1, m))
    P0 = line_problem(orc, sig, mask=mask, n_img=0)
    Plead = orc.Problem(mask[None], sig[None], sig[None], n_img=4)
    y0 = P0.apply_dir(x, "x")[0]
    y4 = Plead.apply_dir(x, "x")[0]
    # only trailing imaginary points (after the run) change the sea output
    G = brute_rf3_segment(orc.coef3(sig[6:39], 0)[:3], orc.coef3(sig[6:39], 0)[3])
    xs = np.where(mask[6:39] == 1, x[0, 6:39], 0.0)
    np.testing.assert_allclose(y4[6:39], (G @ xs) * mask[6:39], rtol=1e-12, atol=1e-14)
    Gnolead = brute_rf3_segment(orc.coef3(sig[10:39], 0)[:3], orc.coef3(sig[10:39], 0)[3])
    np.testing.assert_allclose(y4[10:35], (Gnolead @ xs[4:])[:25], rtol=1e-12, atol=1e-14)
    assert np.abs(y4[10:35] - y0[10:35]).max() > 1e-6      # the trailing extension matters


def test_edge_variance_damping_is_one_sided(orc):
    """Zero-state initial conditions: diag(G) stays near its interior value at the start of the causal
    sweep and collapses at the far end."""
    P = line_problem(orc, np.full(40, 4.0))
    G = dense_operator(orc, P)
    d = np.diag(G) / G[20, 20]
    assert d[0] > 0.5 and d[-1] < 0.02


# ---------------------------------------------------------------- 2-D operator
def random_problem(orc, ny, nx, rng, land=0.3, n_img=2, qmode=0, nlev=1):
    mask = (rng.uniform(size=(nlev, ny, nx)) > land).astype(np.uint8)
    sx = rng.uniform(1.0, 6.0, (nlev, ny, nx))
    sy = rng.uniform(1.0, 6.0, (nlev, ny, nx))
    return orc.Problem(mask, sx, sy, n_img=n_img, qmode=qmode)


@pytest.mark.parametrize("qmode", [0, 2])
def test_2d_adjoint_identity(orc, qmode):
    rng = np.random.default_rng(9)
    P = random_problem(orc, 23, 31, rng, qmode=qmode, nlev=3)
    x = rng.standard_normal((2, 3, 23, 31))
    y = rng.standard_normal((2, 3, 23, 31))
    lhs = np.vdot(P.rf3(x), y)
    rhs = np.vdot(x, P.rf3_adjoint(y))
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("op", ["rf3", "rf3_adjoint", "rf1"])
def test_per_level_mask_and_sigma_slices_are_single_level_problems(orc, op):
    """Depth-dependent mask and sigma (mask_nlev = sigma_nlev = nlev) with several fields: every
    (field, level) slice of the output equals the single-level problem built from that level's
    mask and sigma alone, and the 2-D broadcast form (mask_nlev = sigma_nlev = 1) equals per-level
    tables that repeat the 2-D ones."""
    rng = np.random.default_rng(31)
    nf, nlev, ny, nx = 2, 3, 19, 26
    mask = (rng.uniform(size=(nlev, ny, nx)) > np.array([0.2, 0.35, 0.5])[:, None, None]).astype(np.uint8)
    sx = rng.uniform(1.2, 7.0, (nlev, ny, nx))
    sy = rng.uniform(1.2, 7.0, (nlev, ny, nx))
    x = rng.standard_normal((nf, nlev, ny, nx))
    P = orc.Problem(mask, sx, sy, n_img=2, qmode=2, k1=3)
    run = {"rf3": lambda Q, f: Q.rf3(f), "rf3_adjoint": lambda Q, f: Q.rf3_adjoint(f),
           "rf1": lambda Q, f: Q.rf1(f, K=3)}[op]
    out = run(P, x)
    for k in range(nlev):
        Q = orc.Problem(mask[k], sx[k], sy[k], n_img=2, qmode=2, k1=3)
        for f in range(nf):
            np.testing.assert_array_equal(out[f, k], run(Q, x[f, k]))
    # levels really differ (a per-level table indexing slip would show here)
    assert not np.array_equal(mask[0], mask[2])
    P2 = orc.Problem(mask[1], sx[1], sy[1], n_img=2, qmode=2, k1=3)
    Prep = orc.Problem(np.repeat(mask[1:2], nlev, 0), np.repeat(sx[1:2], nlev, 0), np.repeat(sy[1:2], nlev, 0),
                       n_img=2, qmode=2, k1=3)
    np.testing.assert_array_equal(run(P2, x), run(Prep, x))


def test_2d_is_rows_then_columns(orc):
    """V_H = G_y G_x (Sec. 2.2): the 2-D oracle equals the dense Kronecker-structured product."""
    rng = np.random.default_rng(12)
    ny, nx = 6, 7
    P = random_problem(orc, ny, nx, rng, land=0.2, n_img=1)
    N = ny * nx
    E = np.eye(N).reshape(N, ny, nx)
    V = np.stack([P.rf3(E[k]).ravel() for k in range(N)], axis=1)
    Gx = np.stack([P.apply_dir(E[k], "x").ravel() for k in range(N)], axis=1)
    Gy = np.stack([P.apply_dir(E[k], "y").ravel() for k in range(N)], axis=1)
    np.testing.assert_allclose(V, Gy @ Gx, rtol=1e-12, atol=1e-14)
    # each direction acts on single lines only
    for k in range(N):
        j, i = divmod(k, nx)
        col = Gx[:, k].reshape(ny, nx)
        assert np.all(np.delete(col, j, axis=0) == 0)
        col = Gy[:, k].reshape(ny, nx)
        assert np.all(np.delete(col, i, axis=1) == 0)


def test_2d_constant_field_interior(orc):
    ny, nx, sx, sy = 181, 201, 3.0, 4.5
    P = orc.Problem(np.ones((ny, nx)), np.full((ny, nx), sx), np.full((ny, nx), sy))
    out = P.rf3(np.full((ny, nx), 2.0))
    assert out[90, 100] == pytest.approx(2.0 * 2 * np.pi * sx * sy, rel=1e-7)  # IIR tail truncated ~20 e-folds from the edge
    out1 = P.rf1(np.full((ny, nx), 2.0), K=5)
    assert out1[90, 100] == pytest.approx(2.0, rel=1e-9)


def test_remark1_corrected_bound_against_gaussian_convolution(orc):
    """Remark 1 with Cauchy-Schwarz in the infinity norm: |eps_s|_inf <= |eps_h|_2 |s0|_2 for uniform sigma
    away from the ends, and Young's form |eps_s|_2 <= |eps_h|_1 |s0|_2."""
    rng = np.random.default_rng(8)
    m, sigma = 801, 4.0
    for qmode in (0, 2):
        h = impulse(orc, m, sigma, qmode)
        g = gaussian(m, sigma)
        eh = g - h
        s0 = np.zeros(m)
        s0[350:451] = rng.standard_normal(101)
        P = line_problem(orc, np.full(m, sigma), qmode=qmode)
        srf = P.apply_dir(s0[None], "x")[0]
        sstar = np.convolve(s0, g, mode="same")
        es = sstar - srf
        assert np.abs(es).max() <= np.linalg.norm(eh) * np.linalg.norm(s0) * (1 + 1e-9)
        assert np.linalg.norm(es) <= np.abs(eh).sum() * np.linalg.norm(s0) * (1 + 1e-9)


def test_2d_brute_force_gaussian_convolution_tiny_grid(orc):
    """On an all-sea grid the 2-D filter approximates the separable Gaussian convolution; the error
    obeys the corrected Remark-1 bound with the 2-D impulse-response error."""
    rng = np.random.default_rng(10)
    ny, nx, sigma = 121, 121, 3.0
    P = orc.Problem(np.ones((ny, nx)), np.full((ny, nx), sigma), np.full((ny, nx), sigma), qmode=2)
    imp = np.zeros((ny, nx))
    imp[60, 60] = 1.0
    h = P.rf3(imp)
    yy, xx = np.mgrid[0:ny, 0:nx]
    g = np.exp(-((yy - 60) ** 2 + (xx - 60) ** 2) / (2 * sigma * sigma))
    s0 = np.zeros((ny, nx))
    s0[50:71, 50:71] = rng.standard_normal((21, 21))
    srf = P.rf3(s0)
    gs = gaussian(ny, sigma)
    sstar = np.apply_along_axis(lambda r: np.convolve(r, gs, "same"), 1, s0)
    sstar = np.apply_along_axis(lambda c: np.convolve(c, gs, "same"), 0, sstar)
    eh = np.linalg.norm(g - h)
    assert np.abs(sstar - srf).max() <= eh * np.linalg.norm(s0) * (1 + 1e-9)
    assert np.linalg.norm(sstar - srf) / np.linalg.norm(sstar) < 0.05
