/*
 * FP64 CPU oracle for the recursive-filter horizontal covariance operator of
 * Farina, Dobricic, Storto, Masina, Cuomo, "A Revised Scheme to Compute
 * Horizontal Covariances in an Oceanographic 3D-VAR Assimilation System"
 * (arXiv:1404.5756).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or constant with the GPU path.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark load it.
 *
 * Every routine follows the paper step by step, in double precision:
 *   - 3rd-RF coefficients: Theorem 3.1 (Sec. 3.1) and its proof (Appendix A,
 *     eqs. "indietro"/"avanti" and the gain constraint eqs. "avanti3/4").
 *   - 3rd-RF sweeps: eqs. "fort" (causal) and "bact" (anti-causal) with the
 *     heuristic initial conditions of Sec. 3.1 (zero state before the line).
 *   - 1st-RF: eqs. "proc1-1"/"proc1-2" with the Hayden relation, eq. "crucial",
 *     solved as in eq. "evi" and the expressions that follow it.
 *   - V_H = G_y G_x: Sec. 2.2; the 2-D filter is the 1-D filter applied on
 *     every row and then on every column (Sec. 3, separability).
 *   - Adjoint: the transpose of the composed sweeps (derived, see below).
 *
 * Readings of points the paper leaves open:
 *   - coasts: each maximal run of sea points along a line is extended by
 *     up to n_img "imaginary sea points" taken from the adjacent land points;
 *     a land point goes to the nearer run (ties: the lower-index run).  The
 *     extended runs ("segments") are filtered independently; imaginary points
 *     take zero input, run the recursion with their own sigma, and their
 *     output is set to zero.
 *   - the heuristic initial conditions equal a zero state outside a segment,
 *     at both of its ends.
 *   - q(sigma): the Theorem inserts sigma = R/dx into the a_k polynomials.
 *     Mode LITERAL does exactly that; VARMATCH and FIT substitute a
 *     re-parametrised q while beta keeps the true sigma (so the DC gain stays
 *     sqrt(2 pi) sigma per direction).
 *   - 1st-RF order: all K iterations along x, then all K along y; values at
 *     imaginary points are kept between iterations.
 *
 * Two options beyond the paper's scheme (flags of the grid):
 *   - ORC_PERIODIC_X: rows are zonally periodic (a global grid; the paper treats
 *     finite lines only).  Sea runs and imaginary points are found on the cycle
 *     (a run may wrap from i = nx-1 to i = 0); a row with no land at all is one
 *     cyclic line whose recurrences have no start: their periodic solution is
 *     the fixed point of one lap, x = Phi x + b, a 3x3 solve per line.
 *   - ORC_EXACT_ENDS: end conditions of the anti-causal 3rd-RF sweep that make
 *     each segment's operator the infinite-line filter restricted to the
 *     segment (input zero outside it, the coefficients of the segment's last
 *     point continued past its end).  The causal sweep's zero start is already
 *     exact for zero input before the segment; past the end the causal output
 *     decays through the homogeneous recurrence, and the anti-causal sweep's
 *     three starting values are a 3x3 matrix times the last three causal values
 *     (Sec. 6 names other boundary conditions at coasts as further work).  The
 *     1st-RF keeps the paper's zero ends.
 *
 * Parity pins for this file live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* q(sigma) readings                                                       */
/* ---------------------------------------------------------------------- */

/* Theorem 3.1 constants of the a_{i,k} polynomials (Sec. 3.1). */
static const double TH_C0 = 3.738128;
static const double TH_C1 = 5.788982;
static const double TH_C2 = 3.382473;

/* Variance of one causal sweep of the Theorem's filter, as a function of q,
 * from the generating function 1/D(1-w) with
 *   D(s) = C0 + C1 q s + C2 q^2 s^2 + q^3 s^3:
 *   mean = (C1/C0) q,  var = (C1/C0) q + ((C1/C0)^2 - 2 C2/C0) q^2.
 * The causal + anti-causal pair has zero mean and twice this variance. */
static double pair_var_coef_lin(void) { return 2.0 * TH_C1 / TH_C0; }
static double pair_var_coef_sq(void)
{
    double r = TH_C1 / TH_C0;
    return 2.0 * (r * r - 2.0 * TH_C2 / TH_C0);
}

/* FIT reading: q = sigma - F0 + F1/(sigma + F2).  The three constants were
 * fitted to the minimiser of the mass-normalised shape error against the
 * Gaussian of width sigma (oracle/fit_q.py, the only script that produced
 * them, calls nothing but this oracle). */
static const double FIT_F0 = 1.3460094;
static const double FIT_F1 = 1.2463293;
static const double FIT_F2 = 0.6031649;

double orc_qmap(int mode, double sigma)
{
    if (mode == 0) return sigma;                       /* LITERAL */
    if (mode == 1) {                                   /* VARMATCH */
        double A = pair_var_coef_sq(), B = pair_var_coef_lin();
        return (-B + sqrt(B * B + 4.0 * A * sigma * sigma)) / (2.0 * A);
    }
    /* FIT */
    return sigma - FIT_F0 + FIT_F1 / (sigma + FIT_F2);
}

double orc_pair_var_coef(int which) { return which ? pair_var_coef_sq() : pair_var_coef_lin(); }

/* ---------------------------------------------------------------------- */
/* Coefficients                                                            */
/* ---------------------------------------------------------------------- */

/* Theorem 3.1: a_{i,0..3} from q = R_i/dx_i (or its re-parametrisation),
 * alpha_{i,k} = a_{i,k}/a_{i,0},
 * beta_i = (2 pi sigma^2)^(1/4) (1 - (alpha_1 + alpha_2 + alpha_3)). */
void orc_coef3(int mode, double sigma, double *al1, double *al2, double *al3, double *beta)
{
    double q = orc_qmap(mode, sigma);
    double q2 = q * q, q3 = q2 * q;
    double a0 = 3.738128 + 5.788982 * q + 3.382473 * q2 + 1.000000 * q3;
    double a1 = 5.788982 * q + 6.764946 * q2 + 3.000000 * q3;
    double a2 = -3.382473 * q2 - 3.000000 * q3;
    double a3 = 1.000000 * q3;
    *al1 = a1 / a0;
    *al2 = a2 / a0;
    *al3 = a3 / a0;
    *beta = pow(2.0 * M_PI * sigma * sigma, 0.25) * (1.0 - (*al1 + *al2 + *al3));
}

/* 1st-RF (Sec. 3.1): with E = K dx^2/R^2 = K/sigma^2 the Hayden relation
 * R^2 = 2 K alpha/(1-alpha)^2 dx^2 gives
 *   alpha = 1 + E - sqrt(E (E + 2)),   beta = -E + sqrt(E (E + 2)). */
void orc_coef1(int K, double sigma, double *al, double *beta)
{
    double E = (double)K / (sigma * sigma);
    double r = sqrt(E * (E + 2.0));
    *al = 1.0 + E - r;
    *beta = -E + r;
}

/* ---------------------------------------------------------------------- */
/* Segments along one line                                                 */
/* ---------------------------------------------------------------------- */

/* seg[i] = index of the segment point i belongs to, or -1 (inactive land).
 * kind[i] = 1 sea, 2 imaginary, 0 inactive.  Returns the segment count and
 * fills starts[]/ends[] (inclusive), which must hold n entries. */
int orc_segments(const uint8_t *mask, long stride, int n, int n_img,
                 int *seg, uint8_t *kind, int *starts, int *ends)
{
    /* maximal sea runs */
    int nrun = 0;
    for (int i = 0; i < n; ++i) {
        int sea = mask[(long)i * stride] != 0;
        if (sea && (i == 0 || mask[(long)(i - 1) * stride] == 0)) {
            starts[nrun] = i;
            ends[nrun] = i;
            ++nrun;
        }
        if (sea) ends[nrun - 1] = i;
    }
    for (int i = 0; i < n; ++i) { seg[i] = -1; kind[i] = 0; }
    for (int r = 0; r < nrun; ++r)
        for (int i = starts[r]; i <= ends[r]; ++i) { seg[i] = r; kind[i] = 1; }
    /* imaginary points: each land point within n_img of a run joins the
     * nearer run; equal distance goes to the lower-index run. */
    for (int i = 0; i < n; ++i) {
        if (kind[i] == 1) continue;
        int best = -1, bestd = n_img + 1;
        for (int r = 0; r < nrun; ++r) {
            int d;
            if (i < starts[r]) d = starts[r] - i;
            else if (i > ends[r]) d = i - ends[r];
            else continue;
            if (d < bestd) { bestd = d; best = r; }   /* strict: ties keep lower r */
        }
        if (best >= 0 && bestd <= n_img) { seg[i] = best; kind[i] = 2; }
    }
    /* extended segment bounds */
    for (int r = 0; r < nrun; ++r) {
        int a = starts[r], e = ends[r];
        while (a - 1 >= 0 && seg[a - 1] == r) --a;
        while (e + 1 < n && seg[e + 1] == r) ++e;
        starts[r] = a;
        ends[r] = e;
    }
    return nrun;
}

/* ---------------------------------------------------------------------- */
/* Small dense solves (Gaussian elimination with partial pivoting)         */
/* ---------------------------------------------------------------------- */

/* Solve A x = b in place for an n x n row-major A (n <= 9); b becomes x. */
static void solve_dense(int n, double *A, double *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) { double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double v = b[r];
        for (int k = r + 1; k < n; ++k) v -= A[r * n + k] * b[k];
        b[r] = v / A[r * n + r];
    }
}

/* ---------------------------------------------------------------------- */
/* Exact end of a segment (ORC_EXACT_ENDS)                                 */
/* ---------------------------------------------------------------------- */

/* Past the segment end e the input is zero and the coefficients of e
 * (al1, al2, al3, beta) continue.  With the companion matrix
 *   C = [[al1, al2, al3], [1, 0, 0], [0, 1, 0]]
 * the causal state x_j = (p_j, p_{j-1}, p_{j-2}) follows x_j = C x_{j-1} for
 * j > e, and the anti-causal triple y_j = (o_j, o_{j+1}, o_{j+2}) obeys
 * y_j = C y_{j+1} + beta p_j e1, whose decaying solution is
 * y_j = beta sum_{m>=0} C^m e1 p_{j+m}.  Hence
 *   (o_{e+1}, o_{e+2}, o_{e+3}) = M (p_e, p_{e-1}, p_{e-2}),
 *   M = beta X C,  X = sum_{m>=0} C^m e1 e1^T C^m,
 * and X solves X = e1 e1^T + C X C, a 9x9 linear system.  M is row-major. */
static void exact_end_matrix(double al1, double al2, double al3, double beta, double *M)
{
    const double C[9] = {al1, al2, al3, 1, 0, 0, 0, 1, 0};
    double A[81], x[9];
    /* unknowns X[r][c] at index 3r + c; equation (r, c):
     * X[r][c] - sum_{k,l} C[r][k] X[k][l] C[l][c] = (r == 0 && c == 0) */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double *row = A + 9 * (3 * r + c);
            for (int u = 0; u < 9; ++u) row[u] = (u == 3 * r + c) ? 1.0 : 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) row[3 * k + l] -= C[3 * r + k] * C[3 * l + c];
            x[3 * r + c] = (r == 0 && c == 0) ? 1.0 : 0.0;
        }
    solve_dense(9, A, x);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += x[3 * r + k] * C[3 * k + c];
            M[3 * r + c] = beta * v;
        }
}

/* ---------------------------------------------------------------------- */
/* Recurrences on a cycle (ORC_PERIODIC_X, a row with no land)             */
/* ---------------------------------------------------------------------- */

/* Periodic solution of x_i = u_i + sum_{k=1..3} c[3i+k-1] x_{(i-k) mod n}
 * (dir > 0, ascending) or x_i = u_i + sum_k c[3i+k-1] x_{(i+k) mod n}
 * (dir < 0, descending), i = 0..n-1.  One lap of the recurrence from the state
 * s (the three values before the first step) ends in Phi s + b, with b the lap
 * from a zero state and the columns of Phi the laps from unit states with zero
 * input; the periodic solution starts from the fixed point s = (I - Phi)^-1 b. */
static void cyc_lap(int n, int dir, const double *c, const double *u, const double *s_in,
                    double *s_out, double *x)
{
    double s0 = s_in[0], s1 = s_in[1], s2 = s_in[2];   /* x one, two, three steps back */
    for (int t = 0; t < n; ++t) {
        int i = dir > 0 ? t : n - 1 - t;
        double v = (u ? u[i] : 0.0) + c[3 * i] * s0 + c[3 * i + 1] * s1 + c[3 * i + 2] * s2;
        if (x) x[i] = v;
        s2 = s1; s1 = s0; s0 = v;
    }
    s_out[0] = s0; s_out[1] = s1; s_out[2] = s2;
}

static void cyc_solve(int n, int dir, const double *c, const double *u, double *x)
{
    const double zero[3] = {0, 0, 0};
    double b[3], A[9];
    cyc_lap(n, dir, c, u, zero, b, NULL);
    for (int k = 0; k < 3; ++k) {
        double e[3] = {0, 0, 0}, col[3];
        e[k] = 1.0;
        cyc_lap(n, dir, c, NULL, e, col, NULL);
        for (int r = 0; r < 3; ++r) A[3 * r + k] = (r == k ? 1.0 : 0.0) - col[r];
    }
    solve_dense(3, A, b);
    double end[3];
    cyc_lap(n, dir, c, u, b, end, x);
}

/* ---------------------------------------------------------------------- */
/* 3rd-RF on one segment                                                   */
/* ---------------------------------------------------------------------- */

/* Causal sweep, eq. "fort" with the forward initial conditions: for
 * i = a..e, p_i = beta_i s_i + sum_{k=1..3, i-k>=a} alpha_{i,k} p_{i-k}.
 * Anti-causal sweep, eq. "bact" with the backward initial conditions: for
 * i = e..a, o_i = beta_i p_i + sum_{k=1..3, i+k<=e} alpha_{i,k} o_{i+k}.
 * al is [n][3], beta [n]; s, p, o are [n]. */
static void rf3_segment(int a, int e, const double *al, const double *beta,
                        const double *s, double *p, double *o, int exact)
{
    for (int i = a; i <= e; ++i) {
        double v = beta[i] * s[i];
        if (i - 1 >= a) v += al[3 * i + 0] * p[i - 1];
        if (i - 2 >= a) v += al[3 * i + 1] * p[i - 2];
        if (i - 3 >= a) v += al[3 * i + 2] * p[i - 3];
        p[i] = v;
    }
    /* o past the end: zero (the paper's initial conditions) or, with exact
     * ends, M (p_e, p_{e-1}, p_{e-2}) */
    double tail[3] = {0, 0, 0};
    if (exact) {
        double M[9], x[3];
        exact_end_matrix(al[3 * e], al[3 * e + 1], al[3 * e + 2], beta[e], M);
        for (int k = 0; k < 3; ++k) x[k] = e - k >= a ? p[e - k] : 0.0;
        for (int r = 0; r < 3; ++r) tail[r] = M[3 * r] * x[0] + M[3 * r + 1] * x[1] + M[3 * r + 2] * x[2];
    }
    for (int i = e; i >= a; --i) {
        double v = beta[i] * p[i];
        v += al[3 * i + 0] * (i + 1 <= e ? o[i + 1] : tail[i + 1 - e - 1]);
        v += al[3 * i + 1] * (i + 2 <= e ? o[i + 2] : tail[i + 2 - e - 1]);
        v += al[3 * i + 2] * (i + 3 <= e ? o[i + 3] : tail[i + 3 - e - 1]);
        o[i] = v;
    }
}

/* Transpose of rf3_segment.  With L = I - A_c ((A_c)_{i,i-k} = alpha_{i,k})
 * and U = I - A_a ((A_a)_{i,i+k} = alpha_{i,k}), the segment operator is
 * G = U^-1 D_beta L^-1 D_beta, so G^T = D_beta L^-T D_beta U^-T:
 *   z_j = y_j + sum_k alpha_{j-k,k} z_{j-k}     (ascending, source-indexed)
 *   w   = beta o z
 *   u_j = w_j + sum_k alpha_{j+k,k} u_{j+k}     (descending, source-indexed)
 *   out = beta o u. */
static void rf3_segment_adj(int a, int e, const double *al, const double *beta,
                            const double *y, double *z, double *o, int exact)
{
    for (int j = a; j <= e; ++j) {
        double v = y[j];
        if (j - 1 >= a) v += al[3 * (j - 1) + 0] * z[j - 1];
        if (j - 2 >= a) v += al[3 * (j - 2) + 1] * z[j - 2];
        if (j - 3 >= a) v += al[3 * (j - 3) + 2] * z[j - 3];
        z[j] = v;
    }
    /* exact ends: the forward anti-causal input at e - t gains
     * sum_k J[t][k] (M x)_k with x = (p_e, p_{e-1}, p_{e-2}) and
     * J = [[al_{e,1}, al_{e,2}, al_{e,3}], [al_{e-1,2}, al_{e-1,3}, 0], [al_{e-2,3}, 0, 0]]
     * (the terms of o_{e+1..e+3} in rows e, e-1, e-2); its transpose adds
     * M^T J^T (z_e, z_{e-1}, z_{e-2}) to (w_e, w_{e-1}, w_{e-2}), w = beta z. */
    double add[3] = {0, 0, 0};
    if (exact) {
        double M[9], J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, zt[3], t[3];
        exact_end_matrix(al[3 * e], al[3 * e + 1], al[3 * e + 2], beta[e], M);
        J[0] = al[3 * e]; J[1] = al[3 * e + 1]; J[2] = al[3 * e + 2];
        if (e - 1 >= a) { J[3] = al[3 * (e - 1) + 1]; J[4] = al[3 * (e - 1) + 2]; }
        if (e - 2 >= a) { J[6] = al[3 * (e - 2) + 2]; }
        for (int k = 0; k < 3; ++k) zt[k] = e - k >= a ? z[e - k] : 0.0;
        for (int k = 0; k < 3; ++k) t[k] = J[k] * zt[0] + J[3 + k] * zt[1] + J[6 + k] * zt[2];   /* J^T zt */
        for (int k = 0; k < 3; ++k) add[k] = M[k] * t[0] + M[3 + k] * t[1] + M[6 + k] * t[2];    /* M^T t */
    }
    for (int j = a; j <= e; ++j) z[j] *= beta[j];
    for (int k = 0; k < 3; ++k)
        if (e - k >= a) z[e - k] += add[k];
    for (int j = e; j >= a; --j) {
        double v = z[j];
        if (j + 1 <= e) v += al[3 * (j + 1) + 0] * o[j + 1];
        if (j + 2 <= e) v += al[3 * (j + 2) + 1] * o[j + 2];
        if (j + 3 <= e) v += al[3 * (j + 3) + 2] * o[j + 3];
        o[j] = v;
    }
    for (int j = a; j <= e; ++j) o[j] *= beta[j];
}

/* 1st-RF, eqs. "proc1-1"/"proc1-2", K iterations on one segment; the input of
 * iteration k+1 is the output of iteration k (values at imaginary points
 * included). */
static void rf1_segment(int a, int e, int K, const double *al, const double *beta,
                        double *s, double *p)
{
    for (int k = 0; k < K; ++k) {
        p[a] = beta[a] * s[a];
        for (int i = a + 1; i <= e; ++i) p[i] = beta[i] * s[i] + al[i] * p[i - 1];
        s[e] = beta[e] * p[e];
        for (int i = e - 1; i >= a; --i) s[i] = beta[i] * p[i] + al[i] * s[i + 1];
    }
}

/* The three line operators on a cycle of n points (a periodic row with no
 * land): the same sweeps as above with indices taken mod n, each sweep the
 * periodic solution of its recurrence (cyc_solve).  al is [n][3], beta [n];
 * s is the input (modified by the 1st-RF), o the output; w is [n][3] scratch. */
static void rf3_cycle(int n, const double *al, const double *beta, const double *s, double *p,
                      double *o, double *u, double *w)
{
    for (int i = 0; i < n; ++i) u[i] = beta[i] * s[i];
    cyc_solve(n, 1, al, u, p);
    for (int i = 0; i < n; ++i) u[i] = beta[i] * p[i];
    cyc_solve(n, -1, al, u, o);
    (void)w;
}

static void rf3_cycle_adj(int n, const double *al, const double *beta, const double *y, double *z,
                          double *o, double *u, double *w)
{
    /* transposed sweeps with source-indexed coefficients:
     * z_j = y_j + sum_k al_{j-k,k} z_{j-k};  u_j = beta_j z_j + sum_k al_{j+k,k} u_{j+k};  out = beta u */
    for (int j = 0; j < n; ++j)
        for (int k = 1; k <= 3; ++k) w[3 * j + k - 1] = al[3 * (((j - k) % n + n) % n) + k - 1];
    cyc_solve(n, 1, w, y, z);
    for (int j = 0; j < n; ++j) {
        u[j] = beta[j] * z[j];
        for (int k = 1; k <= 3; ++k) w[3 * j + k - 1] = al[3 * ((j + k) % n) + k - 1];
    }
    cyc_solve(n, -1, w, u, o);
    for (int j = 0; j < n; ++j) o[j] *= beta[j];
}

static void rf1_cycle(int n, int K, const double *al, const double *beta, double *s, double *p,
                      double *u, double *w)
{
    for (int i = 0; i < n; ++i) { w[3 * i] = al[i]; w[3 * i + 1] = 0.0; w[3 * i + 2] = 0.0; }
    for (int k = 0; k < K; ++k) {
        for (int i = 0; i < n; ++i) u[i] = beta[i] * s[i];
        cyc_solve(n, 1, w, u, p);
        for (int i = 0; i < n; ++i) u[i] = beta[i] * p[i];
        cyc_solve(n, -1, w, u, s);
    }
}

/* ---------------------------------------------------------------------- */
/* Lines of a 3-D grid                                                     */
/* ---------------------------------------------------------------------- */

enum { ORC_PERIODIC_X = 1, ORC_EXACT_ENDS = 2 };

typedef struct {
    int nx, ny, nlev, mask_nlev, sigma_nlev, n_img, qmode, k1, flags;
} orc_grid;

/* Segments of a periodic line (ORC_PERIODIC_X): the same reading as
 * orc_segments with distances taken around the cycle; a land point at equal
 * distance from two runs joins the run before it.  A segment is the run's
 * leading imaginary points (those the run follows), the run, and its trailing
 * ones (those that follow the run); it may wrap (starts[r] > ends[r]).  Returns the segment count; 0 with *whole = 1 when
 * the line has no land (one cyclic line), 0 with *whole = 0 when it has no sea. */
int orc_segments_cyclic(const uint8_t *mask, long stride, int n, int n_img,
                        int *seg, uint8_t *kind, int *starts, int *ends, int *whole)
{
    int nsea = 0, first_land = -1;
    for (int i = 0; i < n; ++i) {
        if (mask[(long)i * stride]) ++nsea;
        else if (first_land < 0) first_land = i;
    }
    *whole = nsea == n;
    for (int i = 0; i < n; ++i) { seg[i] = nsea == n ? 0 : -1; kind[i] = nsea == n ? 1 : 0; }
    if (nsea == n || nsea == 0) return 0;
    /* runs, scanning the cycle from the first land point */
    int nrun = 0;
    for (int t = 1; t <= n; ++t) {
        int i = (first_land + t) % n, ip = (first_land + t - 1) % n;
        int sea = mask[(long)i * stride] != 0, prev = mask[(long)ip * stride] != 0;
        if (sea && !prev) { starts[nrun] = i; ends[nrun] = i; ++nrun; }
        if (sea) { ends[nrun - 1] = i; seg[i] = nrun - 1; kind[i] = 1; }
    }
    /* trail[i]: the imaginary point i follows its run (it extends the run's end);
     * otherwise it precedes the run (it extends the run's start) */
    uint8_t *trail = malloc(n);
    for (int i = 0; i < n; ++i) {
        trail[i] = 0;
        if (kind[i] == 1) continue;
        int best = -1, bestd = n_img + 1, best_before = 0;
        for (int r = 0; r < nrun; ++r) {
            int dbefore = ((i - ends[r]) % n + n) % n;     /* run r precedes i */
            int dafter = ((starts[r] - i) % n + n) % n;    /* run r follows i */
            int d = dbefore <= dafter ? dbefore : dafter;
            int before = dbefore <= dafter;
            if (d < bestd || (d == bestd && before && !best_before)) { bestd = d; best = r; best_before = before; }
        }
        if (best >= 0 && bestd <= n_img) { seg[i] = best; kind[i] = 2; trail[i] = (uint8_t)best_before; }
    }
    /* a segment is its leading imaginary points, the run, its trailing ones */
    for (int r = 0; r < nrun; ++r) {
        int a = starts[r], e = ends[r];
        while (seg[(a - 1 + n) % n] == r && kind[(a - 1 + n) % n] == 2 && !trail[(a - 1 + n) % n]) a = (a - 1 + n) % n;
        while (seg[(e + 1) % n] == r && kind[(e + 1) % n] == 2 && trail[(e + 1) % n]) e = (e + 1) % n;
        starts[r] = a;
        ends[r] = e;
    }
    free(trail);
    return nrun;
}

enum { OP_RF3 = 0, OP_RF3_ADJ = 1, OP_RF1 = 2 };

/* Apply one 1-D operator to every line of one direction.  dir 0 = x (rows),
 * dir 1 = y (columns).  fld is [nlev][ny][nx], modified in place. */
static void apply_dir(const orc_grid *g, int dir, int op, int K, const uint8_t *mask,
                      const double *sig, double *fld, int nlev, int nthreads)
{
    const int nx = g->nx, ny = g->ny;
    const int n = dir == 0 ? nx : ny;
    const int nlines = dir == 0 ? ny : nx;
    const long estride = dir == 0 ? 1 : nx;
    const long total = (long)nlev * nlines;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *al = malloc(sizeof(double) * 3 * n);
        double *be = malloc(sizeof(double) * n);
        double *s = malloc(sizeof(double) * n);
        double *p = malloc(sizeof(double) * n);
        double *o = malloc(sizeof(double) * n);
        int *seg = malloc(sizeof(int) * n);
        int *st = malloc(sizeof(int) * n);
        int *en = malloc(sizeof(int) * n);
        uint8_t *kind = malloc(n);
        /* gathered copies of one wrapped segment, and cycle scratch */
        double *gal = malloc(sizeof(double) * 3 * n);
        double *gbe = malloc(sizeof(double) * n);
        double *gs = malloc(sizeof(double) * n);
        double *gp = malloc(sizeof(double) * n);
        double *go = malloc(sizeof(double) * n);
        double *gw = malloc(sizeof(double) * 3 * n);
        const int periodic = dir == 0 && (g->flags & ORC_PERIODIC_X);
        const int exact = (g->flags & ORC_EXACT_ENDS) != 0;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long t = 0; t < total; ++t) {
            int lev = (int)(t / nlines), line = (int)(t % nlines);
            long base = (long)lev * nx * ny + (dir == 0 ? (long)line * nx : line);
            const uint8_t *mk = mask + (g->mask_nlev > 1 ? (long)lev * nx * ny : 0)
                                + (dir == 0 ? (long)line * nx : line);
            const double *sg = sig + (g->sigma_nlev > 1 ? (long)lev * nx * ny : 0)
                               + (dir == 0 ? (long)line * nx : line);
            int whole = 0;
            int nseg = periodic ? orc_segments_cyclic(mk, estride, n, g->n_img, seg, kind, st, en, &whole)
                                : orc_segments(mk, estride, n, g->n_img, seg, kind, st, en);
            for (int i = 0; i < n; ++i) {
                double sv = fld[base + i * estride];
                s[i] = kind[i] == 1 ? sv : 0.0;   /* land and imaginary input ignored */
                p[i] = 0.0;
                o[i] = 0.0;
                if (kind[i] != 0) {
                    if (op == OP_RF1) {
                        orc_coef1(K, sg[i * estride], &al[i], &be[i]);
                    } else {
                        orc_coef3(g->qmode, sg[i * estride], &al[3 * i], &al[3 * i + 1],
                                  &al[3 * i + 2], &be[i]);
                    }
                }
            }
            if (whole) {   /* periodic row without land: one cyclic line */
                if (op == OP_RF3) rf3_cycle(n, al, be, s, p, o, gs, gw);
                else if (op == OP_RF3_ADJ) rf3_cycle_adj(n, al, be, s, p, o, gs, gw);
                else { rf1_cycle(n, K, al, be, s, p, gs, gw); memcpy(o, s, sizeof(double) * n); }
            }
            for (int r = 0; r < nseg; ++r) {
                /* the points of segment r in order (a wrapped segment runs through i = n-1 to 0),
                 * gathered, filtered as one finite line, and scattered back */
                const int m = (en[r] - st[r] + n) % n + 1;
                for (int t = 0; t < m; ++t) {
                    const int i = (st[r] + t) % n;
                    gs[t] = s[i];
                    gbe[t] = be[i];
                    if (op == OP_RF1) gal[t] = al[i];
                    else for (int k = 0; k < 3; ++k) gal[3 * t + k] = al[3 * i + k];
                }
                if (op == OP_RF3) rf3_segment(0, m - 1, gal, gbe, gs, gp, go, exact);
                else if (op == OP_RF3_ADJ) rf3_segment_adj(0, m - 1, gal, gbe, gs, gp, go, exact);
                else { rf1_segment(0, m - 1, K, gal, gbe, gs, gp); memcpy(go, gs, sizeof(double) * m); }
                for (int t = 0; t < m; ++t) o[(st[r] + t) % n] = go[t];
            }
            for (int i = 0; i < n; ++i)
                fld[base + i * estride] = kind[i] == 1 ? o[i] : 0.0;
        }
        free(al); free(be); free(s); free(p); free(o);
        free(seg); free(st); free(en); free(kind);
        free(gal); free(gbe); free(gs); free(gp); free(go); free(gw);
    }
}

/* V_H = G_y G_x on every level of every field (Sec. 2.2).  in/out are
 * [nfields][nlev][ny][nx]; they may alias.  sigma_x/sigma_y are
 * [sigma_nlev][ny][nx] in grid units (R/dx, R/dy); mask is
 * [mask_nlev][ny][nx] with 1 = sea. */
void orc_rf3_apply(const orc_grid *g, const uint8_t *mask, const double *sx, const double *sy,
                   const double *in, double *out, int nlev, int nfields, int nthreads)
{
    long plane = (long)g->nx * g->ny * nlev;
    if (out != in) memcpy(out, in, sizeof(double) * plane * nfields);
    for (int f = 0; f < nfields; ++f) {
        apply_dir(g, 0, OP_RF3, 0, mask, sx, out + f * plane, nlev, nthreads);
        apply_dir(g, 1, OP_RF3, 0, mask, sy, out + f * plane, nlev, nthreads);
    }
}

/* V_H^T = G_x^T G_y^T. */
void orc_rf3_adjoint(const orc_grid *g, const uint8_t *mask, const double *sx, const double *sy,
                     const double *in, double *out, int nlev, int nfields, int nthreads)
{
    long plane = (long)g->nx * g->ny * nlev;
    if (out != in) memcpy(out, in, sizeof(double) * plane * nfields);
    for (int f = 0; f < nfields; ++f) {
        apply_dir(g, 1, OP_RF3_ADJ, 0, mask, sy, out + f * plane, nlev, nthreads);
        apply_dir(g, 0, OP_RF3_ADJ, 0, mask, sx, out + f * plane, nlev, nthreads);
    }
}

/* 1st-RF: K iterations along x, then K along y. */
void orc_rf1_apply(const orc_grid *g, const uint8_t *mask, const double *sx, const double *sy,
                   int K, const double *in, double *out, int nlev, int nfields, int nthreads)
{
    long plane = (long)g->nx * g->ny * nlev;
    if (out != in) memcpy(out, in, sizeof(double) * plane * nfields);
    for (int f = 0; f < nfields; ++f) {
        apply_dir(g, 0, OP_RF1, K, mask, sx, out + f * plane, nlev, nthreads);
        apply_dir(g, 1, OP_RF1, K, mask, sy, out + f * plane, nlev, nthreads);
    }
}

/* One direction only (tests of the 1-D filter). dir 0 = x, 1 = y; op 0 = 3rd-RF,
 * 1 = its adjoint, 2 = 1st-RF with K iterations. */
void orc_apply_dir(const orc_grid *g, int dir, int op, int K, const uint8_t *mask,
                   const double *sig, double *fld, int nlev, int nthreads)
{
    apply_dir(g, dir, op, K, mask, sig, fld, nlev, nthreads);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
