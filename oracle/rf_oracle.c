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
/* 3rd-RF on one segment                                                   */
/* ---------------------------------------------------------------------- */

/* Causal sweep, eq. "fort" with the forward initial conditions: for
 * i = a..e, p_i = beta_i s_i + sum_{k=1..3, i-k>=a} alpha_{i,k} p_{i-k}.
 * Anti-causal sweep, eq. "bact" with the backward initial conditions: for
 * i = e..a, o_i = beta_i p_i + sum_{k=1..3, i+k<=e} alpha_{i,k} o_{i+k}.
 * al is [n][3], beta [n]; s, p, o are [n]. */
static void rf3_segment(int a, int e, const double *al, const double *beta,
                        const double *s, double *p, double *o)
{
    for (int i = a; i <= e; ++i) {
        double v = beta[i] * s[i];
        if (i - 1 >= a) v += al[3 * i + 0] * p[i - 1];
        if (i - 2 >= a) v += al[3 * i + 1] * p[i - 2];
        if (i - 3 >= a) v += al[3 * i + 2] * p[i - 3];
        p[i] = v;
    }
    for (int i = e; i >= a; --i) {
        double v = beta[i] * p[i];
        if (i + 1 <= e) v += al[3 * i + 0] * o[i + 1];
        if (i + 2 <= e) v += al[3 * i + 1] * o[i + 2];
        if (i + 3 <= e) v += al[3 * i + 2] * o[i + 3];
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
                            const double *y, double *z, double *o)
{
    for (int j = a; j <= e; ++j) {
        double v = y[j];
        if (j - 1 >= a) v += al[3 * (j - 1) + 0] * z[j - 1];
        if (j - 2 >= a) v += al[3 * (j - 2) + 1] * z[j - 2];
        if (j - 3 >= a) v += al[3 * (j - 3) + 2] * z[j - 3];
        z[j] = v;
    }
    for (int j = a; j <= e; ++j) z[j] *= beta[j];
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

/* ---------------------------------------------------------------------- */
/* Lines of a 3-D grid                                                     */
/* ---------------------------------------------------------------------- */

typedef struct {
    int nx, ny, nlev, mask_nlev, sigma_nlev, n_img, qmode, k1;
} orc_grid;

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
            int nseg = orc_segments(mk, estride, n, g->n_img, seg, kind, st, en);
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
            for (int r = 0; r < nseg; ++r) {
                if (op == OP_RF3) rf3_segment(st[r], en[r], al, be, s, p, o);
                else if (op == OP_RF3_ADJ) rf3_segment_adj(st[r], en[r], al, be, s, p, o);
                else { rf1_segment(st[r], en[r], K, al, be, s, p); memcpy(o + st[r], s + st[r], sizeof(double) * (en[r] - st[r] + 1)); }
            }
            for (int i = 0; i < n; ++i)
                fld[base + i * estride] = kind[i] == 1 ? o[i] : 0.0;
        }
        free(al); free(be); free(s); free(p); free(o);
        free(seg); free(st); free(en); free(kind);
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
