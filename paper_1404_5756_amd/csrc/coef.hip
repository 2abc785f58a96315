// Setup of the coefficient block: coast codes of every row and column, and the
// per-point filter coefficients of both directions, computed in FP64 on the GPU.
//
//   3rd-RF (Theorem 3.1, Sec. 3.1):
//     a_{i,0} = 3.738128 + 5.788982 q + 3.382473 q^2 + q^3
//     a_{i,1} = 5.788982 q + 6.764946 q^2 + 3 q^3
//     a_{i,2} = -3.382473 q^2 - 3 q^3
//     a_{i,3} = q^3
//     alpha_{i,k} = a_{i,k}/a_{i,0},  beta_i = (2 pi sigma^2)^(1/4) (1 - sum_k alpha_{i,k})
//   with q = q(sigma) per rf_qmode.
//   1st-RF (Hayden relation, eq. "crucial"): E = K/sigma^2,
//     alpha_i = 1 + E - sqrt(E(E+2)),  beta_i = -E + sqrt(E(E+2)).
//
// The FP32 sweeps use the same recurrence rewritten around the small
// quantities gamma = 1 - sum_k alpha_k (= 3.738128/a_0 exactly, since the
// a_{i,k} sum to a_{i,0} - 3.738128), c2 = alpha_2 + alpha_3, c3 = alpha_3;
// they are formed here in FP64 and rounded once.
#include <math.h>

#include "rf3_internal.h"
#include "sweeps.h"

namespace rf {

__device__ inline double qmap(int mode, double sigma)
{
    if (mode == RF_Q_LITERAL) return sigma;
    if (mode == RF_Q_VARMATCH) {
        // variance of the causal+anti-causal pair on an infinite line:
        //   A q^2 + B q,  A = 2((C1/C0)^2 - 2 C2/C0),  B = 2 C1/C0
        const double C0 = 3.738128, C1 = 5.788982, C2 = 3.382473;
        const double r = C1 / C0;
        const double A = 2.0 * (r * r - 2.0 * C2 / C0), B = 2.0 * r;
        return (-B + sqrt(B * B + 4.0 * A * sigma * sigma)) / (2.0 * A);
    }
    return sigma - 1.3460094 + 1.2463293 / (sigma + 0.6031649);   // RF_Q_FIT
}

__device__ inline bool sigma_ok(double s) { return s > 0.0 && s < INFINITY; }

struct Coef3 {
    double al1, al2, al3, beta, gam, c2, c3, beta_g;
};

__device__ inline Coef3 coef3(int mode, double sigma)
{
    Coef3 c;
    const double q = qmap(mode, sigma), q2 = q * q, q3 = q2 * q;
    const double a0 = 3.738128 + 5.788982 * q + 3.382473 * q2 + q3;
    const double a1 = 5.788982 * q + 6.764946 * q2 + 3.0 * q3;
    const double a2 = -3.382473 * q2 - 3.0 * q3;
    const double a3 = q3;
    c.al1 = a1 / a0;
    c.al2 = a2 / a0;
    c.al3 = a3 / a0;
    const double f = sqrt(sqrt(2.0 * M_PI * sigma * sigma));     // (2 pi sigma^2)^(1/4)
    c.beta = f * (1.0 - (c.al1 + c.al2 + c.al3));
    c.gam = 3.738128 / a0;
    c.c2 = (a2 + a3) / a0;
    c.c3 = a3 / a0;
    c.beta_g = f * c.gam;
    return c;
}

// kind of point i of a line: 0 outside every segment, 1 sea, 2 imaginary point
// of the run before it, 3 imaginary point of the run after it.  On a periodic
// line (per) the neighbours are taken around the cycle.
__device__ inline int classify(const uint8_t *m, long es, int n, int i, int n_img, bool per)
{
    if (m[(long)i * es]) return 1;
    int dl = n_img + 1, dr = n_img + 1;
    for (int k = 1; k <= n_img && (per || i - k >= 0); ++k)
        if (m[(long)(((i - k) % n + n) % n) * es]) { dl = k; break; }
    for (int k = 1; k <= n_img && (per || i + k < n); ++k)
        if (m[(long)((i + k) % n) * es]) { dr = k; break; }
    if (dl > n_img && dr > n_img) return 0;
    return dl <= dr ? 2 : 3;
}

// One thread per (mask level, y, x); writes the codes of both directions
// (rows periodic when periodic_x).
__global__ void k_seg(const uint8_t *__restrict__ mask, uint8_t *__restrict__ code_x,
                      uint8_t *__restrict__ code_y, int nx, int ny, int nl, int n_img, int periodic_x)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long plane = (long)nx * ny;
    if (t >= plane * nl) return;
    const int lev = (int)(t / plane);
    const long r = t % plane;
    const int y = (int)(r / nx), x = (int)(r % nx);
    const uint8_t *mp = mask + lev * plane;
    for (int d = 0; d < 2; ++d) {
        const int n = d == 0 ? nx : ny;
        const int i = d == 0 ? x : y;
        const long es = d == 0 ? 1 : nx;
        const bool per = d == 0 && periodic_x;
        const uint8_t *line = d == 0 ? mp + (long)y * nx : mp + x;
        const int k = classify(line, es, n, i, n_img, per);
        const bool first = !per && i == 0, last = !per && i == n - 1;
        const int kp = first ? 0 : classify(line, es, n, (i - 1 + n) % n, n_img, per);
        const int kn = last ? 0 : classify(line, es, n, (i + 1) % n, n_img, per);
        uint8_t c = 0;
        if (k == 1) c |= CODE_SEA;
        if (k != 0) {
            c |= CODE_ACTIVE;
            // a new segment starts where the previous point is outside every
            // segment or is an imaginary point of the run before a gap whose
            // other side (this point) belongs to the next run (on a periodic
            // row with no land there is neither a start nor an end)
            const bool start = first || kp == 0 || (kp == 2 && (k == 3 || k == 1));
            const bool end = last || kn == 0 || (k == 2 && (kn == 3 || kn == 1));
            if (start) c |= CODE_FRESET;
            if (end) c |= CODE_BRESET;
        } else {
            c |= CODE_FRESET | CODE_BRESET;
        }
        (d == 0 ? code_x : code_y)[t] = c;
    }
}

// alpha_{., k} of the point `off` steps away along the line, 0 outside the line
// or where sigma is not usable (such points never reach a used state term); on
// a periodic line the point is taken around the cycle.
__device__ inline double alpha_at(const double *sig, long es, int n, int i, int off, int k, int mode, bool per)
{
    int j = i + off;
    if (per) j = ((j % n) + n) % n;
    if (j < 0 || j >= n) return 0.0;
    const double s = sig[(long)j * es];
    if (!sigma_ok(s)) return 0.0;
    const Coef3 c = coef3(mode, s);
    return k == 1 ? c.al1 : (k == 2 ? c.al2 : c.al3);
}

// One thread per (sigma level, y, x): coefficient tables of both directions.
__global__ void k_coef(const double *__restrict__ sx, const double *__restrict__ sy,
                       const uint8_t *__restrict__ code_x, const uint8_t *__restrict__ code_y,
                       char *__restrict__ blk, BlockHeader h)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = h.g.nx, ny = h.g.ny;
    const long plane = (long)nx * ny;
    if (t >= (long)h.npts_c) return;
    const int lev = (int)(t / plane);
    const long r = t % plane;
    const int y = (int)(r / nx), x = (int)(r % nx);
    const int mode = h.g.qmode;
    for (int d = 0; d < 2; ++d) {
        const double *sig = (d == 0 ? sx : sy) + lev * plane;
        const uint8_t *code = d == 0 ? code_x : code_y;
        const double s = sig[r];
        // is the point inside a segment on some level that uses this sigma plane?
        bool used = false;
        if (h.g.mask_nlev == h.g.sigma_nlev) {
            used = code[t] & CODE_ACTIVE;
        } else if (h.g.mask_nlev == 1) {
            used = code[r] & CODE_ACTIVE;
        } else {
            for (int l = 0; l < h.g.mask_nlev && !used; ++l) used = code[l * plane + r] & CODE_ACTIVE;
        }
        float4 f = make_float4(0.f, 0.f, 0.f, 0.f), a = f, b = f;
        double4 f64 = make_double4(0.0, 0.0, 0.0, 0.0);
        double2 r1 = make_double2(0.0, 0.0);
        if (sigma_ok(s)) {
            const Coef3 c = coef3(mode, s);
            f = make_float4((float)c.beta_g, (float)c.gam, (float)c.c2, (float)c.c3);
            f64 = make_double4(c.beta, c.al1, c.al2, c.al3);
            // adjoint: source-indexed alphas of the neighbours along the line
            const int n = d == 0 ? nx : ny, i = d == 0 ? x : y;
            const long es = d == 0 ? 1 : nx;
            const double *line = d == 0 ? sig + (long)y * nx : sig + x;
            const bool per = d == 0 && (h.g.flags & RF_PERIODIC_X);
            const double A1 = alpha_at(line, es, n, i, -1, 1, mode, per);
            const double A2 = alpha_at(line, es, n, i, -2, 2, mode, per);
            const double A3 = alpha_at(line, es, n, i, -3, 3, mode, per);
            a = make_float4((float)c.beta_g, (float)(1.0 - A1 - A2 - A3), (float)(A2 + A3), (float)A3);
            const double D1 = alpha_at(line, es, n, i, 1, 1, mode, per);
            const double D2 = alpha_at(line, es, n, i, 2, 2, mode, per);
            const double D3 = alpha_at(line, es, n, i, 3, 3, mode, per);
            b = make_float4((float)c.beta_g, (float)(1.0 - D1 - D2 - D3), (float)(D2 + D3), (float)D3);
            const double E = (double)h.g.k1 / (s * s);
            const double rt = sqrt(E * (E + 2.0));
            r1 = make_double2(1.0 + E - rt, -E + rt);
        } else if (used) {
            atomicAdd(&reinterpret_cast<BlockHeader *>(blk)->sigma_error, 1);
        }
        reinterpret_cast<float4 *>(blk + h.off_f32[d])[t] = f;
        reinterpret_cast<float4 *>(blk + h.off_a32[d])[t] = a;
        reinterpret_cast<float4 *>(blk + h.off_d32[d])[t] = b;
        reinterpret_cast<double4 *>(blk + h.off_f64[d])[t] = f64;
        reinterpret_cast<double2 *>(blk + h.off_r1[d])[t] = r1;
    }
}

// Lane masks of the x kernel: one thread per (mask level, row, step i); bit c
// describes point c*lx + i (points past the row end are outside every segment).
__global__ void k_lanemask_x(const uint8_t *__restrict__ code, uint64_t *__restrict__ lm, int nx, int ny,
                             int nl, int lx)
{
    const int lxp = lmx_stride(lx);
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nl * ny * lxp) return;
    const int i = (int)(t % lxp);
    const long lrow = t / lxp;               // level * ny + row
    const uint8_t *c = code + lrow * nx;
    uint64_t f = ~0ull, b = ~0ull, s = 0, en = 0;   // s collects SEA; the table stores its complement
    if (i < lx) {
        f = b = 0;
        for (int ch = 0; ch < 64; ++ch) {
            const int x = ch * lx + i;
            const uint8_t v = x < nx ? c[x] : (uint8_t)(CODE_FRESET | CODE_BRESET);
            f |= (uint64_t)((v & CODE_FRESET) != 0) << ch;
            b |= (uint64_t)((v & CODE_BRESET) != 0) << ch;
            s |= (uint64_t)((v & CODE_SEA) != 0) << ch;
            en |= (uint64_t)((v & CODE_ACTIVE) && (v & CODE_BRESET)) << ch;
        }
    }
    uint64_t *o = lm + lrow * kLaneMasks * lxp + i;
    o[0] = f;
    o[lxp] = b;
    o[2 * lxp] = ~s;
    o[3 * lxp] = en;
}

// Lane masks of the y kernel: one thread per (mask level, column block, entry e
// < lys); entry e describes row e-8 and bit j column 64*blk + j; rows and
// columns outside the grid (and the guard entries) are outside every segment.
__global__ void k_lanemask_y(const uint8_t *__restrict__ code, uint64_t *__restrict__ lm, int nx, int ny,
                             int nl, int ly)
{
    const int nblk = (nx + kYCols - 1) / kYCols, lys = lmy_stride(ly);
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nl * nblk * lys) return;
    const int e = (int)(t % lys), r = e - 8;
    const long lb = t / lys;                  // level * nblk + blk
    const int blk = (int)(lb % nblk), lev = (int)(lb / nblk);
    uint64_t f = 0, b = 0, s = 0, en = 0;
    for (int j = 0; j < kYCols; ++j) {
        const int x = blk * kYCols + j;
        const uint8_t v = (x < nx && r >= 0 && r < ny) ? code[((long)lev * ny + r) * nx + x]
                                                       : (uint8_t)(CODE_FRESET | CODE_BRESET);
        f |= (uint64_t)((v & CODE_FRESET) != 0) << j;
        b |= (uint64_t)((v & CODE_BRESET) != 0) << j;
        s |= (uint64_t)((v & CODE_SEA) != 0) << j;
        en |= (uint64_t)((v & CODE_ACTIVE) && (v & CODE_BRESET)) << j;
    }
    uint64_t *o = lm + lb * kLaneMasks * lys + e;
    o[0] = f;
    o[lys] = b;
    o[2 * lys] = ~s;
    o[3 * lys] = en;
}

// ---- periodic rows: one-lap fixed points of the line-sequential kernels
__device__ inline void m3_mul(const double *A, const double *B, double *C)   // C = A B
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
// W = (I - Phi)^-1 by the adjugate (Phi: a stable lap, I - Phi well away from singular)
__device__ inline void m3_inv_i_minus(const double *Phi, double *W)
{
    double A[9];
    for (int e = 0; e < 9; ++e) A[e] = (e % 4 == 0 ? 1.0 : 0.0) - Phi[e];
    const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    W[0] = c00 / det; W[1] = (A[2] * A[7] - A[1] * A[8]) / det; W[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    W[3] = c01 / det; W[4] = (A[0] * A[8] - A[2] * A[6]) / det; W[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    W[6] = c02 / det; W[7] = (A[1] * A[6] - A[0] * A[7]) / det; W[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

// One thread per (sigma level, row).  For a periodic row with no land the
// sequential kernels run one lap from a zero state (ending in b), start the
// real lap from the fixed point W b, W = (I - Phi_lap)^-1.  Laps of the four
// sweeps (forward ascending/descending, adjoint ascending/descending), in the
// printed form (state: the last three values; step matrix rows
// (a1, a2, a3), (1, 0, 0), (0, 1, 0) with the adjoint's source-indexed alphas)
// and in the FP32 increment form (state (p, d1, d2), step matrix
// (1-g, -c2, -c3), (-g, -c2, -c3), (0, 1, 0) with the kernel's FP32 table),
// and the 1st-RF's scalar lap prod(alpha).
__global__ void k_perseq(const char *__restrict__ blk, double *__restrict__ out, BlockHeader h)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = h.g.nx, ny = h.g.ny;
    if (t >= (long)h.g.sigma_nlev * ny) return;
    const long base = t * nx;   // (level * ny + row) * nx
    const double4 *C = reinterpret_cast<const double4 *>(blk + h.off_f64[0]) + base;
    const float4 *T[3] = {reinterpret_cast<const float4 *>(blk + h.off_f32[0]) + base,
                          reinterpret_cast<const float4 *>(blk + h.off_a32[0]) + base,
                          reinterpret_cast<const float4 *>(blk + h.off_d32[0]) + base};
    const double2 *R1 = reinterpret_cast<const double2 *>(blk + h.off_r1[0]) + base;
    double *o = out + t * kPerSeq;
    auto wrap = [&](int i) { return ((i % nx) + nx) % nx; };
    for (int kind = 0; kind < 4; ++kind) {
        const bool desc = kind & 1;
        double Pd[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Pf[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, N[9];
        const float4 *Tk = T[kind == 0 || kind == 1 ? 0 : kind - 1];
        for (int s = 0; s < nx; ++s) {
            const int i = desc ? nx - 1 - s : s;
            double a1, a2, a3;
            if (kind < 2) { a1 = C[i].y; a2 = C[i].z; a3 = C[i].w; }
            else if (kind == 2) { a1 = C[wrap(i - 1)].y; a2 = C[wrap(i - 2)].z; a3 = C[wrap(i - 3)].w; }
            else { a1 = C[wrap(i + 1)].y; a2 = C[wrap(i + 2)].z; a3 = C[wrap(i + 3)].w; }
            const double Md[9] = {a1, a2, a3, 1, 0, 0, 0, 1, 0};
            m3_mul(Md, Pd, N);
            for (int e = 0; e < 9; ++e) Pd[e] = N[e];
            const float4 k = Tk[i];
            const double g = k.y, c2 = k.z, c3 = k.w;
            const double Mf[9] = {1 - g, -c2, -c3, -g, -c2, -c3, 0, 1, 0};
            m3_mul(Mf, Pf, N);
            for (int e = 0; e < 9; ++e) Pf[e] = N[e];
        }
        m3_inv_i_minus(Pd, o + 9 * kind);
        m3_inv_i_minus(Pf, o + kPerSeqDelta + 9 * kind);
    }
    double prod = 1.0;
    for (int i = 0; i < nx; ++i) prod *= R1[i].x;
    o[kPerSeqRf1] = o[kPerSeqRf1 + 1] = 1.0 / (1.0 - prod);
    o[kPerSeqRf1 + 2] = o[kPerSeqRf1 + 3] = 0.0;
}

// ---- exact end conditions: the 3x3 end matrices at every segment end
// Solve A x = b (n x n row-major, partial pivoting), b overwritten by x.
__device__ inline void solve_dense(int n, double *A, double *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) { const double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
            const double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r * n + c] / A[c * n + c];
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

// Past a segment end e the input is zero and e's coefficients continue, so the
// causal state x_j = (p_j, p_{j-1}, p_{j-2}) follows x_j = C x_{j-1} with the
// companion matrix C = ((a1, a2, a3), (1, 0, 0), (0, 1, 0)), and the anti-causal
// values past e are (o_{e+1}, o_{e+2}, o_{e+3}) = M (p_e, p_{e-1}, p_{e-2}) with
// M = beta X C, X = sum_m C^m e1 e1^T C^m, i.e. X = e1 e1^T + C X C (9x9 solve).
// Those values enter the anti-causal steps of e, e-1, e-2 through
// J = ((a1_e, a2_e, a3_e), (a2_{e-1}, a3_{e-1}, 0), (a3_{e-2}, 0, 0)): the
// forward anti-causal input at e - t gains (J M x)_t, and the adjoint adds
// (M^T J^T z)_t to the transposed pass's w = beta z at e - t.  Rows of points
// e-1, e-2 outside the segment are zero.
//
// For large sigma M has large entries that cancel on smooth data, so the FP32
// paths apply the maps to accurately computed states, not to three stored
// values: the causal state in increment form (p_e, p_e - p_{e-1}, p_{e-1} -
// p_{e-2}) = D x with D = ((1,0,0), (1,-1,0), (0,1,-1)) (forward: J M D^-1;
// line-sequential adjoint, whose first pass carries z in the same form:
// M^T J^T D^-1), and, in the tiled adjoint, the transposed pass's state at e,
// which is the costate of the anti-causal start state in increment form, mu =
// D^-T J^T z (M^T D^T).
// One thread per (end level, y, x), both directions: FP64 J M and M^T J^T (on
// the values themselves), FP32 [3][12]: J M D^-1, M^T D^T, M^T J^T D^-1.
__global__ void k_end(const char *__restrict__ blk, char *__restrict__ wblk, BlockHeader h)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = h.g.nx, ny = h.g.ny;
    const long plane = (long)nx * ny;
    if (t >= (long)h.end_nlev * plane) return;
    const int lev = (int)(t / plane);
    const long r = t % plane;
    const int y = (int)(r / nx), x = (int)(r % nx);
    const long mb = (h.g.mask_nlev > 1 ? lev : 0) * plane, cb = (h.g.sigma_nlev > 1 ? lev : 0) * plane;
    for (int d = 0; d < 2; ++d) {
        double *od = reinterpret_cast<double *>(wblk + h.off_endd[d]) + t * 18;
        float *of = reinterpret_cast<float *>(wblk + h.off_endf[d]) + t * 36;
        for (int q = 0; q < 18; ++q) od[q] = 0.0;
        for (int q = 0; q < 36; ++q) of[q] = 0.f;
        const uint8_t *code = reinterpret_cast<const uint8_t *>(blk + h.off_code[d]) + mb;
        const double4 *C4 = reinterpret_cast<const double4 *>(blk + h.off_f64[d]) + cb;
        const uint8_t ce = code[r];
        if (!(ce & CODE_ACTIVE) || !(ce & CODE_BRESET)) continue;
        const bool per = d == 0 && (h.g.flags & RF_PERIODIC_X);
        const int n = d == 0 ? nx : ny, i = d == 0 ? x : y;
        auto pt = [&](int k) -> long {   // point k steps before e along the line
            int j = i - k;
            if (per) j = ((j % n) + n) % n;
            return d == 0 ? (long)y * nx + j : (long)j * nx + x;
        };
        const bool in1 = !(ce & CODE_FRESET);
        const bool in2 = in1 && !(code[pt(1)] & CODE_FRESET);
        const double4 c0 = C4[r];
        const double4 c1 = in1 ? C4[pt(1)] : make_double4(1, 0, 0, 0);
        const double4 c2 = in2 ? C4[pt(2)] : make_double4(1, 0, 0, 0);
        const double Cm[9] = {c0.y, c0.z, c0.w, 1, 0, 0, 0, 1, 0};
        double A[81], X[9];
        for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v) {
                double *row = A + 9 * (3 * u + v);
                for (int w = 0; w < 9; ++w) row[w] = w == 3 * u + v ? 1.0 : 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) row[3 * k + l] -= Cm[3 * u + k] * Cm[3 * l + v];
                X[3 * u + v] = (u == 0 && v == 0) ? 1.0 : 0.0;
            }
        solve_dense(9, A, X);
        double M[9];
        for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v)
                M[3 * u + v] = c0.x * (X[3 * u] * Cm[v] + X[3 * u + 1] * Cm[3 + v] + X[3 * u + 2] * Cm[6 + v]);
        const double J[9] = {c0.y, c0.z, c0.w, in1 ? c1.z : 0.0, in1 ? c1.w : 0.0, 0.0, in2 ? c2.w : 0.0, 0.0, 0.0};
        const bool keep[3] = {true, in1, in2};
        // JM and (JM)^T; D^-1 = ((1,0,0), (1,-1,0), (1,-1,-1)), D^T = ((1,1,0), (0,-1,1), (0,0,-1))
        const double Di[9] = {1, 0, 0, 1, -1, 0, 1, -1, -1};
        const double Dt[9] = {1, 1, 0, 0, -1, 1, 0, 0, -1};
        double JM[9], JMt[9], Mt[9];
        for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v) {
                double f = 0.0;
                for (int k = 0; k < 3; ++k) f += J[3 * u + k] * M[3 * k + v];
                JM[3 * u + v] = f;
                Mt[3 * v + u] = M[3 * u + v];
            }
        for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v) JMt[3 * u + v] = JM[3 * v + u];
        auto mul = [](const double *P, const double *Q, double *R) {
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v) R[3 * u + v] = P[3 * u] * Q[v] + P[3 * u + 1] * Q[3 + v] + P[3 * u + 2] * Q[6 + v];
        };
        double F[9], Ta[9], Sa[9];
        mul(JM, Di, F);    // forward, on the causal increment state
        mul(Mt, Dt, Ta);   // tiled adjoint, on the transposed pass's state
        mul(JMt, Di, Sa);  // sequential adjoint, on z in increment form
        for (int u = 0; u < 3; ++u)
            for (int v = 0; v < 3; ++v) {
                const bool k = keep[u];
                const bool kk = keep[u] && keep[v];
                od[3 * u + v] = kk ? JM[3 * u + v] : 0.0;
                od[9 + 3 * u + v] = kk ? JMt[3 * u + v] : 0.0;
                of[3 * u + v] = k ? (float)F[3 * u + v] : 0.f;
                of[12 + 3 * u + v] = k ? (float)Ta[3 * u + v] : 0.f;
                of[24 + 3 * u + v] = k ? (float)Sa[3 * u + v] : 0.f;
            }
    }
}

bool grid_ok(const rf_grid *g)
{
    if (!g) return false;
    if (g->nx < 1 || g->ny < 1 || g->nx > 65535 || g->ny > 65535 || g->nlev < 1) return false;
    if (g->mask_nlev != 1 && g->mask_nlev != g->nlev) return false;
    if (g->sigma_nlev != 1 && g->sigma_nlev != g->nlev) return false;
    if (g->n_img < 0 || g->n_img > 64) return false;
    if (g->qmode < RF_Q_LITERAL || g->qmode > RF_Q_FIT) return false;
    if (g->k1 < 1) return false;
    if (g->flags & ~(RF_PERIODIC_X | RF_EXACT_ENDS)) return false;
    return true;
}

BlockHeader layout(const rf_grid *g)
{
    BlockHeader h{};
    h.magic = kMagic;
    h.version = kVersion;
    h.g = *g;
    const size_t plane = (size_t)g->nx * g->ny;
    h.npts_c = plane * g->sigma_nlev;
    h.npts_m = plane * g->mask_nlev;
    size_t off = kHeaderBytes;
    for (int d = 0; d < 2; ++d) {
        h.off_f32[d] = off; off = align256(off + 16 * h.npts_c);
        h.off_a32[d] = off; off = align256(off + 16 * h.npts_c);
        h.off_d32[d] = off; off = align256(off + 16 * h.npts_c);
        h.off_f64[d] = off; off = align256(off + 32 * h.npts_c);
        h.off_r1[d] = off;  off = align256(off + 16 * h.npts_c);
    }
    for (int d = 0; d < 2; ++d) { h.off_code[d] = off; off = align256(off + h.npts_m); }
    h.lx = tile_lx(g->nx);
    h.ly = tile_ly(g->ny);
    h.off_lmx = off;
    if (h.lx) off = align256(off + (size_t)g->mask_nlev * g->ny * lmx_stride(h.lx) * kLaneMasks * 8);
    h.off_lmy = off;
    if (h.ly) off = align256(off + (size_t)g->mask_nlev * ((g->nx + kYCols - 1) / kYCols) * lmy_stride(h.ly) * kLaneMasks * 8);
    const size_t clev = (size_t)coef_levels(g);
    h.off_phiy = off;
    if (h.ly) off = align256(off + clev * phiy_level_floats(g->nx) * 4);
    h.off_phix = off;
    if (h.lx) off = align256(off + clev * phix_level_floats(g->ny) * 4);
    h.off_ky = off;
    if (h.ly) off = align256(off + clev * ky_level_floats(g->nx, g->ny) * 4);
    h.off_perx = h.off_perseq = 0;
    if (g->flags & RF_PERIODIC_X) {
        if (h.lx) { h.off_perx = off; off = align256(off + clev * perx_level_floats(g->ny) * 4); }
        h.off_perseq = off;
        off = align256(off + (size_t)g->sigma_nlev * g->ny * kPerSeq * 8);
    }
    h.end_nlev = 0;
    for (int d = 0; d < 2; ++d) h.off_endd[d] = h.off_endf[d] = 0;
    if (g->flags & RF_EXACT_ENDS) {
        h.end_nlev = g->mask_nlev > g->sigma_nlev ? g->mask_nlev : g->sigma_nlev;
        for (int d = 0; d < 2; ++d) {
            h.off_endd[d] = off;
            off = align256(off + (size_t)h.end_nlev * plane * 2 * 9 * 8);
            h.off_endf[d] = off;
            off = align256(off + (size_t)h.end_nlev * plane * 3 * 12 * 4);
        }
    }
    h.total_bytes = off;
    return h;
}

}  // namespace rf

using namespace rf;

extern "C" size_t rf_coeffs_bytes(const rf_grid *g)
{
    if (!grid_ok(g)) return 0;
    return layout(g).total_bytes;
}

extern "C" int rf_coeffs(const rf_grid *g, const uint8_t *mask, const double *sigma_x,
                         const double *sigma_y, void *coef, void *stream)
{
    if (!g || !mask || !sigma_x || !sigma_y || !coef) return RF_E_ARG;
    if (!grid_ok(g)) return RF_E_SHAPE;
    if (reinterpret_cast<uintptr_t>(coef) % 256) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    BlockHeader h = layout(g);
    char *blk = reinterpret_cast<char *>(coef);
    if (hipMemcpyAsync(blk, &h, sizeof(h), hipMemcpyHostToDevice, st) != hipSuccess) return RF_E_HIP;
    const long nm = (long)h.npts_m, nc = (long)h.npts_c;
    k_seg<<<(unsigned)((nm + 255) / 256), 256, 0, st>>>(mask, (uint8_t *)(blk + h.off_code[0]),
                                                      (uint8_t *)(blk + h.off_code[1]), g->nx, g->ny,
                                                      g->mask_nlev, g->n_img, (g->flags & RF_PERIODIC_X) != 0);
    if (hipGetLastError() != hipSuccess) return RF_E_HIP;
    k_coef<<<(unsigned)((nc + 255) / 256), 256, 0, st>>>(sigma_x, sigma_y, (const uint8_t *)(blk + h.off_code[0]),
                                                       (const uint8_t *)(blk + h.off_code[1]), blk, h);
    if (hipGetLastError() != hipSuccess) return RF_E_HIP;
    if (h.lx) {
        const long n = (long)g->mask_nlev * g->ny * lmx_stride(h.lx);
        k_lanemask_x<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((const uint8_t *)(blk + h.off_code[0]),
                                                                (uint64_t *)(blk + h.off_lmx), g->nx, g->ny,
                                                                g->mask_nlev, h.lx);
        if (hipGetLastError() != hipSuccess) return RF_E_HIP;
    }
    if (h.ly) {
        const long n = (long)g->mask_nlev * ((g->nx + kYCols - 1) / kYCols) * lmy_stride(h.ly);
        k_lanemask_y<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((const uint8_t *)(blk + h.off_code[1]),
                                                                (uint64_t *)(blk + h.off_lmy), g->nx, g->ny,
                                                                g->mask_nlev, h.ly);
        if (hipGetLastError() != hipSuccess) return RF_E_HIP;
    }
    // scan tables per coefficient level, from that level's coefficients and codes
    const size_t plane = (size_t)g->nx * g->ny;
    for (int l = 0; l < coef_levels(g); ++l) {
        const size_t ls = g->sigma_nlev > 1 ? l * plane : 0, lm = g->mask_nlev > 1 ? l * plane : 0;
        if (h.lx && setup_phi_x((const float4 *)(blk + h.off_f32[0]) + ls, (const uint8_t *)(blk + h.off_code[0]) + lm,
                                (float *)(blk + h.off_phix) + l * phix_level_floats(g->ny), g->nx, g->ny, h.lx,
                                st) != hipSuccess)
            return RF_E_HIP;
        if (h.ly && setup_phi_y((const float4 *)(blk + h.off_f32[1]) + ls, (const uint8_t *)(blk + h.off_code[1]) + lm,
                                (float *)(blk + h.off_phiy) + l * phiy_level_floats(g->nx), g->nx, g->ny, h.ly,
                                st) != hipSuccess)
            return RF_E_HIP;
        if (h.ly && setup_ky_y((const float4 *)(blk + h.off_f32[1]) + ls, (const uint8_t *)(blk + h.off_code[1]) + lm,
                               (float *)(blk + h.off_ky) + l * ky_level_floats(g->nx, g->ny), g->nx, g->ny, h.ly,
                               st) != hipSuccess)
            return RF_E_HIP;
    }
    for (int l = 0; h.off_perx && l < coef_levels(g); ++l) {
        const size_t ls = g->sigma_nlev > 1 ? l * plane : 0, lm = g->mask_nlev > 1 ? l * plane : 0;
        if (setup_per_x((const float4 *)(blk + h.off_f32[0]) + ls, (const uint8_t *)(blk + h.off_code[0]) + lm,
                        (float *)(blk + h.off_perx) + l * perx_level_floats(g->ny), g->nx, g->ny, h.lx,
                        st) != hipSuccess)
            return RF_E_HIP;
    }
    if (h.end_nlev) {
        const long n = (long)h.end_nlev * g->nx * g->ny;
        k_end<<<(unsigned)((n + 63) / 64), 64, 0, st>>>(blk, blk, h);
        if (hipGetLastError() != hipSuccess) return RF_E_HIP;
    }
    if (h.off_perseq) {
        const long n = (long)g->sigma_nlev * g->ny;
        k_perseq<<<(unsigned)((n + 63) / 64), 64, 0, st>>>(blk, (double *)(blk + h.off_perseq), h);
        if (hipGetLastError() != hipSuccess) return RF_E_HIP;
    }
    int32_t err = 0;
    if (hipMemcpyAsync(&err, blk + offsetof(BlockHeader, sigma_error), sizeof(err), hipMemcpyDeviceToHost, st) != hipSuccess)
        return RF_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return RF_E_HIP;
    return err ? RF_E_SIGMA : RF_OK;
}
