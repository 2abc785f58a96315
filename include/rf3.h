/*
 * rf3.h -- C ABI of librf3, the MI355X (gfx950) implementation of the
 * recursive-filter horizontal covariance operator of Farina et al.,
 * "A Revised Scheme to Compute Horizontal Covariances in an Oceanographic
 * 3D-VAR Assimilation System" (arXiv:1404.5756).
 *
 * The library applies V_H = G_y G_x (Sec. 2.2) to temperature/salinity-like
 * fields on every vertical level, where G_x and G_y are one-dimensional
 * recursive filters along grid rows and grid columns:
 *   - the third-order filter (3rd-RF) of Theorem 3.1: a causal sweep
 *     (eq. "fort") followed by an anti-causal sweep (eq. "bact"), with the
 *     heuristic initial conditions of Sec. 3.1 (zero state before a line);
 *   - the first-order filter (1st-RF) of eqs. "proc1-1"/"proc1-2", K times,
 *     with the coefficients of the Hayden relation (eq. "crucial").
 * Filter coefficients vary per grid point with sigma = R/dx (Sec. 3.1).
 * Coasts: each sea run along a line is extended by up to n_img imaginary
 * sea points (Sec. 1 and Sec. 4 mention them; their definition is this
 * library's reading: a land point within n_img points of a run joins the
 * nearer run, ties to the lower index; imaginary points take zero input and
 * give zero output).
 *
 * Conventions (all entry points):
 *   - Every array argument is a DEVICE pointer.  The caller allocates and
 *     owns all memory; the library allocates nothing and keeps no state
 *     between calls.
 *   - Fields are contiguous [nfields][nlev][ny][nx] (x fastest), FP32 or FP64
 *     per rf_prec.  in == out is allowed; any other overlap of in and out is
 *     rejected with RF_E_ARG.
 *   - Field values at land and imaginary points are ignored (read as 0); the
 *     output is 0 there.  So the operator is P V_H P with P the sea mask.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call except
 *     rf_coeffs only enqueues work on it and returns: it does not
 *     synchronise and may be captured into a hipGraph.
 *   - Return value: RF_OK (0) or a negative rf_status.  When a host-side check
 *     fails nothing has been enqueued.
 */
#ifndef RF3_H
#define RF3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RF_OK = 0,
    RF_E_ARG = -1,          /* null pointer, bad enum, bad count, overlapping in/out */
    RF_E_SHAPE = -2,        /* grid sizes out of range or inconsistent with the coefficient block */
    RF_E_SIGMA = -3,        /* sigma <= 0, NaN or Inf at a sea or imaginary point */
    RF_E_HIP = -4,          /* a HIP runtime call failed */
    RF_E_UNSUPPORTED = -5   /* valid request the library does not handle */
} rf_status;

typedef enum { RF_FP32 = 0, RF_FP64 = 1 } rf_prec;

/* How q enters the Theorem 3.1 polynomials a_{i,k}(q).  beta always uses the
 * true sigma, (2 pi sigma^2)^(1/4) (1 - sum alpha), so each direction keeps
 * the DC gain sqrt(2 pi) sigma of Appendix A (eqs. "avanti3", "avanti4").
 *   LITERAL : q = sigma, exactly as printed in the Theorem.
 *   VARMATCH: q solves A q^2 + B q = sigma^2, where A q^2 + B q is the
 *             variance of the causal+anti-causal impulse response
 *             (A = 2((C1/C0)^2 - 2 C2/C0), B = 2 C1/C0 with C0, C1, C2 the
 *             constant terms 3.738128, 5.788982, 3.382473 of the Theorem).
 *   FIT     : q = sigma - 1.3460094 + 1.2463293/(sigma + 0.6031649), the
 *             least-squares fit of the q that minimises the mass-normalised
 *             distance of the impulse response to exp(-x^2/(2 sigma^2)). */
typedef enum { RF_Q_LITERAL = 0, RF_Q_VARMATCH = 1, RF_Q_FIT = 2 } rf_qmode;

/* Options beyond the paper's scheme (rf_grid.flags, a bitwise or; 0 = the paper):
 *   RF_PERIODIC_X: rows are zonally periodic (global grids; the paper treats
 *     finite lines).  Sea runs and imaginary points are found around each row
 *     (a run may wrap from x = nx-1 to x = 0; a land point at equal distance
 *     from two runs joins the run before it).  A row with no land is one
 *     cyclic line: its recurrences take their periodic solution, the fixed
 *     point of one lap (a 3x3 solve per line).  Columns are never periodic.
 *   RF_EXACT_ENDS: end conditions of the 3rd-RF at coasts and line ends
 *     (Sec. 6 names other boundary conditions at the coasts as further work).
 *     The anti-causal sweep of each segment starts from the three values the
 *     infinite-line filter carries back from past the segment end (input zero
 *     outside the segment, the last point's coefficients continued), a 3x3
 *     matrix of the last three causal values computed in FP64 at setup; each
 *     segment's operator is then the infinite-line filter restricted to it
 *     (for uniform sigma a Toeplitz matrix, equally damped at both ends).
 *     The zero start of the causal sweep is already exact.  The 1st-RF keeps
 *     the paper's zero ends. */
enum { RF_PERIODIC_X = 1, RF_EXACT_ENDS = 2 };

typedef struct {
    int32_t nx, ny, nlev;   /* one level is [ny][nx], x fastest; 1 <= nx, ny <= 65535, nlev >= 1 */
    int32_t mask_nlev;      /* 1 (one 2-D mask for every level) or nlev */
    int32_t sigma_nlev;     /* 1 (2-D sigma fields for every level) or nlev */
    int32_t n_img;          /* imaginary sea points per coast, 0 <= n_img <= 64 */
    int32_t qmode;          /* rf_qmode */
    int32_t k1;             /* iteration count K the 1st-RF coefficients are built for (E = K/sigma^2), >= 1 */
    int32_t flags;          /* RF_PERIODIC_X | RF_EXACT_ENDS, or 0 */
} rf_grid;

/* Size in bytes of the coefficient block rf_coeffs fills for grid g (0 if g is
 * invalid).  The block holds per-point FP32 and FP64 filter coefficients for
 * both directions, forward and adjoint forms, the 1st-RF coefficients, and the
 * per-point coast codes; it is read by every apply call and never written by
 * them.  Caller-allocated, 256-byte aligned, any device memory. */
size_t rf_coeffs_bytes(const rf_grid *g);

/* Build the coefficient block (setup; run once per grid, mask and sigma).
 *   mask    : uint8 [mask_nlev][ny][nx], nonzero = sea.
 *   sigma_x : double [sigma_nlev][ny][nx], R/dx in grid units (x direction).
 *   sigma_y : double [sigma_nlev][ny][nx], R/dy in grid units (y direction).
 *   coef    : rf_coeffs_bytes(g) bytes, written.
 * Computes the coast segments of every row and column and, in FP64 on the
 * device, q(sigma), a_{i,0..3}, alpha_{i,k} = a_{i,k}/a_{i,0} and beta_i of
 * Theorem 3.1 and the 1st-RF alpha_i, beta_i of Sec. 3.1.  sigma must be
 * positive and finite at every sea and imaginary point (values at other land
 * points are not read).  This call synchronises `stream` and returns
 * RF_E_SIGMA if that check fails. */
int rf_coeffs(const rf_grid *g, const uint8_t *mask, const double *sigma_x,
              const double *sigma_y, void *coef, void *stream);

/* out = G_y G_x in (the 3rd-RF, Theorem 3.1), for each of nfields fields and
 * each of the first nlev levels (1 <= nlev <= g->nlev).  FP64 follows the
 * printed recurrence.  FP32 runs an algebraically identical form of it whose
 * state is the last value and the last two increments, with coefficients
 * gamma = 1 - sum_k alpha_k, alpha_2 + alpha_3 and alpha_3 formed in FP64. */
int rf3_apply_xy(const rf_grid *g, const void *coef, rf_prec prec, const void *in,
                 void *out, int32_t nlev, int32_t nfields, void *stream);

/* out = G_x^T G_y^T in, the exact transpose of rf3_apply_xy (needed for
 * B = V V^T, Sec. 2.1).  With varying sigma this is a different operator from
 * rf3_apply_xy. */
int rf3_adjoint_xy(const rf_grid *g, const void *coef, rf_prec prec, const void *in,
                   void *out, int32_t nlev, int32_t nfields, void *stream);

/* One direction of the 3rd-RF: out = G_x in (dir = 0, every row) or
 * out = G_y in (dir = 1, every column); adjoint = 1 applies the transpose of
 * that direction instead.  rf3_apply_xy is rf3_apply_dir(x) followed by
 * rf3_apply_dir(y) in place on out; rf3_adjoint_xy runs y^T then x^T.  Same
 * conventions as rf3_apply_xy. */
int rf3_apply_dir(const rf_grid *g, const void *coef, rf_prec prec, int32_t dir, int32_t adjoint,
                  const void *in, void *out, int32_t nlev, int32_t nfields, void *stream);

/* out = G_y^(K) G_x^(K) in with the 1st-RF: K causal+anti-causal iterations
 * along x (eqs. "proc1-1", "proc1-2"), then K along y.  K must equal g->k1
 * (the coefficients depend on K).  Only RF_FP64 is provided: this is the
 * paper's baseline filter. */
int rf1_apply_xy(const rf_grid *g, const void *coef, rf_prec prec, int32_t K,
                 const void *in, void *out, int32_t nlev, int32_t nfields, void *stream);

/* The same operator as rf1_apply_xy, fused: all K iterations along x in one
 * kernel and all K along y in a second, each line kept on chip between
 * iterations (the field crosses HBM once per direction, not once per
 * iteration; the sweeps of a line are chunked and joined by scans).  FP32 or
 * FP64.  Results equal rf1_apply_xy up to rounding.  This is the fast 1st-RF
 * the 3rd-RF is compared with (the paper compares with its 1st-RF at K = 1, 5,
 * 10, Sec. 4.1, 5.1).  RF_E_UNSUPPORTED for grids whose mask or sigma vary
 * with level, periodic rows, or rows/columns longer than the tiled kernels
 * take (nx > 2112, ny > 1024); rf1_apply_xy covers those. */
int rf1_apply_xy_fused(const rf_grid *g, const void *coef, rf_prec prec, int32_t K,
                       const void *in, void *out, int32_t nlev, int32_t nfields, void *stream);

/* Many independent fields on possibly different grids in one pass (T and S
 * on every level of several grids: the paper runs the levels of its global
 * configuration in parallel, Sec. 5.1).  Each item applies rf3_apply_xy
 * (adjoint = 0) or rf3_adjoint_xy (adjoint = 1) to its own nfields fields over
 * all g->nlev levels of its grid.
 *
 * The x rows and y column blocks of all items form one work list; it runs as
 * one y launch and at most four x launches (one per occupancy class of the x
 * tile sizes; one with rf_batch_tuning.x_one_launch) per direction, for any
 * number of items.  Items whose mask or sigma vary with
 * level (mask_nlev or sigma_nlev > 1), or with flags set, are not in the work list: they are
 * applied one by one, as rf3_apply_xy / rf3_adjoint_xy would.
 *
 * Two steps, so that the apply step can be captured into a hipGraph:
 *   1. rf3_batch_plan (host only, no HIP call) writes the work list into host
 *      memory `plan` of exactly rf3_batch_plan_bytes(items, n) bytes (0 when
 *      the items are invalid); the caller copies those bytes to device memory
 *      it owns, 256-byte aligned.  The plan records the items' device
 *      pointers: rebuild it when any item changes.
 *   2. rf3_apply_batch re-derives the same work list on the host (to know the
 *      launches), then enqueues them on `stream` reading `plan_dev`.  It
 *      neither allocates nor synchronises; `plan_bytes` must equal
 *      rf3_batch_plan_bytes(items, n).  Passing a plan built from other items
 *      is undefined.
 * RF_FP32 uses the batched kernels; RF_FP64 applies the items one by one
 * (plan_dev is then not read and may be NULL).  Items must not overlap each
 * other's buffers.  Errors: as for rf3_apply_xy, per item; RF_E_ARG for a
 * wrong plan size or alignment. */
typedef struct {
    const rf_grid *g;       /* host pointer to the item's grid */
    const void *coef;       /* device: its coefficient block */
    const void *in;         /* device: [nfields][g->nlev][ny][nx] */
    void *out;              /* device: same shape; may equal in */
    int32_t nfields;
} rf_batch_item;

size_t rf3_batch_plan_bytes(const rf_batch_item *items, int32_t n);
int rf3_batch_plan(const rf_batch_item *items, int32_t n, void *plan, size_t plan_bytes);
int rf3_apply_batch(const rf_batch_item *items, int32_t n, rf_prec prec, int32_t adjoint,
                    const void *plan_dev, size_t plan_bytes, void *stream);

/* Work-list shape of a batch.  A zero field selects its default; the calls
 * above use the defaults.  The best shape depends on the items (their sizes
 * and level counts), so the Python binding's Batch.autotune times candidate
 * shapes on the actual items and keeps the fastest.  Results do not depend on
 * the shape (bitwise).  Out-of-range values give 0 / RF_E_ARG.  The _ex calls
 * behave as the plain ones; rf3_apply_batch_ex must get the tuning the plan
 * was built with (a different one is undefined, like other items). */
typedef struct {
    int32_t x_groups_max;   /* max workgroups sharing the planes of one x row, 1..64 (a power of two
                               is used: the largest not above it); default 8 */
    int32_t y_planes;       /* planes per y work unit (one workgroup), 1..4096; default 8 */
    int32_t x_one_launch;   /* 0 (default): one x launch per occupancy class of the x tile sizes;
                               1: all x units in one launch, sized (registers, LDS) for the largest
                               class present */
} rf_batch_tuning;

size_t rf3_batch_plan_bytes_ex(const rf_batch_item *items, int32_t n, const rf_batch_tuning *t);
int rf3_batch_plan_ex(const rf_batch_item *items, int32_t n, const rf_batch_tuning *t, void *plan,
                      size_t plan_bytes);
int rf3_apply_batch_ex(const rf_batch_item *items, int32_t n, const rf_batch_tuning *t, rf_prec prec,
                       int32_t adjoint, const void *plan_dev, size_t plan_bytes, void *stream);

/* 3D-VAR harness: bilinear observation operator H and its adjoint H^T.
 * The minimiser of Sec. 2 needs V and V^T (above) and the observation
 * operator with its transpose in every iteration.  Observation o is at level
 * lev[o] (0 <= lev < g->nlev) and position (x[o], y[o]) in grid units
 * (0 <= x <= nx-1, 0 <= y <= ny-1); it reads the 4 surrounding points of one
 * level with bilinear weights.  The field is one [g->nlev][ny][nx] stack.
 *
 *   rf_obs_plan_bytes / rf_obs_plan: host only (no HIP call).  Build the
 *     gather tables into host memory `plan` of exactly the returned size (0 on
 *     error: invalid grid, nobs < 1, a position outside the grid); *nuniq_out
 *     receives the number of distinct grid points touched.  The caller copies
 *     the plan to device memory it owns (256-byte aligned).
 *   rf_obs_apply:   obs[o] = sum_c w[o][c] field[p[o][c]]  (H field)
 *   rf_obs_adjoint: field = H^T obs, every point written (0 where no
 *     observation reads it).  Deterministic: each point sums its entries in
 *     observation order, without atomics.
 * nobs, nuniq and npts = nx*ny*nlev must be the plan's; otherwise the kernels
 * read nothing past the plan header and set every output to NaN (the plan
 * lives in device memory, so the mismatch is detected on the device and shows
 * in the results, not in the return code).  Asynchronous on
 * `stream`, no allocation; obs and field are device arrays of `prec`. */
size_t rf_obs_plan_bytes(const rf_grid *g, int32_t nobs, const int32_t *lev, const double *x, const double *y,
                         int32_t *nuniq_out);
int rf_obs_plan(const rf_grid *g, int32_t nobs, const int32_t *lev, const double *x, const double *y, void *plan,
                size_t plan_bytes);
int rf_obs_apply(const void *plan_dev, int32_t nobs, int32_t nuniq, int64_t npts, rf_prec prec, const void *field,
                 void *obs, void *stream);
int rf_obs_adjoint(const void *plan_dev, int32_t nobs, int32_t nuniq, int64_t npts, rf_prec prec, const void *obs,
                   void *field, void *stream);
/* Weighted innovation of the cost of Sec. 2.1 (eq. `functional2`), in
 * observation space, with R = diag(1 / rinv):
 *   d = H field - yobs,   rd = scale * rinv o d
 * field or yobs may be NULL (that term is 0); rinv may be NULL (weight 1);
 * d may be NULL (not stored).  rd = R^-1 (H V v - y) for the cost and its
 * gradient; R^-1 H V p inside CG (yobs NULL); R^-1 y for CG's first residual
 * (field NULL, scale -1).  Same plan and size rules as rf_obs_apply; vectors
 * are device arrays of nobs values of `prec`. */
int rf_obs_innovation(const void *plan_dev, int32_t nobs, int32_t nuniq, int64_t npts, rf_prec prec,
                      const void *field, const void *yobs, const void *rinv, double scale, void *d, void *rd,
                      void *stream);

/* 3D-VAR harness: vector steps of conjugate gradients (Sec. 2.1 solves its
 * preconditioned system by CG).  The iteration's scalars live in device
 * memory `s` (double[RF_CG_SLOTS], caller-owned), so an iteration is a chain
 * of launches without host round trips.  Dot products accumulate in FP64 and
 * are deterministic: a fixed grid of blocks writes partial sums into `work`
 * (caller-owned, device, rf_cg_work_bytes() bytes), then one block adds them
 * in a fixed order.  Vectors are n elements of `prec`, device memory.
 *   rf_dot:      s[slot] = a.b
 *   rf_cg_q_dot: q = p + w;  s[RF_CG_PQ] = p.q  (q may be NULL: not stored)
 *   rf_cg_step:  a = s[RF_CG_RR] / s[RF_CG_PQ] (0 if s[RF_CG_PQ] <= 0);
 *                v += a p;  r -= a q;  s[RF_CG_RR_NEW] = r.r
 *   rf_cg_step_pw: the same with q = p + w formed on the fly (A p = p + w for
 *                the system of Sec. 2.1, so q need not be stored)
 *   rf_cg_dir:   p = r + (s[RF_CG_RR_NEW] / s[RF_CG_RR]) p;  s[RF_CG_RR] = s[RF_CG_RR_NEW]
 *   rf_axpy:     y += a x  (the gradient v + V^T H^T rd, the Hessian product p + w)
 * Asynchronous on `stream`; no allocation.  RF_E_ARG on null pointers,
 * n < 1, a bad precision or slot. */
enum { RF_CG_RR = 0, RF_CG_PQ = 1, RF_CG_RR_NEW = 2, RF_CG_SLOTS = 8 };
size_t rf_cg_work_bytes(void);
int rf_dot(rf_prec prec, int64_t n, const void *a, const void *b, void *work, double *s, int32_t slot,
           void *stream);
int rf_cg_q_dot(rf_prec prec, int64_t n, const void *p, const void *w, void *q, void *work, double *s,
                void *stream);

/* rf_dot without the `work` argument, for callers that cannot allocate device
 * memory (code under hipGraph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same result, bit for bit, as rf_dot.  The partial sums go
 * to a fixed scratch array inside the library, rf_dot_noalloc_scratch_bytes()
 * bytes (8 KiB: one FP64 partial per block of the fixed 1024-block reduction
 * grid, whatever n), which each GPU the library runs on holds until the process
 * ends.  Its device address is looked up on the first call on a device (with
 * that device current).  The call allocates nothing.  All calls on one GPU share
 * that GPU's scratch: calls that overlap in time on one GPU (different streams
 * without ordering) race and give wrong sums; calls ordered on a stream do not.
 * The scratch needs no clearing (every partial is written before it is read).
 * Errors: as rf_dot; RF_E_HIP if the scratch address cannot be obtained. */
size_t rf_dot_noalloc_scratch_bytes(void);
int rf_dot_noalloc(rf_prec prec, int64_t n, const void *a, const void *b, double *s, int32_t slot,
                   void *stream);
int rf_cg_step(rf_prec prec, int64_t n, const void *p, const void *q, void *v, void *r, void *work, double *s,
               void *stream);
int rf_cg_step_pw(rf_prec prec, int64_t n, const void *p, const void *w, void *v, void *r, void *work, double *s,
                  void *stream);
int rf_cg_dir(rf_prec prec, int64_t n, const void *r, void *p, double *s, void *stream);
int rf_axpy(rf_prec prec, int64_t n, double a, const void *x, void *y, void *stream);

/* Static description of a status code. */
const char *rf_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* RF3_H */
