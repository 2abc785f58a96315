// Line-sequential sweep kernels: one lane runs one whole line.  They serve the
// FP64 path (printed recurrence, same order of operations as the paper), the
// 1st-RF baseline, and any FP32 shape the tiled kernels do not cover.
//
// The causal sweep writes its result into `out` and the anti-causal sweep
// reads it back in reverse, so one line is processed entirely by one lane.
#include "rf3_internal.h"
#include "sweeps.h"

namespace rf {

__device__ inline long line_base(const LineGeom &G, long t, int &pl)
{
    pl = (int)(t / G.nlines);
    const int ln = (int)(t % G.nlines);
    return (long)ln * G.lstride;
}

// Where the two laps over a line start.  A line runs ascending from i0 and
// descending from i1, n points each, wrapping around on a periodic row.  On
// ordinary lines i0 = 0 and i1 = n-1.  A periodic row starts each lap at a
// point where the state is reset (a segment start for the ascending lap, a
// segment end for the descending one), so the lap needs no incoming state; a
// periodic row with no land has no such point: W then points at its one-lap
// fixed points (the state to start from is W times the state one lap from
// zero leaves).
struct Laps {
    int i0, i1;
    const double *W;
};
__device__ inline Laps laps(const LineGeom &G, long t, int pl, const uint8_t *code, long mb)
{
    Laps L{0, G.n - 1, nullptr};
    if (!G.periodic) return L;
    int a = -1, b = -1;
    for (int i = 0; i < G.n && (a < 0 || b < 0); ++i) {
        const uint8_t c = code[mb + (long)i * G.estride];
        if (a < 0 && (c & CODE_FRESET)) a = i;
        if (b < 0 && (c & CODE_BRESET)) b = i;
    }
    if (a >= 0) {
        L.i0 = a;
        L.i1 = b;
    } else {
        const int lev = G.coef_per_lev ? pl % G.nlev : 0;
        L.W = G.per + ((long)lev * G.nlines + t % G.nlines) * kPerSeq;
    }
    return L;
}
__device__ inline int lap_index(int start, int step, int n, bool desc)
{
    int i = desc ? start - step : start + step;
    return i < 0 ? i + n : (i >= n ? i - n : i);
}
// Exact ends, FP64 (G.endd): the anti-causal input at a segment end e and at
// e-1, e-2 gains N (v_e, v_{e-1}, v_{e-2}), N the point's 3x3 end matrix
// (forward: J M on the causal values p; adjoint: M^T J^T on the transposed
// pass's z), v the values the causal lap left in `out`.  The corrections of e-1
// and e-2 wait in pend1/pend2 for the next two descending steps.  (The FP32
// kernel applies the same corrections in its ascending lap, from the state in
// increment form, which large sigma needs: M's entries cancel on smooth data.)
struct EndCorr {
    double pend1 = 0.0, pend2 = 0.0;
    template <class F>
    __device__ inline double step(const LineGeom &G, long eb, int i, uint8_t c, const F *vals, long fb,
                                  bool adj)
    {
        double add = pend1;
        pend1 = pend2;
        pend2 = 0.0;
        if ((c & CODE_ACTIVE) && (c & CODE_BRESET)) {
            const double *N = G.endd + (eb + (long)i * G.estride) * 18 + (adj ? 9 : 0);
            double x[3];
            for (int k = 0; k < 3; ++k) {
                int j = i - k;
                if (G.periodic) j = j < 0 ? j + G.n : j;
                x[k] = j >= 0 ? (double)vals[fb + (long)j * G.estride] : 0.0;
            }
            add += N[0] * x[0] + N[1] * x[1] + N[2] * x[2];
            pend1 += N[3] * x[0] + N[4] * x[1] + N[5] * x[2];
            pend2 += N[6] * x[0] + N[7] * x[1] + N[8] * x[2];
        }
        return add;
    }
};

// (a, b, c) <- W (a, b, c), W row-major 3x3
template <class F>
__device__ inline void apply_w(const double *W, F &a, F &b, F &c)
{
    const F x = a, y = b, z = c;
    a = (F)(W[0] * x + W[1] * y + W[2] * z);
    b = (F)(W[3] * x + W[4] * y + W[5] * z);
    c = (F)(W[6] * x + W[7] * y + W[8] * z);
}

// ---------------------------------------------------------------- FP32
// Third-order recurrence of eqs. "fort"/"bact" written on the state
// (p_{i-1}, d1 = p_{i-1}-p_{i-2}, d2 = p_{i-2}-p_{i-3}):
//   t_i = g_i s_i - gamma_i p_{i-1} - c2_i d1 - c3_i d2,  p_i = p_{i-1} + t_i,
// which equals p_i = beta_i s_i + sum_k alpha_{i,k} p_{i-k} exactly in real
// arithmetic (gamma = 1 - sum alpha, c2 = alpha2 + alpha3, c3 = alpha3) and
// keeps the small increment t_i as state, so FP32 rounding of p does not feed
// back through the near-unit-root recursion.
template <bool ADJ>
__global__ void k_rf3_seq_f32(const float *in, float *out, const float4 *__restrict__ T1,
                              const float4 *__restrict__ T2, const uint8_t *__restrict__ code,
                              LineGeom G)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)G.nplanes * G.nlines) return;
    int pl;
    const long lb = line_base(G, t, pl);
    const long fb = (long)pl * G.plane + lb;
    const long cb = plane_offset(G, pl, G.coef_per_lev) + lb;
    const long mb = plane_offset(G, pl, G.mask_per_lev) + lb;
    const Laps lp = laps(G, t, pl, code, mb);
    const long eb = plane_offset(G, pl, G.end_per_lev) + lb;
    float p1 = 0.f, d1 = 0.f, d2 = 0.f;
    auto asc = [&](int i, bool store) {
        const long e = (long)i * G.estride;
        const uint8_t c = code[mb + e];
        if (c & CODE_FRESET) { p1 = 0.f; d1 = 0.f; d2 = 0.f; }
        const float4 k = T1[cb + e];
        const float s = (c & CODE_SEA) ? in[fb + e] : 0.f;
        const float g = ADJ ? 1.f : k.x;
        const float tt = fmaf(-k.w, d2, fmaf(-k.z, d1, fmaf(-k.y, p1, g * s)));
        const float p = p1 + tt;
        d2 = d1; d1 = tt; p1 = p;
        if (!store) return;
        out[fb + e] = p;
        if (G.endf && (c & CODE_ACTIVE) && (c & CODE_BRESET)) {
            // exact end: the anti-causal input beta v at e - q gains N (p, d1, d2), the
            // state in increment form; stored as v += N(...) / beta
            const float *N = G.endf + (eb + e) * 36 + (ADJ ? 24 : 0);
            for (int q = 0; q < 3; ++q) {
                const float cq = fmaf(N[3 * q], p1, fmaf(N[3 * q + 1], d1, N[3 * q + 2] * d2));
                if (cq == 0.f) continue;
                int j = i - q;
                if (j < 0) {
                    if (!G.periodic) continue;
                    j += G.n;
                }
                const long ej = (long)j * G.estride;
                out[fb + ej] += cq / T1[cb + ej].x;
            }
        }
    };
    if (lp.W) {
        for (int i = 0; i < G.n; ++i) asc(i, false);
        apply_w(lp.W + kPerSeqDelta + 9 * (ADJ ? 2 : 0), p1, d1, d2);
    }
    for (int s = 0; s < G.n; ++s) asc(lap_index(lp.i0, s, G.n, false), true);
    p1 = 0.f; d1 = 0.f; d2 = 0.f;
    auto desc = [&](int i, bool store) {
        const long e = (long)i * G.estride;
        const uint8_t c = code[mb + e];
        if (c & CODE_BRESET) { p1 = 0.f; d1 = 0.f; d2 = 0.f; }
        const float4 k = T2[cb + e];
        const float v = out[fb + e];
        const float tt = fmaf(-k.w, d2, fmaf(-k.z, d1, fmaf(-k.y, p1, k.x * v)));
        const float p = p1 + tt;
        d2 = d1; d1 = tt; p1 = p;
        if (store) out[fb + e] = (c & CODE_SEA) ? (ADJ ? k.x * p : p) : 0.f;
    };
    if (lp.W) {
        for (int i = G.n - 1; i >= 0; --i) desc(i, false);
        apply_w(lp.W + kPerSeqDelta + 9 * (ADJ ? 3 : 1), p1, d1, d2);
    }
    for (int s = 0; s < G.n; ++s) desc(lap_index(lp.i1, s, G.n, true), true);
}

// ---------------------------------------------------------------- FP64
// Printed form: p_i = beta_i s_i + alpha_{i,1} p_{i-1} + alpha_{i,2} p_{i-2} + alpha_{i,3} p_{i-3}
// (eq. "fort"), o_i = beta_i p_i + sum_k alpha_{i,k} o_{i+k} (eq. "bact").
__global__ void k_rf3_seq_f64(const double *in, double *out, const double4 *__restrict__ C,
                              const uint8_t *__restrict__ code, LineGeom G)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)G.nplanes * G.nlines) return;
    int pl;
    const long lb = line_base(G, t, pl);
    const long fb = (long)pl * G.plane + lb;
    const long cb = plane_offset(G, pl, G.coef_per_lev) + lb;
    const long mb = plane_offset(G, pl, G.mask_per_lev) + lb;
    const Laps lp = laps(G, t, pl, code, mb);
    double p1 = 0, p2 = 0, p3 = 0;
    auto asc = [&](int i, bool store) {
        const long e = (long)i * G.estride;
        const uint8_t c = code[mb + e];
        if (c & CODE_FRESET) { p1 = 0; p2 = 0; p3 = 0; }
        const double4 k = C[cb + e];
        const double s = (c & CODE_SEA) ? in[fb + e] : 0.0;
        double v = k.x * s;
        v += k.y * p1;
        v += k.z * p2;
        v += k.w * p3;
        p3 = p2; p2 = p1; p1 = v;
        if (store) out[fb + e] = v;
    };
    if (lp.W) {
        for (int i = 0; i < G.n; ++i) asc(i, false);
        apply_w(lp.W, p1, p2, p3);
    }
    for (int s = 0; s < G.n; ++s) asc(lap_index(lp.i0, s, G.n, false), true);
    p1 = 0; p2 = 0; p3 = 0;
    EndCorr ec;
    const long eb = plane_offset(G, pl, G.end_per_lev) + lb;
    auto desc = [&](int i, bool store) {
        const long e = (long)i * G.estride;
        const uint8_t c = code[mb + e];
        if (c & CODE_BRESET) { p1 = 0; p2 = 0; p3 = 0; }
        const double4 k = C[cb + e];
        double v = k.x * out[fb + e];
        if (G.endd) v += ec.step(G, eb, i, c, out, fb, false);
        v += k.y * p1;
        v += k.z * p2;
        v += k.w * p3;
        p3 = p2; p2 = p1; p1 = v;
        if (store) out[fb + e] = (c & CODE_SEA) ? v : 0.0;
    };
    if (lp.W) {
        for (int i = G.n - 1; i >= 0; --i) desc(i, false);
        apply_w(lp.W + 9, p1, p2, p3);
    }
    for (int s = 0; s < G.n; ++s) desc(lap_index(lp.i1, s, G.n, true), true);
}

// Transpose of k_rf3_seq_f64 (G^T = D_beta L^-T D_beta U^-T):
//   z_j = y_j + alpha_{j-1,1} z_{j-1} + alpha_{j-2,2} z_{j-2} + alpha_{j-3,3} z_{j-3}
//   u_j = beta_j z_j + alpha_{j+1,1} u_{j+1} + alpha_{j+2,2} u_{j+2} + alpha_{j+3,3} u_{j+3}
//   out_j = beta_j u_j
__global__ void k_rf3_seq_f64_adj(const double *in, double *out, const double4 *__restrict__ C,
                                  const uint8_t *__restrict__ code, LineGeom G)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)G.nplanes * G.nlines) return;
    int pl;
    const long lb = line_base(G, t, pl);
    const long fb = (long)pl * G.plane + lb;
    const long cb = plane_offset(G, pl, G.coef_per_lev) + lb;
    const long mb = plane_offset(G, pl, G.mask_per_lev) + lb;
    const Laps lp = laps(G, t, pl, code, mb);
    const int n = G.n;
    auto coef = [&](int i) { return C[cb + (long)(((i % n) + n) % n) * G.estride]; };
    double z1 = 0, z2 = 0, z3 = 0;
    double4 k1 = make_double4(0, 0, 0, 0), k2 = k1, k3 = k1;   // coefficients of j-1, j-2, j-3
    auto asc = [&](int i, bool store) {
        const long e = (long)i * G.estride;
        const uint8_t c = code[mb + e];
        if (c & CODE_FRESET) { z1 = 0; z2 = 0; z3 = 0; }
        const double4 k = C[cb + e];
        double v = (c & CODE_SEA) ? in[fb + e] : 0.0;
        v += k1.y * z1;
        v += k2.z * z2;
        v += k3.w * z3;
        z3 = z2; z2 = z1; z1 = v;
        k3 = k2; k2 = k1; k1 = k;
        if (store) out[fb + e] = v;   // z; the descending lap takes beta z
    };
    if (lp.W) {   // a cycle: the points before j = 0 are n-1, n-2, n-3
        k1 = coef(-1); k2 = coef(-2); k3 = coef(-3);
        for (int i = 0; i < n; ++i) asc(i, false);
        apply_w(lp.W + 18, z1, z2, z3);
    }
    for (int s = 0; s < n; ++s) asc(lap_index(lp.i0, s, n, false), true);
    z1 = 0; z2 = 0; z3 = 0;
    k1 = make_double4(0, 0, 0, 0); k2 = k1; k3 = k1;              // coefficients of j+1, j+2, j+3
    EndCorr ec;
    const long eb = plane_offset(G, pl, G.end_per_lev) + lb;
    auto desc = [&](int i, bool store) {
        const long e = (long)i * G.estride;
        const uint8_t c = code[mb + e];
        if (c & CODE_BRESET) { z1 = 0; z2 = 0; z3 = 0; }
        const double4 k = C[cb + e];
        double v = k.x * out[fb + e];
        if (G.endd) v += ec.step(G, eb, i, c, out, fb, true);
        v += k1.y * z1;
        v += k2.z * z2;
        v += k3.w * z3;
        z3 = z2; z2 = z1; z1 = v;
        k3 = k2; k2 = k1; k1 = k;
        if (store) out[fb + e] = (c & CODE_SEA) ? k.x * v : 0.0;
    };
    if (lp.W) {   // the points after j = n-1 are 0, 1, 2
        k1 = coef(n); k2 = coef(n + 1); k3 = coef(n + 2);
        for (int i = n - 1; i >= 0; --i) desc(i, false);
        apply_w(lp.W + 27, z1, z2, z3);
    }
    for (int s = 0; s < n; ++s) desc(lap_index(lp.i1, s, n, true), true);
}

// ---------------------------------------------------------------- 1st-RF
// One iteration of eqs. "proc1-1"/"proc1-2" on every line: p_i = beta_i s_i +
// alpha_i p_{i-1} ascending, s_i = beta_i p_i + alpha_i s_{i+1} descending.
// FIRST masks the input to sea points; LAST zeroes non-sea outputs (values at
// imaginary points are carried from one iteration to the next).
template <bool FIRST, bool LAST>
__global__ void k_rf1_seq_f64(const double *in, double *out, const double2 *__restrict__ C,
                              const uint8_t *__restrict__ code, LineGeom G)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)G.nplanes * G.nlines) return;
    int pl;
    const long lb = line_base(G, t, pl);
    const long fb = (long)pl * G.plane + lb;
    const long cb = plane_offset(G, pl, G.coef_per_lev) + lb;
    const long mb = plane_offset(G, pl, G.mask_per_lev) + lb;
    const Laps lp = laps(G, t, pl, code, mb);
    double p = 0;
    auto asc = [&](int i, bool store) {
        const long e = (long)i * G.estride;
        const uint8_t c = code[mb + e];
        if (c & CODE_FRESET) p = 0;
        const double2 k = C[cb + e];
        double s = in[fb + e];
        if (FIRST && !(c & CODE_SEA)) s = 0.0;
        p = k.y * s + k.x * p;
        if (store) out[fb + e] = p;
    };
    if (lp.W) {
        for (int i = 0; i < G.n; ++i) asc(i, false);
        p *= lp.W[kPerSeqRf1];
    }
    for (int s = 0; s < G.n; ++s) asc(lap_index(lp.i0, s, G.n, false), true);
    p = 0;
    auto desc = [&](int i, bool store) {
        const long e = (long)i * G.estride;
        const uint8_t c = code[mb + e];
        if (c & CODE_BRESET) p = 0;
        const double2 k = C[cb + e];
        p = k.y * out[fb + e] + k.x * p;
        if (store) out[fb + e] = (LAST && !(c & CODE_SEA)) ? 0.0 : p;
    };
    if (lp.W) {
        for (int i = G.n - 1; i >= 0; --i) desc(i, false);
        p *= lp.W[kPerSeqRf1 + 1];
    }
    for (int s = 0; s < G.n; ++s) desc(lap_index(lp.i1, s, G.n, true), true);
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblocks(const LineGeom &G, int bs)
{
    return (unsigned)(((long)G.nplanes * G.nlines + bs - 1) / bs);
}

hipError_t seq_rf3_f32(const float *in, float *out, const float4 *T1, const float4 *T2,
                       const uint8_t *code, const LineGeom &G, bool adj, hipStream_t st)
{
    if (adj) k_rf3_seq_f32<true><<<nblocks(G, 256), 256, 0, st>>>(in, out, T1, T2, code, G);
    else k_rf3_seq_f32<false><<<nblocks(G, 256), 256, 0, st>>>(in, out, T1, T2, code, G);
    return hipGetLastError();
}

hipError_t seq_rf3_f64(const double *in, double *out, const double4 *C, const uint8_t *code,
                       const LineGeom &G, bool adj, hipStream_t st)
{
    if (adj) k_rf3_seq_f64_adj<<<nblocks(G, 256), 256, 0, st>>>(in, out, C, code, G);
    else k_rf3_seq_f64<<<nblocks(G, 256), 256, 0, st>>>(in, out, C, code, G);
    return hipGetLastError();
}

hipError_t seq_rf1_f64(const double *in, double *out, const double2 *C, const uint8_t *code,
                       const LineGeom &G, bool first, bool last, hipStream_t st)
{
    const unsigned nb = nblocks(G, 256);
    if (first && last) k_rf1_seq_f64<true, true><<<nb, 256, 0, st>>>(in, out, C, code, G);
    else if (first) k_rf1_seq_f64<true, false><<<nb, 256, 0, st>>>(in, out, C, code, G);
    else if (last) k_rf1_seq_f64<false, true><<<nb, 256, 0, st>>>(in, out, C, code, G);
    else k_rf1_seq_f64<false, false><<<nb, 256, 0, st>>>(in, out, C, code, G);
    return hipGetLastError();
}

}  // namespace rf
