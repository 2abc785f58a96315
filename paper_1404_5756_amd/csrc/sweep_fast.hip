// Tiled FP32 kernels of the 3rd-RF sweeps (forward and adjoint), gfx950.
//
// Both sweeps of eqs. "fort"/"bact" are linear recurrences in a 3-value state.
// A line is cut into chunks; each chunk first runs from a zero state (its
// local end state b), a scan over chunks composes the affine maps
// state_out = Phi state_in + b (Phi: the chunk's 3x3 transfer matrix), and each
// chunk then reruns from its true incoming state.  All data of a line stays in
// registers between the causal and the anti-causal sweep.
//
// Arithmetic (FP32).  Forward steps use the state (p, d1, d2) =
// (p_{i-1}, p_{i-1}-p_{i-2}, p_{i-2}-p_{i-3}):
//   t = beta_i s_i - gamma_i p - c2_i d1 - c3_i d2,  (p, d1, d2) <- (p + t, t, d1)
// which is the printed recurrence with gamma = 1 - sum alpha, c2 = alpha2 +
// alpha3, c3 = alpha3.  Adjoint sweeps run the transposed state-space system
// x_j = M_j x_{j-1} + v_j s_j  ->  lambda_j = e1 r_j + M_{j+1}^T lambda_{j+1},
// carried as nu = M_j^T lambda_j so that a step uses only its own point's
// coefficients:
//   w0 = r_j + nu0,  u = w0 + nu1,  output beta_j u,
//   nu <- (w0 - gamma_j u, nu2 - c2_j u, -c3_j u).
// A forward state is zeroed before a point where a segment starts (causal) or
// ends (anti-causal), an adjoint state after such a point (the paper's zero
// initial conditions at coasts and line ends).
#include "rf3_internal.h"
#include "sweeps.h"

namespace rf {

namespace {

// (lane bit of m set) ? 0 : x, m a wave-uniform 64-bit lane mask held in SGPRs
__device__ __forceinline__ float zero_if(float x, uint64_t m)
{
    float r;
    asm("v_cndmask_b32_e64 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(m));
    return r;
}

typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16 dwords from wave-uniform memory into SGPRs.  The wait is inside the same
// asm block, so the destination registers are complete when the block ends.
__device__ __forceinline__ u32x16 sload16(const void *p)
{
    u32x16 r;
    asm volatile("s_load_dwordx16 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p) : "memory");
    return r;
}

// compiler-only barrier for memory operations (keeps loads near their use)
__device__ __forceinline__ void mem_fence_compiler() { asm volatile("" ::: "memory"); }

// p unchanged, but opaque to the optimiser: addresses derived from it in
// different passes are not merged and kept live across the passes
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL T *fresh(T *p)
{
    GLOBAL T *q = (GLOBAL T *)p;
    asm volatile("" : "+s"(q));
    return q;
}
__device__ __forceinline__ int fresh_int(int v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// mask q of a block of eight 64-bit masks
__device__ __forceinline__ uint64_t m64_of(const u32x16 &r, int q) { return (uint64_t)r[2 * q] | ((uint64_t)r[2 * q + 1] << 32); }

struct St {
    float a, b, c;
};

__device__ __forceinline__ void st_reset(St &x, uint64_t m)
{
    x.a = zero_if(x.a, m);
    x.b = zero_if(x.b, m);
    x.c = zero_if(x.c, m);
}

// forward step, gs = beta_i * s_i
__device__ __forceinline__ void fwd_step(St &x, float gs, float gm, float c2, float c3)
{
    const float t = fmaf(-c3, x.c, fmaf(-c2, x.b, fmaf(-gm, x.a, gs)));
    x.c = x.b;
    x.b = t;
    x.a = x.a + t;
}

// transposed step at point j (own coefficients), r = input; returns the output
// beta_j * u before the reset of the state
__device__ __forceinline__ float adj_step(St &x, float r, float bt, float gm, float c2, float c3)
{
    const float w0 = x.a + r;
    const float u = w0 + x.b;
    x.a = fmaf(-gm, u, w0);
    x.b = fmaf(-c2, u, x.c);
    x.c = -c3 * u;
    float o = bt * u;
    asm volatile("" : "+v"(o));   // evaluate now: deferring it keeps u and beta live for many steps
    return o;
}

// y = A x + y with A 3x3 row-major
__device__ __forceinline__ void mat_acc(const float *A, const St &x, St &y)
{
    y.a = fmaf(A[0], x.a, fmaf(A[1], x.b, fmaf(A[2], x.c, y.a)));
    y.b = fmaf(A[3], x.a, fmaf(A[4], x.b, fmaf(A[5], x.c, y.b)));
    y.c = fmaf(A[6], x.a, fmaf(A[7], x.b, fmaf(A[8], x.c, y.c)));
}

__device__ __forceinline__ St st_shfl_up(const St &x, int d)
{
    return St{__shfl_up(x.a, d, 64), __shfl_up(x.b, d, 64), __shfl_up(x.c, d, 64)};
}
__device__ __forceinline__ St st_shfl_down(const St &x, int d)
{
    return St{__shfl_down(x.a, d, 64), __shfl_down(x.b, d, 64), __shfl_down(x.c, d, 64)};
}

}  // namespace

// ======================================================================
// x direction: one wave per line (row), lane c owns points [c*L, c*L + L).
// All waves of a workgroup work on the same row (different planes), so the
// row's coefficients, lane masks and scan matrices are shared.
// ======================================================================
constexpr int kXWaves = 4;

template <int L, bool ADJ>
struct XRow {
    static constexpr int LP = (L + 7) & ~7;   // mask array length (whole 8-blocks)
    float kb[L], kg[L], k2[L], k3[L];          // beta, gamma, c2, c3 of my chunk's points
    const uint64_t *lm;                        // this row's masks: [3][LP] FRESET, BRESET, not-SEA

    // ascending sweep over my chunk.  MODE 0: zero input (homogeneous),
    // 1: input v, no output, 2: input v, output written back into v.
    template <int MODE>
    __device__ __forceinline__ void asc(St &x, float *v) const
    {
        // forward: zero the state before a segment start; adjoint: after a segment end
        const uint64_t *rp = lm + (ADJ ? LP : 0);
#pragma unroll
        for (int b = 0; b < LP / 8; ++b) {
            const u32x16 m = sload16(rp + 8 * b);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i = 8 * b + q;
                if (i >= L) break;
                if (!ADJ) {
                    st_reset(x, m64_of(m, q));
                    fwd_step(x, MODE ? kb[i] * v[i] : 0.f, kg[i], k2[i], k3[i]);
                    if (MODE == 2) v[i] = x.a;
                } else {
                    const float o = adj_step(x, MODE ? v[i] : 0.f, kb[i], kg[i], k2[i], k3[i]);
                    st_reset(x, m64_of(m, q));
                    if (MODE == 2) v[i] = o;
                }
            }
        }
    }
    // descending sweep over my chunk; MODE 2 also applies the sea mask to the output
    template <int MODE>
    __device__ __forceinline__ void desc(St &x, float *v) const
    {
        // forward: zero the state before a segment end; adjoint: after a segment start
        const uint64_t *rp = lm + (ADJ ? 0 : LP);
#pragma unroll
        for (int b = LP / 8 - 1; b >= 0; --b) {
            const u32x16 m = sload16(rp + 8 * b);
            u32x16 sm;
            if (MODE == 2) sm = sload16(lm + 2 * LP + 8 * b);
#pragma unroll
            for (int q = 7; q >= 0; --q) {
                const int i = 8 * b + q;
                if (i >= L) continue;
                if (!ADJ) {
                    st_reset(x, m64_of(m, q));
                    fwd_step(x, MODE ? kb[i] * v[i] : 0.f, kg[i], k2[i], k3[i]);
                    if (MODE == 2) v[i] = zero_if(x.a, m64_of(sm, q));
                } else {
                    const float o = adj_step(x, MODE ? v[i] : 0.f, kb[i], kg[i], k2[i], k3[i]);
                    st_reset(x, m64_of(m, q));
                    if (MODE == 2) v[i] = zero_if(o, m64_of(sm, q));
                }
            }
        }
    }
    // 3x3 transfer matrix of the chunk for one sweep (columns = images of the basis states)
    template <bool DESC>
    __device__ __forceinline__ void transfer(float *A) const
    {
        float dummy[L];
        St e[3] = {{1.f, 0.f, 0.f}, {0.f, 1.f, 0.f}, {0.f, 0.f, 1.f}};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (DESC) desc<0>(e[k], dummy);
            else asc<0>(e[k], dummy);
            A[0 + k] = e[k].a;
            A[3 + k] = e[k].b;
            A[6 + k] = e[k].c;
        }
    }
};

// Kogge-Stone over the 64 chunks of a line with precomputed matrices.
// ks: [6 rounds][64 lanes][12] (9 used).  DESC scans from lane 63 down.
template <bool DESC>
__device__ __forceinline__ St ks_carry(St b, const float *ks, int lane)
{
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const int d = 1 << r;
        const St bp = DESC ? st_shfl_down(b, d) : st_shfl_up(b, d);
        const bool has = DESC ? lane + d < 64 : lane >= d;
        const float4 *q = reinterpret_cast<const float4 *>(ks + (r * 64 + lane) * 12);
        const float4 q0 = q[0], q1 = q[1], q2 = q[2];
        const float A[9] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x};
        St nb = b;
        mat_acc(A, bp, nb);
        if (has) b = nb;
    }
    // exclusive: state entering my chunk = inclusive state of the previous chunk
    St c = DESC ? st_shfl_down(b, 1) : st_shfl_up(b, 1);
    if (DESC ? lane == 63 : lane == 0) c = St{0.f, 0.f, 0.f};
    return c;
}

// round matrices A^(r) of the Kogge-Stone scan (accumulated product before round r)
template <bool DESC>
__device__ __forceinline__ void ks_build(float *A, float *ks, int lane)
{
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const int d = 1 << r;
        float *q = ks + (r * 64 + lane) * 12;
#pragma unroll
        for (int e = 0; e < 9; ++e) q[e] = A[e];
        float P[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) P[e] = DESC ? __shfl_down(A[e], d, 64) : __shfl_up(A[e], d, 64);
        const bool has = DESC ? lane + d < 64 : lane >= d;
        float N[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                N[3 * i + j] = fmaf(A[3 * i], P[j], fmaf(A[3 * i + 1], P[3 + j], A[3 * i + 2] * P[6 + j]));
#pragma unroll
        for (int e = 0; e < 9; ++e) A[e] = has ? N[e] : A[e];
    }
}

template <int L, bool ADJ>
__global__ __launch_bounds__(64 * kXWaves) void k_rf3x(const float *in, float *out, const float4 *__restrict__ T,
                                                        const uint64_t *__restrict__ LM, int nx, int ny,
                                                        int nplanes, int groups)
{
    __shared__ __align__(16) float ks[2][6 * 64 * 12];
    __shared__ float stage[kXWaves][64 * (L + 1)];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware order: consecutive blocks go to different XCDs; all groups of a row
    // land on the same XCD so its coefficients are shared in that XCD's L2.
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int row = (slot / groups) * 8 + xcd, grp = slot % groups;
    if (row >= ny) return;
    const long plane = (long)nx * ny;
    const int x0 = lane * L;

    XRow<L, ADJ> R;
    const float4 *trow = T + (long)row * nx;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int x = x0 + i;
        const float4 c = x < nx ? trow[x] : make_float4(0.f, 0.f, 0.f, 0.f);
        R.kb[i] = c.x;
        R.kg[i] = c.y;
        R.k2[i] = c.z;
        R.k3[i] = c.w;
    }
    R.lm = LM + (long)row * 3 * XRow<L, ADJ>::LP;

    if (wave == 0) {
        float A[9];
        R.template transfer<false>(A);
        ks_build<false>(A, ks[0], lane);
        R.template transfer<true>(A);
        ks_build<true>(A, ks[1], lane);
    }
    __syncthreads();

    float *stg = stage[wave];
    for (int ln = grp + groups * wave; ln < nplanes; ln += groups * kXWaves) {
        const float *src = in + ln * plane + (long)row * nx;
        float *dst = out + ln * plane + (long)row * nx;
        float v[L];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int x = x0 + i;
            v[i] = x < nx ? src[x] : 0.f;
        }
#pragma unroll
        for (int b = 0; b < XRow<L, ADJ>::LP / 8; ++b) {
            const u32x16 sm = sload16(R.lm + 2 * XRow<L, ADJ>::LP + 8 * b);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (8 * b + q < L) v[8 * b + q] = zero_if(v[8 * b + q], m64_of(sm, q));
        }
        St x{0.f, 0.f, 0.f};
        R.template asc<1>(x, v);
        x = ks_carry<false>(x, ks[0], lane);
        R.template asc<2>(x, v);
        St y{0.f, 0.f, 0.f};
        R.template desc<1>(y, v);
        y = ks_carry<true>(y, ks[1], lane);
        R.template desc<2>(y, v);
        // stage through LDS (chunk stride L+1 words) and store coalesced
#pragma unroll
        for (int i = 0; i < L; ++i) stg[lane * (L + 1) + i] = v[i];
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS writes done
        __builtin_amdgcn_wave_barrier();
        for (int k = lane; k < nx; k += 64) dst[k] = stg[(k / L) * (L + 1) + k % L];
        __builtin_amdgcn_wave_barrier();
    }
}

// ======================================================================
// y direction: 16 waves x 64 lanes per workgroup; wave w owns rows
// [w*L, w*L + L) of 32 columns; lane = (column j = lane & 31, plane h = lane >> 5).
// The chunk transfer matrices (per column, chunk and sweep) come from the
// coefficient block; carries pass between waves through LDS.  Coefficients are
// read from L2 one row at a time through a rolling window of kYWin loads.
// ======================================================================
constexpr int kYWin = 4;

template <int L, bool ADJ>
struct YCol {
    static constexpr int LP = (L + 7) & ~7;     // steps covered by whole 8-entry mask blocks
    const float4 *T;                            // coefficient table (column 0)
    uint32_t colb;                              // byte offset of this lane's column (clamped into the grid)
    const uint64_t *lm;                         // this column block's masks [3][lys], entry r+1 = row r
    int nx, ny, r0, lys;
    bool colok;

    // rows outside the grid are clamped: their coefficients are never used with a
    // nonzero state (the masks reset the state there), they only need to be finite
    // uniform row base + per-lane column offset
    __device__ __forceinline__ f4 coef(GLOBAL const float4 *Tb, int r) const
    {
        GLOBAL const char *row = (GLOBAL const char *)Tb + (long)min(max(r, 0), ny - 1) * nx * 16;
        return *(GLOBAL const f4 *)(row + colb);
    }
    // One pass over the chunk.  DESC: descending rows.  MODE 1: no output,
    // MODE 2: output into v (DESC also applies the sea mask).
    template <bool DESC, int MODE>
    __device__ __forceinline__ void pass(St &x, float *v) const
    {
        // ascending uses FRESET (forward: before the step) or BRESET (adjoint: after);
        // descending uses BRESET (forward) or FRESET (adjoint)
        const uint64_t *rp = lm + ((ADJ ? !DESC : DESC) ? lys : 0) + 1;
        GLOBAL const float4 *Tb = fresh(T);
        const int r0 = fresh_int(this->r0);
        f4 win[kYWin];
#pragma unroll
        for (int q = 0; q < kYWin; ++q) win[q] = coef(Tb, DESC ? r0 + L - 1 - q : r0 + q);
#pragma unroll
        for (int bb = 0; bb < LP / 8; ++bb) {
            const int b = DESC ? LP / 8 - 1 - bb : bb;
            const u32x16 m = sload16(rp + r0 + 8 * b);
            u32x16 sm;
            if (DESC && MODE == 2) sm = sload16(lm + 2 * lys + 1 + r0 + 8 * b);
#pragma unroll
            for (int qq = 0; qq < 8; ++qq) {
                const int q = DESC ? 7 - qq : qq;
                const int i = 8 * b + q;
                if (i >= L) continue;
                const int ii = DESC ? L - 1 - i : i;     // step number within the pass
                const f4 k = win[ii % kYWin];
                if (ii + kYWin < L) win[ii % kYWin] = coef(Tb, DESC ? r0 + i - kYWin : r0 + i + kYWin);
                float o;
                if (!ADJ) {
                    st_reset(x, m64_of(m, q));
                    fwd_step(x, k.x * v[i], k.y, k.z, k.w);
                    o = x.a;
                } else {
                    o = adj_step(x, v[i], k.x, k.y, k.z, k.w);
                    st_reset(x, m64_of(m, q));
                }
                if (MODE == 2) v[i] = (DESC) ? zero_if(o, m64_of(sm, q)) : o;
                mem_fence_compiler();   // keep the window's loads from being hoisted further
            }
        }
    }
};

template <int L, bool ADJ>
__global__ __launch_bounds__(64 * kYWaves, 1) void k_rf3y(const float *in, float *out,
                                                         const float4 *__restrict__ T,
                                                         const uint64_t *__restrict__ LM,
                                                         const float *__restrict__ PHI, int nx, int ny,
                                                         int nplanes, int nblk, int npairs)
{
    __shared__ __align__(16) float phi[2][kYWaves][kYCols][12];
    __shared__ float bsh[2][kYWaves][64][3];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = lane & 31, h = lane >> 5;
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    // XCD-aware order: all plane pairs of a column block run on one XCD (shared L2)
    const int blk = (slot / npairs) * 8 + xcd, pr = slot % npairs;
    if (blk >= nblk) return;
    const int col = blk * kYCols + j;
    const long plane = (long)nx * ny;
    YCol<L, ADJ> C;
    C.T = T;
    C.colb = (uint32_t)min(col, nx - 1) * 16u;   // columns past the grid are inactive (masks); any finite value will do
    C.nx = nx;
    C.ny = ny;
    C.r0 = w * L;
    C.lys = lmy_stride(L);
    C.colok = col < nx;
    C.lm = LM + (long)blk * 3 * C.lys;

    // transfer matrices of all chunks of this column block: [sweep][chunk][col][12]
    {
        const int k0 = ADJ ? 2 : 0;
        const float *src = PHI + (long)blk * 4 * kYWaves * kYCols * 12;
        for (int e = threadIdx.x; e < 2 * kYWaves * kYCols * 12; e += 64 * kYWaves) {
            const int s = e / (kYWaves * kYCols * 12), rest = e % (kYWaves * kYCols * 12);
            (&phi[0][0][0][0])[e] = src[(long)(k0 + s) * kYWaves * kYCols * 12 + rest];
        }
    }

    {
        const int pl = 2 * pr + h;
        const bool ok = C.colok && pl < nplanes;
        // lanes without a line read a valid address (their results are never stored)
        const uint32_t vb = ok ? ((uint32_t)h * (uint32_t)plane + (uint32_t)col) * 4u : 0u;
        GLOBAL const char *ib = (GLOBAL const char *)fresh(in) + (long)(2 * pr) * plane * 4;
        float v[L];
#pragma unroll
        for (int i = 0; i < L; ++i)
            v[i] = *(GLOBAL const float *)(ib + (long)min(C.r0 + i, ny - 1) * nx * 4 + vb);
#pragma unroll
        for (int b = 0; b < YCol<L, ADJ>::LP / 8; ++b) {
            const u32x16 sm = sload16(C.lm + 2 * C.lys + 1 + C.r0 + 8 * b);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (8 * b + q < L) v[8 * b + q] = zero_if(v[8 * b + q], m64_of(sm, q));
        }
        // ---- ascending sweep: local pass, chain over the chunks above, rerun
        St x{0.f, 0.f, 0.f};
        C.template pass<false, 1>(x, v);
        bsh[0][w][lane][0] = x.a;
        bsh[0][w][lane][1] = x.b;
        bsh[0][w][lane][2] = x.c;
        __syncthreads();
        St c{0.f, 0.f, 0.f};
        for (int k = 0; k < w; ++k) {
            const float4 *q = reinterpret_cast<const float4 *>(phi[0][k][j]);
            const float4 q0 = q[0], q1 = q[1], q2 = q[2];
            const float A[9] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x};
            St n{bsh[0][k][lane][0], bsh[0][k][lane][1], bsh[0][k][lane][2]};
            mat_acc(A, c, n);
            c = n;
        }
        x = c;
        C.template pass<false, 2>(x, v);
        // ---- descending sweep
        x = St{0.f, 0.f, 0.f};
        C.template pass<true, 1>(x, v);
        bsh[1][w][lane][0] = x.a;
        bsh[1][w][lane][1] = x.b;
        bsh[1][w][lane][2] = x.c;
        __syncthreads();
        c = St{0.f, 0.f, 0.f};
        for (int k = kYWaves - 1; k > w; --k) {
            const float4 *q = reinterpret_cast<const float4 *>(phi[1][k][j]);
            const float4 q0 = q[0], q1 = q[1], q2 = q[2];
            const float A[9] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x};
            St n{bsh[1][k][lane][0], bsh[1][k][lane][1], bsh[1][k][lane][2]};
            mat_acc(A, c, n);
            c = n;
        }
        x = c;
        C.template pass<true, 2>(x, v);
        if (ok) {
            GLOBAL char *ob = (GLOBAL char *)fresh(out) + (long)(2 * pr) * plane * 4;
#pragma unroll
            for (int i = 0; i < L; ++i)
                if (C.r0 + i < ny) *(GLOBAL float *)(ob + (long)(C.r0 + i) * nx * 4 + vb) = v[i];
        }
    }
}

// ---------------------------------------------------------------- setup
// Transfer matrices of the y kernel's chunks, FP64 from the FP32 table:
// PHI[blk][kind][w][j][12], kind 0 forward ascending, 1 forward descending,
// 2 adjoint ascending, 3 adjoint descending.  One thread per (column, chunk, kind).
__global__ void k_phi_y(const float4 *__restrict__ T, const uint8_t *__restrict__ code, float *__restrict__ PHI,
                        int nx, int ny, int L, int nblk)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nblk * kYCols * kYWaves * 4) return;
    const int j = (int)(t % kYCols);
    const int w = (int)((t / kYCols) % kYWaves);
    const int kind = (int)((t / (kYCols * kYWaves)) % 4);
    const int blk = (int)(t / (kYCols * kYWaves * 4));
    const int col = blk * kYCols + j;
    float *dst = PHI + ((((long)blk * 4 + kind) * kYWaves + w) * kYCols + j) * 12;
    auto cf = [&](int r) -> float4 {
        return (col < nx && r >= 0 && r < ny) ? T[(long)r * nx + col] : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto cd = [&](int r) -> uint8_t {
        return (col < nx && r >= 0 && r < ny) ? code[(long)r * nx + col] : (uint8_t)(CODE_FRESET | CODE_BRESET);
    };
    double A[9];
    for (int k = 0; k < 3; ++k) {
        double s0 = k == 0, s1 = k == 1, s2 = k == 2;
        for (int ii = 0; ii < L; ++ii) {
            const bool desc = kind & 1;
            const int r = w * L + (desc ? L - 1 - ii : ii);
            const float4 c = cf(r);
            const double gm = c.y, c2 = c.z, c3 = c.w;
            // forward kinds: zero before the step at a segment start (0) / end (1);
            // adjoint kinds: zero after the step at a segment end (2) / start (3)
            const uint8_t flag = kind == 0 ? CODE_FRESET : kind == 1 ? CODE_BRESET : kind == 2 ? CODE_BRESET : CODE_FRESET;
            const bool rs = cd(r) & flag;
            if (kind < 2) {
                if (rs) { s0 = 0; s1 = 0; s2 = 0; }
                const double tt = -gm * s0 - c2 * s1 - c3 * s2;
                s2 = s1;
                s1 = tt;
                s0 = s0 + tt;
            } else {
                const double u = s0 + s1;
                const double a = s0 - gm * u;
                s1 = s2 - c2 * u;
                s2 = -c3 * u;
                s0 = a;
                if (rs) { s0 = 0; s1 = 0; s2 = 0; }
            }
        }
        A[0 + k] = s0;
        A[3 + k] = s1;
        A[6 + k] = s2;
    }
    for (int e = 0; e < 9; ++e) dst[e] = (float)A[e];
    dst[9] = dst[10] = dst[11] = 0.f;
}

// ---------------------------------------------------------------- dispatch
template <int L, bool ADJ>
static hipError_t launch_x(const float *in, float *out, const float4 *T, const uint64_t *LM, int nx, int ny,
                           int nplanes, hipStream_t st)
{
    // groups per row: enough workgroups to cover the chip several times
    int groups = 1;
    while (groups < 8 && (long)((ny + 7) / 8) * 8 * groups < 2048 && groups * kXWaves * 2 <= nplanes) groups *= 2;
    const unsigned nb = (unsigned)(((ny + 7) / 8) * 8 * groups);
    k_rf3x<L, ADJ><<<nb, 64 * kXWaves, 0, st>>>(in, out, T, LM, nx, ny, nplanes, groups);
    return hipGetLastError();
}

template <int L, bool ADJ>
static hipError_t launch_y(const float *in, float *out, const float4 *T, const uint64_t *LM, const float *PHI,
                           int nx, int ny, int nplanes, hipStream_t st)
{
    const int nblk = (nx + kYCols - 1) / kYCols;
    const int npairs = (nplanes + 1) / 2;
    const unsigned nb = (unsigned)(((nblk + 7) / 8) * 8 * npairs);
    k_rf3y<L, ADJ><<<nb, 64 * kYWaves, 0, st>>>(in, out, T, LM, PHI, nx, ny, nplanes, nblk, npairs);
    return hipGetLastError();
}

#define RF_X_CASE(Lv)                                                                                     \
    case Lv:                                                                                              \
        return adj ? launch_x<Lv, true>(in, out, T, LM, nx, ny, nplanes, st)                              \
                   : launch_x<Lv, false>(in, out, T, LM, nx, ny, nplanes, st);
#define RF_Y_CASE(Lv)                                                                                     \
    case Lv:                                                                                              \
        return adj ? launch_y<Lv, true>(in, out, T, LM, PHI, nx, ny, nplanes, st)                         \
                   : launch_y<Lv, false>(in, out, T, LM, PHI, nx, ny, nplanes, st);

hipError_t fast_rf3_x(const float *in, float *out, const float4 *T, const uint64_t *LM, int lx, int nx, int ny,
                      int nplanes, bool adj, hipStream_t st)
{
    switch (lx) {
        RF_X_CASE(1) RF_X_CASE(2) RF_X_CASE(3) RF_X_CASE(4) RF_X_CASE(6) RF_X_CASE(8)
        RF_X_CASE(12) RF_X_CASE(16) RF_X_CASE(20) RF_X_CASE(24) RF_X_CASE(28) RF_X_CASE(32)
    default: return hipErrorNotSupported;
    }
}

hipError_t fast_rf3_y(const float *in, float *out, const float4 *T, const uint64_t *LM, const float *PHI, int ly,
                      int nx, int ny, int nplanes, bool adj, hipStream_t st)
{
    switch (ly) {
        RF_Y_CASE(2) RF_Y_CASE(4) RF_Y_CASE(8) RF_Y_CASE(12) RF_Y_CASE(16) RF_Y_CASE(24)
        RF_Y_CASE(32) RF_Y_CASE(40) RF_Y_CASE(48) RF_Y_CASE(56) RF_Y_CASE(64)
    default: return hipErrorNotSupported;
    }
}

hipError_t setup_phi_y(const float4 *T, const uint8_t *code, float *PHI, int nx, int ny, int ly, hipStream_t st)
{
    const int nblk = (nx + kYCols - 1) / kYCols;
    const long n = (long)nblk * kYCols * kYWaves * 4;
    k_phi_y<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(T, code, PHI, nx, ny, ly, nblk);
    return hipGetLastError();
}

}  // namespace rf
