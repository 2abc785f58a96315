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


}  // namespace

// ======================================================================
// x direction: one wave per line (a row of one plane); lane c owns points
// [c*L, c*L + L) with L odd.  All waves of a workgroup work on lines of the
// same row, which share its coefficients, lane masks and scan matrices.
// Loads go straight into the chunk layout (range-checked buffer loads; the
// next line is prefetched into registers while the current one is filtered).
// Results go through LDS so that the stores are coalesced; the odd L keeps the
// chunk-major LDS writes free of bank conflicts.
// ======================================================================
constexpr int kXWaves = 4;

typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));

// raw buffer over nbytes at p: loads past the end read 0, stores past it are dropped
__device__ __forceinline__ Rsrc make_rsrc(const void *p, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)nbytes, 0x00020000);
}

// L consecutive floats at byte offset off into v (dwordx4 groups, then the rest)
template <int L>
__device__ __forceinline__ void chunk_load(Rsrc r, int off, float *v)
{
#pragma unroll
    for (int j = 0; j + 4 <= L; j += 4) {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, off + 4 * j, 0, 0);
        v[j] = __uint_as_float(a.x);
        v[j + 1] = __uint_as_float(a.y);
        v[j + 2] = __uint_as_float(a.z);
        v[j + 3] = __uint_as_float(a.w);
    }
    constexpr int j = L & ~3, rem = L & 3;
    if (rem == 3) {
        const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(r, off + 4 * j, 0, 0);
        v[j] = __uint_as_float(a.x);
        v[j + 1] = __uint_as_float(a.y);
        v[j + 2] = __uint_as_float(a.z);
    }
    if (rem == 1) v[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off + 4 * j, 0, 0));
    static_assert(rem != 2, "L is odd");
}

template <int L, bool ADJ>
struct XRow {
    static constexpr int LP = (L + 7) & ~7;   // mask array length (whole 8-blocks)
    float kb[L], kg[L], k2[L], k3[L];          // beta, gamma, c2, c3 of my chunk's points
    const uint64_t *lm;                        // this row's masks: [3][LP] FRESET, BRESET, not-SEA

    // ascending sweep over my chunk.  MODE 1: input v, no output;
    // MODE 2: input v, output written back into v.
    template <int MODE>
    __device__ __forceinline__ void asc(St &x, float *v) const
    {
        // forward: zero the state before a segment start; adjoint: after a segment end.
        // The opaque zero keeps this pass's mask loads inside the pass.
        const uint64_t *rp = lm + (ADJ ? LP : 0) + fresh_int(0);
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const uint64_t m = rp[i];
            if (!ADJ) {
                st_reset(x, m);
                fwd_step(x, kb[i] * v[i], kg[i], k2[i], k3[i]);
                if (MODE == 2) v[i] = x.a;
            } else {
                const float o = adj_step(x, v[i], kb[i], kg[i], k2[i], k3[i]);
                st_reset(x, m);
                if (MODE == 2) v[i] = o;
            }
        }
    }
    // descending sweep over my chunk; MODE 2 also applies the sea mask to the output
    template <int MODE>
    __device__ __forceinline__ void desc(St &x, float *v) const
    {
        // forward: zero the state before a segment end; adjoint: after a segment start
        const int z = fresh_int(0);
        const uint64_t *rp = lm + (ADJ ? 0 : LP) + z;
        const uint64_t *sp = lm + 2 * LP + z;
#pragma unroll
        for (int i = L - 1; i >= 0; --i) {
            const uint64_t m = rp[i];
            if (!ADJ) {
                st_reset(x, m);
                fwd_step(x, kb[i] * v[i], kg[i], k2[i], k3[i]);
                if (MODE == 2) v[i] = zero_if(x.a, sp[i]);
            } else {
                const float o = adj_step(x, v[i], kb[i], kg[i], k2[i], k3[i]);
                st_reset(x, m);
                if (MODE == 2) v[i] = zero_if(o, sp[i]);
            }
        }
    }
};

// ---- carry scan over the 64 chunks of a line, in registers (DPP) ----------
// Chunk c maps its incoming state s to Phi_c s + b_c.  The scan turns the local
// end states b into the state entering every chunk.  Ascending order (lane 0
// first): four in-row rounds (row_shr 1, 2, 4, 8 within 16-lane rows), then
// the standard row broadcasts (lane 15 -> rows 1 and 3, lane 31 -> rows 2 and
// 3).  Descending order mirrors this with row_shl; its two cross-row rounds
// take lane 16/48 -> rows 0/2 and lane 32 -> rows 0 and 1.  Round r adds
// K[r] * (state received), with K[r] the product of the Phi between the two
// chunks (zero where nothing is received).
constexpr int kKs = 55;   // floats per lane in the round-matrix table: 6 x 9, odd stride

template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWMASK, 0xF, true));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ St st_dpp(const St &x)
{
    return St{dpp<CTRL, ROWMASK>(x.a), dpp<CTRL, ROWMASK>(x.b), dpp<CTRL, ROWMASK>(x.c)};
}
enum : int {
    DPP_ROW_SHL = 0x100, DPP_ROW_SHR = 0x110, DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138,
    DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143,
};

// C = A B, 3x3 row-major
__device__ __forceinline__ void mat_mul(const float *A, const float *B, float *C)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = fmaf(A[3 * i], B[j], fmaf(A[3 * i + 1], B[3 + j], A[3 * i + 2] * B[6 + j]));
}
__device__ __forceinline__ void mat_put(float *q, const float *A, bool keep)
{
#pragma unroll
    for (int e = 0; e < 9; ++e) q[e] = keep ? A[e] : 0.f;
}

// round matrices of one scan direction from this lane's Phi; K: [64 lanes][kKs]
template <bool DESC>
__device__ __forceinline__ void ks_build(const float *Phi, float *K, int lane)
{
    const int p = lane & 15, row = lane >> 4;
    float *k = K + lane * kKs;
    float A[9], Q[9], T[9], N[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) A[e] = Q[e] = Phi[e];
    // A: product over the d chunks ending (in scan order) at mine; Q: over my row so far
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int d = 1 << r;
        const bool in_row = DESC ? p + d <= 15 : p >= d;
        mat_put(k + 9 * r, A, in_row);
#pragma unroll
        for (int e = 0; e < 9; ++e) T[e] = DESC ? __shfl_down(A[e], d, 64) : __shfl_up(A[e], d, 64);
        mat_mul(A, T, N);
#pragma unroll
        for (int e = 0; e < 9; ++e) A[e] = N[e];
#pragma unroll
        for (int e = 0; e < 9; ++e) T[e] = DESC ? __shfl_down(Q[e], d, 64) : __shfl_up(Q[e], d, 64);
        mat_mul(Q, T, N);
#pragma unroll
        for (int e = 0; e < 9; ++e) Q[e] = in_row ? N[e] : Q[e];
    }
    mat_put(k + 36, Q, DESC ? (row == 0 || row == 2) : (row == 1 || row == 3));
    // whole-row product of the row between mine and the source of the last round
#pragma unroll
    for (int e = 0; e < 9; ++e) T[e] = __shfl(Q[e], DESC ? 16 : 47, 64);
    mat_mul(Q, T, N);
    const bool two_rows = DESC ? row == 0 : row == 3;
#pragma unroll
    for (int e = 0; e < 9; ++e) Q[e] = two_rows ? N[e] : Q[e];
    mat_put(k + 45, Q, DESC ? row <= 1 : row >= 2);
}

__device__ __forceinline__ void ks_round(const float *k, const St &x, St &y)
{
    float A[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) A[e] = k[e];
    mat_acc(A, x, y);
}

// b: local end state of my chunk; returns the state entering my chunk
template <bool DESC>
__device__ __forceinline__ St ks_carry(St b, const float *K, int lane)
{
    const float *k = K + lane * kKs;
    if (!DESC) {
        ks_round(k + 0, st_dpp<DPP_ROW_SHR + 1, 0xF>(b), b);
        ks_round(k + 9, st_dpp<DPP_ROW_SHR + 2, 0xF>(b), b);
        ks_round(k + 18, st_dpp<DPP_ROW_SHR + 4, 0xF>(b), b);
        ks_round(k + 27, st_dpp<DPP_ROW_SHR + 8, 0xF>(b), b);
        ks_round(k + 36, st_dpp<DPP_ROW_BCAST15, 0xA>(b), b);
        ks_round(k + 45, st_dpp<DPP_ROW_BCAST31, 0xC>(b), b);
        return st_dpp<DPP_WAVE_SHR1, 0xF>(b);
    }
    ks_round(k + 0, st_dpp<DPP_ROW_SHL + 1, 0xF>(b), b);
    ks_round(k + 9, st_dpp<DPP_ROW_SHL + 2, 0xF>(b), b);
    ks_round(k + 18, st_dpp<DPP_ROW_SHL + 4, 0xF>(b), b);
    ks_round(k + 27, st_dpp<DPP_ROW_SHL + 8, 0xF>(b), b);
    const int src = (lane & 16) ? lane : (lane & ~15) + 16;   // rows 0 and 2 take rows 1 and 3
    ks_round(k + 36, St{__shfl(b.a, src, 64), __shfl(b.b, src, 64), __shfl(b.c, src, 64)}, b);
    const St u{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.a), 32)),
               __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.b), 32)),
               __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.c), 32))};
    ks_round(k + 45, u, b);
    return st_dpp<DPP_WAVE_SHL1, 0xF>(b);
}

template <int L>
constexpr int x_stage_floats() { return 256 * ((L + 3) / 4); }   // whole dwordx4 store rounds

template <int L, bool ADJ>
__global__ __launch_bounds__(64 * kXWaves, (L <= 23 ? 3 : 2)) void k_rf3x(
    const float *in, float *out, const float4 *__restrict__ T, const uint64_t *__restrict__ LM,
    const float *__restrict__ PHI, int nx, int ny, int nplanes, int groups)
{
    __shared__ float K[2][64 * kKs];
    __shared__ __align__(16) float stage[kXWaves][x_stage_floats<L>()];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware order: consecutive blocks go to different XCDs; all groups of a row
    // land on the same XCD so its coefficients are shared in that XCD's L2.
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int row = (slot / groups) * 8 + xcd, grp = slot % groups;
    if (row >= ny) return;
    const long plane = (long)nx * ny;
    const int x0 = lane * L;
    const uint32_t line_bytes = (uint32_t)nx * 4u;

    XRow<L, ADJ> R;
    {
        const Rsrc tr = make_rsrc(T + (long)row * nx, (uint32_t)nx * 16u);
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(tr, (x0 + i) * 16, 0, 0);
            R.kb[i] = __uint_as_float(c.x);
            R.kg[i] = __uint_as_float(c.y);
            R.k2[i] = __uint_as_float(c.z);
            R.k3[i] = __uint_as_float(c.w);
        }
    }
    R.lm = LM + (long)row * 3 * XRow<L, ADJ>::LP;
    if (wave < 2) {   // wave 0: ascending scan matrices, wave 1: descending
        const float *p = PHI + (((long)row * 4 + (ADJ ? 2 : 0) + wave) * 64 + lane) * 12;
        float A[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) A[e] = p[e];
        if (wave == 0) ks_build<false>(A, K[0], lane);
        else ks_build<true>(A, K[1], lane);
    }
    __syncthreads();

    float *stg = stage[wave];
    const int lstep = groups * kXWaves;
    const int nst = (nx + 255) / 256;   // dwordx4 store rounds per line
    int ln = grp + groups * wave;
    float v[L], vn[L];   // the current line, and the next one in flight
    if (ln < nplanes) chunk_load<L>(make_rsrc(in + (long)ln * plane + (long)row * nx, line_bytes), x0 * 4, vn);
    for (; ln < nplanes; ln += lstep) {
#pragma unroll
        for (int i = 0; i < L; ++i) v[i] = vn[i];
        if (ln + lstep < nplanes)
            chunk_load<L>(make_rsrc(in + (long)(ln + lstep) * plane + (long)row * nx, line_bytes), x0 * 4, vn);
        {
            const uint64_t *sp = R.lm + 2 * XRow<L, ADJ>::LP + fresh_int(0);
#pragma unroll
            for (int i = 0; i < L; ++i) v[i] = zero_if(v[i], sp[i]);   // input only at sea points
        }
        St x{0.f, 0.f, 0.f};
        R.template asc<1>(x, v);
        x = ks_carry<false>(x, K[0], lane);
        R.template asc<2>(x, v);
        St y{0.f, 0.f, 0.f};
        R.template desc<1>(y, v);
        y = ks_carry<true>(y, K[1], lane);
        R.template desc<2>(y, v);
        // chunk-major into LDS, out in coalesced dwordx4 rounds
#pragma unroll
        for (int i = 0; i < L; ++i) stg[x0 + i] = v[i];
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS writes done
        __builtin_amdgcn_wave_barrier();
        const Rsrc ro = make_rsrc(out + (long)ln * plane + (long)row * nx, line_bytes);
#pragma unroll
        for (int it = 0; it < (L + 3) / 4; ++it) {
            if (it < nst) {
                const f4 q = *reinterpret_cast<const f4 *>(stg + 4 * lane + 256 * it);
                u32x4 w;
                w.x = __float_as_uint(q.x);
                w.y = __float_as_uint(q.y);
                w.z = __float_as_uint(q.z);
                w.w = __float_as_uint(q.w);
                __builtin_amdgcn_raw_buffer_store_b128(w, ro, (4 * lane + 256 * it) * 4, 0, 0);
            }
        }
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
// 3x3 transfer matrix of one chunk of n points, FP64 from the FP32 table.
// kind 0 forward ascending, 1 forward descending, 2 adjoint ascending,
// 3 adjoint descending.  Forward kinds zero the state before the step at a
// segment start (0) / end (1); adjoint kinds after the step at a segment end
// (2) / start (3).  cf(i), cd(i): coefficients and code of chunk point i
// (ascending position).
template <class CF, class CD>
__device__ void chunk_transfer(int kind, int n, CF cf, CD cd, float *dst)
{
    const bool desc = kind & 1;
    const uint8_t flag = kind == 0 ? CODE_FRESET : kind == 1 ? CODE_BRESET : kind == 2 ? CODE_BRESET : CODE_FRESET;
    double A[9];
    for (int k = 0; k < 3; ++k) {
        double s0 = k == 0, s1 = k == 1, s2 = k == 2;
        for (int ii = 0; ii < n; ++ii) {
            const int i = desc ? n - 1 - ii : ii;
            const float4 c = cf(i);
            const double gm = c.y, c2 = c.z, c3 = c.w;
            const bool rs = cd(i) & flag;
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

// y kernel's chunks: PHI[blk][kind][w][j][12], one thread per (column, chunk, kind)
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
    const bool cok = col < nx;
    auto cf = [&](int i) -> float4 {
        const int r = w * L + i;
        return (cok && r < ny) ? T[(long)r * nx + col] : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto cd = [&](int i) -> uint8_t {
        const int r = w * L + i;
        return (cok && r < ny) ? code[(long)r * nx + col] : (uint8_t)(CODE_FRESET | CODE_BRESET);
    };
    chunk_transfer(kind, L, cf, cd, dst);
}

// x kernel's chunks: PHI[row][kind][c][12], one thread per (row, kind, chunk)
__global__ void k_phi_x(const float4 *__restrict__ T, const uint8_t *__restrict__ code, float *__restrict__ PHI,
                        int nx, int ny, int L)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)ny * 4 * 64) return;
    const int c = (int)(t % 64);
    const int kind = (int)((t / 64) % 4);
    const int row = (int)(t / 256);
    const float4 *tr = T + (long)row * nx;
    const uint8_t *cr = code + (long)row * nx;
    auto cf = [&](int i) -> float4 {
        const int x = c * L + i;
        return x < nx ? tr[x] : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto cd = [&](int i) -> uint8_t {
        const int x = c * L + i;
        return x < nx ? cr[x] : (uint8_t)(CODE_FRESET | CODE_BRESET);
    };
    chunk_transfer(kind, L, cf, cd, PHI + t * 12);
}

// ---------------------------------------------------------------- dispatch
template <int L, bool ADJ>
static hipError_t launch_x(const float *in, float *out, const float4 *T, const uint64_t *LM, const float *PHI,
                           int nx, int ny, int nplanes, hipStream_t st)
{
    // groups per row: enough workgroups to cover the chip several times
    int groups = 1;
    while (groups < 8 && (long)((ny + 7) / 8) * 8 * groups < 2048 && groups * kXWaves * 2 <= nplanes) groups *= 2;
    const unsigned nb = (unsigned)(((ny + 7) / 8) * 8 * groups);
    k_rf3x<L, ADJ><<<nb, 64 * kXWaves, 0, st>>>(in, out, T, LM, PHI, nx, ny, nplanes, groups);
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
        return adj ? launch_x<Lv, true>(in, out, T, LM, PHI, nx, ny, nplanes, st)                         \
                   : launch_x<Lv, false>(in, out, T, LM, PHI, nx, ny, nplanes, st);
#define RF_Y_CASE(Lv)                                                                                     \
    case Lv:                                                                                              \
        return adj ? launch_y<Lv, true>(in, out, T, LM, PHI, nx, ny, nplanes, st)                         \
                   : launch_y<Lv, false>(in, out, T, LM, PHI, nx, ny, nplanes, st);

hipError_t fast_rf3_x(const float *in, float *out, const float4 *T, const uint64_t *LM, const float *PHI, int lx,
                      int nx, int ny, int nplanes, bool adj, hipStream_t st)
{
    switch (lx) {
        RF_X_CASE(1) RF_X_CASE(3) RF_X_CASE(5) RF_X_CASE(7) RF_X_CASE(9) RF_X_CASE(11) RF_X_CASE(13)
        RF_X_CASE(15) RF_X_CASE(17) RF_X_CASE(19) RF_X_CASE(21) RF_X_CASE(23) RF_X_CASE(25) RF_X_CASE(27)
        RF_X_CASE(29) RF_X_CASE(31) RF_X_CASE(33)
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

hipError_t setup_phi_x(const float4 *T, const uint8_t *code, float *PHI, int nx, int ny, int lx, hipStream_t st)
{
    const long n = (long)ny * 4 * 64;
    k_phi_x<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(T, code, PHI, nx, ny, lx);
    return hipGetLastError();
}

hipError_t setup_phi_y(const float4 *T, const uint8_t *code, float *PHI, int nx, int ny, int ly, hipStream_t st)
{
    const int nblk = (nx + kYCols - 1) / kYCols;
    const long n = (long)nblk * kYCols * kYWaves * 4;
    k_phi_y<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(T, code, PHI, nx, ny, ly, nblk);
    return hipGetLastError();
}

}  // namespace rf
