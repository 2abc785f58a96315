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

#include <type_traits>

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
// read-only tables read with scalar loads: constant address space
#define CONST_AS __attribute__((address_space(4)))
typedef const CONST_AS uint64_t *mask_ptr;
__device__ __forceinline__ mask_ptr as_const(const uint64_t *p) { return (mask_ptr)p; }
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

// a wave-uniform value read from memory, as a scalar (the compiler cannot always
// prove that such loads are uniform)
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <class T>
__device__ __forceinline__ T *uni(T *p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
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
// beta_j * u before the reset of the state (OUT), or nothing (local passes)
template <bool OUT>
__device__ __forceinline__ float adj_step(St &x, float r, float bt, float gm, float c2, float c3)
{
    const float w0 = x.a + r;
    const float u = w0 + x.b;
    x.a = fmaf(-gm, u, w0);
    x.b = fmaf(-c2, u, x.c);
    x.c = -c3 * u;
    if (!OUT) return 0.f;
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
// Lines are loaded and stored in coalesced dwordx4 rounds (range-checked
// buffer accesses) and pass through LDS between that order and the chunk
// layout; the odd L keeps the chunk-major LDS accesses free of bank conflicts.
// The next line is in flight in registers while the current one is filtered.
// ======================================================================
constexpr int kXWaves = 4;

typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));

// cache policies of the field accesses (data read or written once): the
// non-temporal hint, so that streaming a field does not evict the coefficient
// tables the sweeps re-read from L2 (the x kernel's coalesced line loads and
// stores too: it keeps its own coefficients in registers, but the y kernel
// after it needs L2 for its tables).
constexpr int kStreamLoadY = 2, kStreamStoreY = 2, kStreamLoadX = 2, kStreamStoreX = 2;

// raw buffer over nbytes at p: loads past the end read 0, stores past it are dropped
__device__ __forceinline__ Rsrc make_rsrc(const void *p, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)nbytes, 0x00020000);
}

template <int L, bool ADJ>
struct XRow {
    static constexpr int LP = (L + 7) & ~7;   // mask array length (whole 8-blocks)
    float kb[L], kg[L], k2[L], k3[L];          // beta, gamma, c2, c3 of my chunk's points
    mask_ptr lm;                               // this row's masks: [3][LP] FRESET, BRESET, not-SEA

    // ascending sweep over my chunk.  MODE 1: input v, no output;
    // MODE 2: input v, output written back into v.  Forward inputs are beta_i s_i
    // (formed once for both passes), and the forward output is beta_i u_i, the
    // input of the anti-causal passes.
    // PER (periodic rows): `save` receives the state after step s_hook (the
    // row's last point, in the last real chunk), and desc sets the state of lane
    // `inj_lane` to `inj` before step s_hook.
    template <int MODE, bool PER = false>
    __device__ __forceinline__ void asc(St &x, float *v, int s_hook = 0, St *save = nullptr) const
    {
        // forward: zero the state before a segment start; adjoint: after a segment end.
        // The opaque zero keeps this pass's mask loads inside the pass.
        mask_ptr rp = lm + (ADJ ? LP : 0) + fresh_int(0);
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const uint64_t m = rp[i];
            if (!ADJ) {
                st_reset(x, m);
                fwd_step(x, v[i], kg[i], k2[i], k3[i]);
                if (MODE == 2) v[i] = kb[i] * x.a;
            } else {
                const float o = adj_step<MODE == 2>(x, v[i], kb[i], kg[i], k2[i], k3[i]);
                st_reset(x, m);
                if (MODE == 2) v[i] = o;
            }
            if (PER && i == s_hook) *save = x;
        }
    }
    // asc<2> with exact ends: at a segment end (fourth mask slab) the state after
    // the step (forward: the causal state (p, d1, d2); adjoint: before the reset,
    // the costate of the anti-causal start state) times the point's 3x3 map N
    // (EN: this row's maps, 36 floats per point, this kernel's at offset 0)
    // is added to v at the point and the two before it; corrections for points
    // of the previous chunk accumulate in co1 (its last point) and co2 (the one
    // before).
    __device__ __forceinline__ void asc2_end(St &x, float *v, const float *EN, int lane, float &co1, float &co2) const
    {
        const int z = fresh_int(0);
        mask_ptr rp = lm + (ADJ ? LP : 0) + z;
        mask_ptr ep = lm + 3 * LP + z;
        const int x0 = lane * L;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const uint64_t m = rp[i];
            const uint64_t em = ep[i];
            St s;
            if (!ADJ) {
                st_reset(x, m);
                fwd_step(x, v[i], kg[i], k2[i], k3[i]);
                v[i] = kb[i] * x.a;
                s = x;
            } else {
                v[i] = adj_step<true>(x, v[i], kb[i], kg[i], k2[i], k3[i]);
                s = x;
                st_reset(x, m);
            }
            if (em != 0 && ((em >> lane) & 1)) {
                const float *N = EN + (long)(x0 + i) * 36;
                float n[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) n[q] = N[q];
                const float r0 = fmaf(n[0], s.a, fmaf(n[1], s.b, n[2] * s.c));
                const float r1 = fmaf(n[3], s.a, fmaf(n[4], s.b, n[5] * s.c));
                const float r2 = fmaf(n[6], s.a, fmaf(n[7], s.b, n[8] * s.c));
                v[i] += r0;
                if (i >= 1) v[i >= 1 ? i - 1 : 0] += r1;
                else co1 += r1;
                if (i >= 2) v[i >= 2 ? i - 2 : 0] += r2;
                else if (i == 1) co1 += r2;
                else co2 += r2;
            }
        }
    }
    // descending sweep over my chunk; MODE 2 also applies the sea mask to the output
    template <int MODE, bool PER = false>
    __device__ __forceinline__ void desc(St &x, float *v, int s_hook = 0, bool inj_lane = false,
                                         St inj = St{0.f, 0.f, 0.f}) const
    {
        // forward: zero the state before a segment end; adjoint: after a segment start
        const int z = fresh_int(0);
        mask_ptr rp = lm + (ADJ ? 0 : LP) + z;
        mask_ptr sp = lm + 2 * LP + z;
#pragma unroll
        for (int i = L - 1; i >= 0; --i) {
            const uint64_t m = rp[i];
            if (PER && i == s_hook) {
                x.a = inj_lane ? inj.a : x.a;
                x.b = inj_lane ? inj.b : x.b;
                x.c = inj_lane ? inj.c : x.c;
            }
            if (!ADJ) {
                st_reset(x, m);
                fwd_step(x, v[i], kg[i], k2[i], k3[i]);
                if (MODE == 2) v[i] = zero_if(x.a, sp[i]);
            } else {
                const float o = adj_step<MODE == 2>(x, v[i], kb[i], kg[i], k2[i], k3[i]);
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

// b: local end state of my chunk; returns the state entering my chunk.  With
// incl0, the descending scan also returns the state leaving chunk 0 (lane 0's
// inclusive value).
template <bool DESC>
__device__ __forceinline__ St ks_carry(St b, const float *K, int lane, St *incl0 = nullptr)
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
    if (incl0)
        *incl0 = St{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.a), 0)),
                    __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.b), 0)),
                    __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.c), 0))};
    return st_dpp<DPP_WAVE_SHL1, 0xF>(b);
}

// a wave-uniform 3x3 (row-major, 12-float entry) of a read-only table
__device__ __forceinline__ void load_m3(const float *p, float *A)
{
#pragma unroll
    for (int e = 0; e < 9; ++e) A[e] = p[e];
}

template <int L>
constexpr int x_stage_floats() { return 256 * ((L + 3) / 4); }   // whole dwordx4 store rounds

// Lines of one row: planes grp, grp + groups, ... (4 waves, interleaved).
// K: [2][64 * kKs] scan matrices, stage: this wave's LDS staging area.
template <int L, bool ADJ, bool PER = false, bool END = false>
__device__ __forceinline__ void x_rows(const float *in, float *out, const float4 *T, const uint64_t *LM,
                                       const float *PHI, int nx, int ny, int nplanes, int row, int grp,
                                       int groups, float *K, float *stg, const float *PERT = nullptr,
                                       const float *ENDT = nullptr)
{
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
    R.lm = as_const(LM + (long)row * kLaneMasks * XRow<L, ADJ>::LP);
    if (wave < 2) {   // wave 0: ascending scan matrices, wave 1: descending
        const float *p = PHI + (((long)row * 4 + (ADJ ? 2 : 0) + wave) * 64 + lane) * 12;
        float A[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) A[e] = p[e];
        if (wave == 0) ks_build<false>(A, K, lane);
        else ks_build<true>(A, K + 64 * kKs, lane);
    }
    __syncthreads();

    const int lstep = groups * kXWaves;
    const int nst = (nx + 255) / 256;   // dwordx4 store rounds per line
    int ln = grp + groups * wave;
    // lines arrive in coalesced dwordx4 rounds (lane l: floats 4l .. 4l+3 of each
    // 256) with the non-temporal hint, and go into chunk layout through this
    // wave's LDS staging area; the next line is in flight while one is filtered
    constexpr int NR = (L + 3) / 4;
    float v[L];
    u32x4 q[NR];
    auto line_load = [&](int l) {
        const Rsrc r = make_rsrc(in + (long)l * plane + (long)row * nx, line_bytes);
#pragma unroll
        for (int it = 0; it < NR; ++it)
            q[it] = __builtin_amdgcn_raw_buffer_load_b128(r, (4 * lane + 256 * it) * 4, 0, kStreamLoadX);
    };
    if (ln < nplanes) line_load(ln);
    for (; ln < nplanes; ln += lstep) {
#pragma unroll
        for (int it = 0; it < NR; ++it) *reinterpret_cast<u32x4 *>(stg + 4 * lane + 256 * it) = q[it];
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS writes done
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < L; ++i) v[i] = stg[x0 + i];
        if (ln + lstep < nplanes) line_load(ln + lstep);
        {
            mask_ptr sp = R.lm + 2 * XRow<L, ADJ>::LP + fresh_int(0);
#pragma unroll
            for (int i = 0; i < L; ++i) {
                v[i] = zero_if(v[i], sp[i]);   // input only at sea points
                if (!ADJ) v[i] = R.kb[i] * v[i];
            }
        }
        St x{0.f, 0.f, 0.f};
        if (!PER) {
            R.template asc<1>(x, v);
            x = ks_carry<false>(x, K, lane);
            if (!END) {
                R.template asc<2>(x, v);
            } else {
                // exact ends: at a segment end the pass adds N (its state) to the
                // anti-causal inputs of the point and the two before it; those of the
                // previous chunk go back to it (wave shifts)
                float co1 = 0.f, co2 = 0.f;
                R.asc2_end(x, v, ENDT + (long)row * nx * 36 + (ADJ ? 12 : 0), lane, co1, co2);
                const float b1 = dpp<DPP_WAVE_SHL1, 0xF>(co1), b2 = dpp<DPP_WAVE_SHL1, 0xF>(co2);
                v[L - 1] += b1;
                if (L >= 2) v[L >= 2 ? L - 2 : 0] += b2;
                else v[L - 1] += dpp<DPP_WAVE_SHL1, 0xF>(b2);
            }
            St y{0.f, 0.f, 0.f};
            R.template desc<1>(y, v);
            y = ks_carry<true>(y, K + 64 * kKs, lane);
            R.template desc<2>(y, v);
        } else {
            // periodic row: the carry scans are cyclic.  Ascending: the state after
            // the row's last point (x = nx-1, step s_last of chunk c_last) with a zero
            // state entering x = 0 is Phi_last carry(c_last) + (its local state); the
            // state entering x = 0 is the fixed point x0 = W that, and every chunk's
            // carry gains P_c x0.  Descending: mirrored, from the state leaving chunk
            // 0, with lane c_last's state set at its last real point.
            const int clast = (nx - 1) / L, slast = (nx - 1) % L;
            const float *pa = PERT + ((long)row * 4 + (ADJ ? 2 : 0)) * kPerXEntries * 12;
            const float *pd = PERT + ((long)row * 4 + (ADJ ? 3 : 1)) * kPerXEntries * 12;
            St saved{0.f, 0.f, 0.f};
            R.template asc<1, true>(x, v, slast, &saved);
            x = ks_carry<false>(x, K, lane);
            {
                float A[9];
                load_m3(pa + 65 * 12, A);
                St bw = saved;
                mat_acc(A, x, bw);
                const St b{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(bw.a), clast)),
                           __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bw.b), clast)),
                           __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bw.c), clast))};
                load_m3(pa + 64 * 12, A);
                St x0{0.f, 0.f, 0.f};
                mat_acc(A, b, x0);
                load_m3(pa + lane * 12, A);
                mat_acc(A, x0, x);
            }
            R.template asc<2>(x, v);
            St y{0.f, 0.f, 0.f};
            R.template desc<1>(y, v);
            St out0;
            y = ks_carry<true>(y, K + 64 * kKs, lane, &out0);
            St xw{0.f, 0.f, 0.f};
            {
                float A[9];
                load_m3(pd + 64 * 12, A);
                mat_acc(A, out0, xw);
                load_m3(pd + lane * 12, A);
                mat_acc(A, xw, y);
            }
            R.template desc<2, true>(y, v, slast, lane == clast, xw);
        }
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
                __builtin_amdgcn_raw_buffer_store_b128(w, ro, (4 * lane + 256 * it) * 4, 0, kStreamStoreX);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <int L, bool ADJ, bool PER, bool END>
__global__ __launch_bounds__(64 * kXWaves, (L <= 23 ? 3 : 2)) void k_rf3x(
    const float *in, float *out, const float4 *__restrict__ T, const uint64_t *__restrict__ LM,
    const float *__restrict__ PHI, int nx, int ny, int nplanes, int groups, const float *__restrict__ PERT,
    const float *__restrict__ ENDT)
{
    __shared__ float K[2 * 64 * kKs];
    __shared__ __align__(16) float stage[kXWaves][x_stage_floats<L>()];
    // XCD-aware order: consecutive blocks go to different XCDs; all groups of a row
    // land on the same XCD so its coefficients are shared in that XCD's L2.
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int row = (slot / groups) * 8 + xcd, grp = slot % groups;
    if (row >= ny) return;
    x_rows<L, ADJ, PER, END>(in, out, T, LM, PHI, nx, ny, nplanes, row, grp, groups, K,
                             stage[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)], PERT, ENDT);
}

// Depth-dependent tables (LevTabs): each level has its own coefficients, lane
// masks, scan matrices and (periodic rows) cyclic-scan tables, so every wave
// takes one (level, row) on its own (that row's line in each field) and builds
// its scan matrices itself, one sweep at a time, in its own LDS slice.  A wave
// reads and writes only its own slices, so the kernel has no workgroup barrier
// and a wave past the last row returns.
template <int L, bool ADJ, bool PER, bool END>
__global__ __launch_bounds__(64 * kXWaves, 2) void k_rf3x_lev(const float *in, float *out,
                                                             const float4 *__restrict__ T,
                                                             const uint64_t *__restrict__ LM,
                                                             const float *__restrict__ PHI, int nx, int ny,
                                                             int nfields, LevTabs S, const float *__restrict__ PERT,
                                                             const float *__restrict__ ENDT)
{
    static_assert(!(PER && END), "periodic rows with exact ends run the line-sequential kernels");
    __shared__ float K[kXWaves][64 * kKs];
    __shared__ __align__(16) float stage[kXWaves][x_stage_floats<L>()];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long u = (long)blockIdx.x * kXWaves + wave;   // level * ny + row
    if (u >= (long)S.nlev * ny) return;
    const int lev = (int)(u / ny), row = (int)(u % ny);
    T += lev * S.t;
    LM += lev * S.lm;
    PHI += lev * S.phi;
    float *Kw = K[wave], *stg = stage[wave];
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
    R.lm = as_const(LM + (long)row * kLaneMasks * XRow<L, ADJ>::LP);
    const float *ph = PHI + (((long)row * 4 + (ADJ ? 2 : 0)) * 64 + lane) * 12;   // ascending; descending next
    const int nst = (nx + 255) / 256;
    constexpr int NR = (L + 3) / 4;
    for (int f = 0; f < nfields; ++f) {
        const long ln = (long)f * S.nlev + lev;
        {
            const Rsrc r = make_rsrc(in + ln * plane + (long)row * nx, line_bytes);
            u32x4 q[NR];
#pragma unroll
            for (int it = 0; it < NR; ++it)
                q[it] = __builtin_amdgcn_raw_buffer_load_b128(r, (4 * lane + 256 * it) * 4, 0, kStreamLoadX);
#pragma unroll
            for (int it = 0; it < NR; ++it) *reinterpret_cast<u32x4 *>(stg + 4 * lane + 256 * it) = q[it];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS writes done
        __builtin_amdgcn_wave_barrier();
        float v[L];
#pragma unroll
        for (int i = 0; i < L; ++i) v[i] = stg[x0 + i];
        {
            mask_ptr sp = R.lm + 2 * XRow<L, ADJ>::LP + fresh_int(0);
#pragma unroll
            for (int i = 0; i < L; ++i) {
                v[i] = zero_if(v[i], sp[i]);   // input only at sea points
                if (!ADJ) v[i] = R.kb[i] * v[i];
            }
        }
        float A[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) A[e] = ph[e];
        ks_build<false>(A, Kw, lane);
        St x{0.f, 0.f, 0.f};
        if (!PER) {
            R.template asc<1>(x, v);
            x = ks_carry<false>(x, Kw, lane);
            if (!END) {
                R.template asc<2>(x, v);
            } else {
                float co1 = 0.f, co2 = 0.f;
                R.asc2_end(x, v, ENDT + lev * S.end + (long)row * nx * 36 + (ADJ ? 12 : 0), lane, co1, co2);
                const float b1 = dpp<DPP_WAVE_SHL1, 0xF>(co1), b2 = dpp<DPP_WAVE_SHL1, 0xF>(co2);
                v[L - 1] += b1;
                if (L >= 2) v[L >= 2 ? L - 2 : 0] += b2;
                else v[L - 1] += dpp<DPP_WAVE_SHL1, 0xF>(b2);
            }
#pragma unroll
            for (int e = 0; e < 9; ++e) A[e] = ph[64 * 12 + e];
            ks_build<true>(A, Kw, lane);
            St y{0.f, 0.f, 0.f};
            R.template desc<1>(y, v);
            y = ks_carry<true>(y, Kw, lane);
            R.template desc<2>(y, v);
        } else {
            // periodic row: the cyclic carry scans of the 2-D kernel (x_rows), with
            // this level's cyclic-scan tables
            const int clast = (nx - 1) / L, slast = (nx - 1) % L;
            const float *qa = PERT + lev * S.per + ((long)row * 4 + (ADJ ? 2 : 0)) * kPerXEntries * 12;
            const float *qd = PERT + lev * S.per + ((long)row * 4 + (ADJ ? 3 : 1)) * kPerXEntries * 12;
            St saved{0.f, 0.f, 0.f};
            R.template asc<1, true>(x, v, slast, &saved);
            x = ks_carry<false>(x, Kw, lane);
            {
                float M[9];
                load_m3(qa + 65 * 12, M);
                St bw = saved;
                mat_acc(M, x, bw);
                const St b{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(bw.a), clast)),
                           __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bw.b), clast)),
                           __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bw.c), clast))};
                load_m3(qa + 64 * 12, M);
                St x0{0.f, 0.f, 0.f};
                mat_acc(M, b, x0);
                load_m3(qa + lane * 12, M);
                mat_acc(M, x0, x);
            }
            R.template asc<2>(x, v);
#pragma unroll
            for (int e = 0; e < 9; ++e) A[e] = ph[64 * 12 + e];
            ks_build<true>(A, Kw, lane);
            St y{0.f, 0.f, 0.f};
            R.template desc<1>(y, v);
            St out0;
            y = ks_carry<true>(y, Kw, lane, &out0);
            St xw{0.f, 0.f, 0.f};
            {
                float M[9];
                load_m3(qd + 64 * 12, M);
                mat_acc(M, out0, xw);
                load_m3(qd + lane * 12, M);
                mat_acc(M, xw, y);
            }
            R.template desc<2, true>(y, v, slast, lane == clast, xw);
        }
#pragma unroll
        for (int i = 0; i < L; ++i) stg[x0 + i] = v[i];
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        const Rsrc ro = make_rsrc(out + ln * plane + (long)row * nx, line_bytes);
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            if (it < nst) {
                const f4 q = *reinterpret_cast<const f4 *>(stg + 4 * lane + 256 * it);
                u32x4 w;
                w.x = __float_as_uint(q.x);
                w.y = __float_as_uint(q.y);
                w.z = __float_as_uint(q.z);
                w.w = __float_as_uint(q.w);
                __builtin_amdgcn_raw_buffer_store_b128(w, ro, (4 * lane + 256 * it) * 4, 0, kStreamStoreX);
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);   // the staging reads are done before the next line's writes
        __builtin_amdgcn_wave_barrier();
    }
}

// Batched form: one workgroup per work unit {item, row, group, groups}; the
// second pass of a V_H application reads the first pass's output (src_out).
// One launch serves every tile size of an occupancy class (x_batch_class):
// the class's largest tile sets the LDS staging area and the register budget,
// which the smaller tiles of the class fit without losing occupancy.
#define RF_XB_UNIT(Lv)                                                                                    \
    case Lv:                                                                                              \
        if constexpr (ALL ? x_batch_class(Lv) <= LMAX : x_batch_class(Lv) == LMAX)                        \
            x_rows<Lv, ADJ>(in, out, T, LM, PHI, nx, ny, nplanes, row, grp, groups, K, stg);              \
        break;

// ALL: the launch also serves the units of every smaller class (one x launch
// for the whole work list)
template <int LMAX, bool ADJ, bool ALL>
__global__ __launch_bounds__(64 * kXWaves, (LMAX <= 23 ? 3 : 2)) void k_rf3x_batch(
    const BatchEntry *__restrict__ E, const BatchUnit *__restrict__ U, int src_out)
{
    __shared__ float K[2 * 64 * kKs];
    __shared__ __align__(16) float stage[kXWaves][x_stage_floats<LMAX>()];
    const BatchUnit *up = U + blockIdx.x;
    const int item = uni(up->item);
    if (item < 0) return;
    const BatchEntry *e = E + item;
    const float *in = uni(src_out ? (const float *)e->out : e->in);
    float *out = uni(e->out);
    const float4 *T = uni(e->T[0]);
    const uint64_t *LM = uni(e->LM[0]);
    const float *PHI = uni(e->PHI[0]);
    const int nx = uni(e->nx), ny = uni(e->ny), nplanes = uni(e->nplanes);
    const int row = uni(up->a), grp = uni(up->b), groups = uni(up->c);
    float *stg = stage[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
    switch (tile_lx(nx)) {
        RF_XB_UNIT(1) RF_XB_UNIT(3) RF_XB_UNIT(5) RF_XB_UNIT(7) RF_XB_UNIT(9) RF_XB_UNIT(11) RF_XB_UNIT(13)
        RF_XB_UNIT(15) RF_XB_UNIT(17) RF_XB_UNIT(19) RF_XB_UNIT(21) RF_XB_UNIT(23) RF_XB_UNIT(25) RF_XB_UNIT(27)
        RF_XB_UNIT(29) RF_XB_UNIT(31) RF_XB_UNIT(33)
    default: break;
    }
}
#undef RF_XB_UNIT

// ======================================================================
// y direction: 16 waves per block of 64 columns; wave w owns rows
// [w*L, w*L + L), lane = column, and every lane carries P planes (P = 2 when
// L <= 45) so that each coefficient load serves P recurrences.  The local
// passes are dot products with precomputed K vectors; the chunk transfer
// matrices (per column, chunk and sweep) come from the coefficient block, and
// local end states pass between the waves through LDS.  Coefficients and K
// vectors are read one row at a time through a rolling window.  A workgroup
// takes a contiguous range of planes of its column block.  Row offsets are
// scalar buffer offsets, clamped to the grid: rows past the end are outside
// every segment (their input is masked off and they are never stored).
// ======================================================================
constexpr int kYWin = 2;

// One unit: planes pl0, pl0 + pst, .., pl0 + (P-1) pst of one column block, each
// lane one column of each plane.  phi: [2][16][64 * 9] in LDS (filled by y_planes); bsh: LDS
// array of [2][16][2][64 * 3] floats, used here as [2][16][P][64 * 3].
// KY: the local passes' K vectors [4 kinds][ny][nx][3].
template <int L, bool ADJ, int P, bool END = false>
__device__ __forceinline__ void y_unit(const float *in, float *out, const float4 *T, const float *KY,
                                       const uint64_t *LM, int nx_, int ny_, int blk, int pl0,
                                       float (*phi)[kYWaves][kYCols * 9], float *bsh_raw,
                                       const float *ENDT = nullptr, float *xch = nullptr, int pst = 1)
{
    auto bsh = reinterpret_cast<float (*)[kYWaves][P][kYCols * 3]>(bsh_raw);
    constexpr int LB = (L + 7) / 8;   // 8-row mask blocks per chunk
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = blk * kYCols + lane;
    const long plane = (long)nx_ * ny_;
    const int lys = lmy_stride(L);
    const uint64_t *lm = LM + (long)blk * kLaneMasks * lys + 8;   // entry r = row r
    // byte offset of my column in the field; columns past the grid get 2^29, past
    // every table (the y kernels need nx * ny < 2^27), so loads read 0 and stores
    // are dropped.  The coefficient (16 B) and K (12 B) offsets are 4x and 3x this,
    // formed inside each pass so that only this one stays live.
    const uint32_t cb = col < nx_ ? (uint32_t)col * 4u : 0x20000000u;
    auto col_off = [&](uint32_t mul) {
        uint32_t o = cb * mul;
        asm volatile("" : "+v"(o));
        return o;
    };
    const Rsrc rt = make_rsrc(T, (uint32_t)(plane * 16));
    {
        // opaque per unit: keeps the per-row offsets and conditions out of the
        // enclosing loop's preheader (hoisted, they would be live in SGPRs across it)
        const int r0 = fresh_int(w * L), ny = fresh_int(ny_), rowb = fresh_int(nx_ * 4), nx = fresh_int(nx_);
        float v[P][L];
        float co1[P], co2[P];   // exact ends: corrections of the two rows above my chunk
#pragma unroll
        for (int p = 0; p < P; ++p) co1[p] = co2[p] = 0.f;
        const uint64_t *ep_end = lm + 3 * lys + r0;
        Rsrc ri[P], ro[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            ri[p] = make_rsrc(in + (long)(pl0 + p * pst) * plane, (uint32_t)(plane * 4));
            ro[p] = make_rsrc(out + (long)(pl0 + p * pst) * plane, (uint32_t)(plane * 4));
        }
        {
            // running row offset (a chain, so the compiler keeps one of them live)
            const int last = (ny - 1) * rowb;
            int roff = fresh_int(min(r0, ny - 1) * rowb);
#pragma unroll
            for (int i = 0; i < L; ++i) {
#pragma unroll
                for (int p = 0; p < P; ++p)
                    v[p][i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ri[p], cb, roff, kStreamLoadY));
                roff = fresh_int(min(roff + rowb, last));
            }
        }
        // local pass: the chunk's end state from a zero state is the dot product of
        // its inputs with the K vectors of this sweep (resets are folded into K, the
        // forward causal K also holds beta).  The first one masks the input to sea
        // points as the rows arrive.
        auto local = [&](St *x, auto DC) {
            constexpr bool desc = decltype(DC)::value;
            constexpr bool first = !desc;
            const int kind = (ADJ ? 2 : 0) + (desc ? 1 : 0);
            const Rsrc rk = make_rsrc(KY + (long)kind * plane * 3, (uint32_t)(plane * 12));
            const uint64_t *sp = lm + 2 * lys + r0;
            const int krow = nx * 12, klast = (ny - 1) * krow;
            const uint32_t cbk = col_off(3);
            int cur = fresh_int(r0 * krow);
            auto kload = [&]() -> u32x3 {
                const u32x3 z = __builtin_amdgcn_raw_buffer_load_b96(rk, cbk, min(cur, klast), 0);
                cur = fresh_int(cur + krow);
                return z;
            };
            u32x3 win[kYWin];
#pragma unroll
            for (int q = 0; q < kYWin; ++q) win[q] = kload();
#pragma unroll
            for (int b = 0; b < LB; ++b) {
                u32x16 sm;
                if (first) sm = sload16(sp + 8 * b);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = 8 * b + q;
                    if (i >= L) continue;
                    const u32x3 k = win[i % kYWin];
                    if (i + kYWin < L) win[i % kYWin] = kload();
                    const float k0 = __uint_as_float(k.x), k1 = __uint_as_float(k.y), k2 = __uint_as_float(k.z);
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        if (first) v[p][i] = zero_if(v[p][i], m64_of(sm, q));
                        x[p].a = fmaf(k0, v[p][i], x[p].a);
                        x[p].b = fmaf(k1, v[p][i], x[p].b);
                        x[p].c = fmaf(k2, v[p][i], x[p].c);
                    }
                    mem_fence_compiler();   // keep the window's loads from being hoisted further
                }
            }
        };
        // rerun over the chunk for all P planes from the true incoming state, output
        // into v; the last pass (descending) applies the output sea mask and stores
        // each row as it is produced.
        auto pass = [&](St *x, auto DC, auto MC) {
            constexpr bool desc = decltype(DC)::value;
            constexpr int mode = decltype(MC)::value;
            static_assert(mode == 2, "local passes use the K vectors");
            // ascending uses FRESET (forward: before the step) or BRESET (adjoint: after);
            // descending uses BRESET (forward) or FRESET (adjoint)
            const uint64_t *rp = lm + ((ADJ ? !desc : desc) ? lys : 0) + r0;
            const uint64_t *sp = lm + 2 * lys + r0;
            // byte offset of the next row to fetch, a chain through opaque values so
            // that the offsets are formed one at a time; clamped at the last row
            const int crow = nx * 16, clast = (ny - 1) * crow;
            const uint32_t cbt = col_off(4);
            int cur = fresh_int((desc ? r0 + L - 1 : r0) * crow);
            auto cload = [&]() -> u32x4 {
                const u32x4 z = __builtin_amdgcn_raw_buffer_load_b128(rt, cbt, min(cur, clast), 0);
                cur = fresh_int(cur + (desc ? -crow : crow));
                return z;
            };
            constexpr bool last = desc;
            const int lim = ny * rowb;
            int soff = fresh_int((r0 + L - 1) * rowb);   // store offset of the current row (last pass)
            u32x4 win[kYWin];
#pragma unroll
            for (int q = 0; q < kYWin; ++q) win[q] = cload();
#pragma unroll
            for (int bb = 0; bb < LB; ++bb) {
                const int b = desc ? LB - 1 - bb : bb;
                const u32x16 m = sload16(rp + 8 * b);
                u32x16 sm;
                if (last) sm = sload16(sp + 8 * b);
#pragma unroll
                for (int qq = 0; qq < 8; ++qq) {
                    const int q = desc ? 7 - qq : qq;
                    const int i = 8 * b + q;
                    if (i >= L) continue;
                    const int ii = desc ? L - 1 - i : i;   // step number within the pass
                    const u32x4 c = win[ii % kYWin];
                    if (ii + kYWin < L) win[ii % kYWin] = cload();
                    const float bt = __uint_as_float(c.x), gm = __uint_as_float(c.y);
                    const float c2 = __uint_as_float(c.z), c3 = __uint_as_float(c.w);
                    const uint64_t mm = m64_of(m, q);
                    // exact ends (ascending pass): lanes at a segment end load the row's map
                    const uint64_t em = (END && !desc) ? ep_end[i] : 0;
                    float n[9];
                    const bool at_end = em != 0 && ((em >> lane) & 1);
                    if (at_end) {
                        const float *N = ENDT + ((long)(r0 + i) * nx + col) * 36 + (ADJ ? 12 : 0);
#pragma unroll
                        for (int e = 0; e < 9; ++e) n[e] = N[e];
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        float o;
                        St sn;
                        if (!ADJ) {   // causal input beta_i s_i; the anti-causal one is prescaled
                            st_reset(x[p], mm);
                            fwd_step(x[p], desc ? v[p][i] : bt * v[p][i], gm, c2, c3);
                            o = x[p].a;
                            sn = x[p];
                        } else {
                            o = adj_step<mode == 2>(x[p], v[p][i], bt, gm, c2, c3);
                            sn = x[p];
                            st_reset(x[p], mm);
                        }
                        // forward ascending output: beta_i u_i, the anti-causal input
                        if (mode == 2) v[p][i] = desc ? zero_if(o, m64_of(sm, q)) : (ADJ ? o : bt * o);
                        if (END && !desc && at_end) {
                            // the anti-causal inputs of this row and the two above gain N (state)
                            const float r0 = fmaf(n[0], sn.a, fmaf(n[1], sn.b, n[2] * sn.c));
                            const float r1 = fmaf(n[3], sn.a, fmaf(n[4], sn.b, n[5] * sn.c));
                            const float r2 = fmaf(n[6], sn.a, fmaf(n[7], sn.b, n[8] * sn.c));
                            v[p][i] += r0;
                            if (i >= 1) v[p][i >= 1 ? i - 1 : 0] += r1;
                            else co1[p] += r1;
                            if (i >= 2) v[p][i >= 2 ? i - 2 : 0] += r2;
                            else if (i == 1) co1[p] += r2;
                            else co2[p] += r2;
                        }
                    }
                    if (last) {
                        if (soff < lim) {   // rows past the grid are not stored
#pragma unroll
                            for (int p = 0; p < P; ++p)
                                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[p][i]), ro[p], cb, soff, kStreamStoreY);
                        }
                        soff = fresh_int(soff - rowb);
                    }
                    mem_fence_compiler();   // keep the window's loads from being hoisted further
                }
            }
        };
        // local pass, chain over the chunks before mine, rerun with the true state
        auto sweep = [&](auto DC) {
            constexpr bool desc = decltype(DC)::value;
            constexpr int sw = desc ? 1 : 0;
            St x[P];
#pragma unroll
            for (int p = 0; p < P; ++p) x[p] = St{0.f, 0.f, 0.f};
            local(x, DC);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                bsh[sw][w][p][lane * 3] = x[p].a;
                bsh[sw][w][p][lane * 3 + 1] = x[p].b;
                bsh[sw][w][p][lane * 3 + 2] = x[p].c;
            }
            __syncthreads();
            // chain over the chunks before mine, nearest last: c <- Phi_k c + b_k
            // (Phi_k read once for all planes)
            St c[P];
#pragma unroll
            for (int p = 0; p < P; ++p) c[p] = St{0.f, 0.f, 0.f};
            const int k_lo = desc ? w + 1 : 0, k_hi = desc ? kYWaves : w;
            for (int kk = k_lo; kk < k_hi; ++kk) {
                const int k = desc ? k_hi - 1 - (kk - k_lo) : kk;
                float A[9];
#pragma unroll
                for (int e = 0; e < 9; ++e) A[e] = phi[sw][k][lane * 9 + e];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    St n{bsh[sw][k][p][lane * 3], bsh[sw][k][p][lane * 3 + 1], bsh[sw][k][p][lane * 3 + 2]};
                    mat_acc(A, c[p], n);
                    c[p] = n;
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) x[p] = c[p];
            pass(x, DC, std::integral_constant<int, 2>{});
        };
        sweep(std::false_type{});
        if (END) {
            // corrections of the rows above my chunk go to the waves that hold them
            float(*corr)[P][2][kYCols] = reinterpret_cast<float(*)[P][2][kYCols]>(xch);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                corr[w][p][0][lane] = co1[p];   // row r0 - 1
                corr[w][p][1][lane] = co2[p];   // row r0 - 2
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (w + 1 < kYWaves) {
                    v[p][L - 1] += corr[w + 1][p][0][lane];
                    if (L >= 2) v[p][L >= 2 ? L - 2 : 0] += corr[w + 1][p][1][lane];
                }
                if (L == 1 && w + 2 < kYWaves) v[p][L - 1] += corr[w + 2][p][1][lane];
            }
        }
        sweep(std::true_type{});
    }
}

// Planes [pa, pb) of one column block: units of two planes (one when L > 45),
// and a one-plane unit for an odd count, run after single_after two-plane
// units (varied across workgroups, so that they do not all reach their memory
// phases together).
template <int L, bool ADJ, bool END = false>
__device__ __forceinline__ void y_planes(const float *in, float *out, const float4 *T, const float *KY,
                                         const uint64_t *LM, const float *PHI, int nx, int ny, int blk, int pa, int pb,
                                         int single_after, float (*phi)[kYWaves][kYCols * 9], float *bsh,
                                         const float *ENDT = nullptr, float *xch = nullptr)
{
    constexpr int PM = y_planes_per_lane(L);
    {
        const int k0 = ADJ ? 2 : 0;
        for (int e = threadIdx.x; e < 2 * kYWaves * kYCols; e += 64 * kYWaves) {
            const int sw = e / (kYWaves * kYCols), rest = e % (kYWaves * kYCols);
            const float *src = PHI + (((long)blk * 4 + k0 + sw) * kYWaves * kYCols + rest) * 12;
#pragma unroll
            for (int q = 0; q < 9; ++q) phi[sw][rest / kYCols][(rest % kYCols) * 9 + q] = src[q];
        }
    }
    __syncthreads();
    for (int k = 0; pa < pb; ++k) {
        // an odd count leaves one one-plane unit: it runs after single_after pairs
        const bool single = PM == 1 || pb - pa == 1 || (((pb - pa) & 1) && k >= single_after);
        if (single) {
            y_unit<L, ADJ, 1, END>(in, out, T, KY, LM, nx, ny, blk, pa, phi, bsh, ENDT, xch);
            pa += 1;
        } else {
            y_unit<L, ADJ, PM, END>(in, out, T, KY, LM, nx, ny, blk, pa, phi, bsh, ENDT, xch);
            pa += PM;
        }
        __syncthreads();   // bsh is rewritten by the next unit
    }
}

// Workgroup (column block, slot): slot j of S takes planes [j n / S, (j+1) n / S),
// its one-plane unit (odd counts) after (j + 2) % 3 two-plane units.
template <int L, bool ADJ, bool END>
__global__ __launch_bounds__(64 * kYWaves, 1) void k_rf3y(const float *in, float *out, const float4 *T,
                                                         const float *KY, const uint64_t *__restrict__ LM,
                                                         const float *__restrict__ PHI, int nx, int ny,
                                                         int nplanes, int nblk, int nslot,
                                                         const float *__restrict__ ENDT)
{
    __shared__ float phi[2][kYWaves][kYCols * 9];
    __shared__ float bsh[2 * kYWaves * 2 * kYCols * 3];
    __shared__ float xch[END ? kYWaves * 2 * 2 * kYCols : 1];   // exact ends: corrections between waves
    // XCD-aware order: all slots of a column block run on one XCD (shared L2)
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int blk = (slot / nslot) * 8 + xcd, j = slot % nslot;
    if (blk >= nblk) return;
    const int pa = (int)((long)j * nplanes / nslot), pb = (int)((long)(j + 1) * nplanes / nslot);
    y_planes<L, ADJ, END>(in, out, T, KY, LM, PHI, nx, ny, blk, pa, pb, (j + 2) % 3, phi, bsh, ENDT, xch);
}

// Depth-dependent tables (LevTabs): the units of one column block are (field
// pair, level): the planes of fields 2q and 2q + 1 at one level share that
// level's tables, so a lane carries both (one plane for the last of an odd field
// count, or when L > 45).  A workgroup takes units [ua, ub) of its column block;
// the level's chunk transfer matrices go into LDS before each unit.
template <int L, bool ADJ, bool END>
__global__ __launch_bounds__(64 * kYWaves, 1) void k_rf3y_lev(const float *in, float *out, const float4 *T,
                                                             const float *KY, const uint64_t *__restrict__ LM,
                                                             const float *__restrict__ PHI, int nx, int ny,
                                                             int nfields, int nunits, int nblk, int nslot,
                                                             LevTabs S, const float *__restrict__ ENDT)
{
    constexpr int PM = y_planes_per_lane(L);
    __shared__ float phi[2][kYWaves][kYCols * 9];
    __shared__ float bsh[2 * kYWaves * 2 * kYCols * 3];
    __shared__ float xch[END ? kYWaves * 2 * 2 * kYCols : 1];
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int blk = (slot / nslot) * 8 + xcd, j = slot % nslot;
    if (blk >= nblk) return;
    const int ua = (int)((long)j * nunits / nslot), ub = (int)((long)(j + 1) * nunits / nslot);
    const int k0 = ADJ ? 2 : 0;
    for (int u = ua; u < ub; ++u) {
        const int lev = u % S.nlev, f0 = (u / S.nlev) * PM;
        const int p = f0 * S.nlev + lev;
        const bool two = PM == 2 && f0 + 1 < nfields;
        const float *ph = PHI + lev * S.phi;
        for (int e = threadIdx.x; e < 2 * kYWaves * kYCols; e += 64 * kYWaves) {
            const int sw = e / (kYWaves * kYCols), rest = e % (kYWaves * kYCols);
            const float *src = ph + (((long)blk * 4 + k0 + sw) * kYWaves * kYCols + rest) * 12;
#pragma unroll
            for (int q = 0; q < 9; ++q) phi[sw][rest / kYCols][(rest % kYCols) * 9 + q] = src[q];
        }
        __syncthreads();
        if (two)
            y_unit<L, ADJ, PM, END>(in, out, T + lev * S.t, KY + lev * S.ky, LM + lev * S.lm, nx, ny, blk, p, phi,
                                    bsh, END ? ENDT + lev * S.end : nullptr, xch, S.nlev);
        else
            y_unit<L, ADJ, 1, END>(in, out, T + lev * S.t, KY + lev * S.ky, LM + lev * S.lm, nx, ny, blk, p, phi,
                                   bsh, END ? ENDT + lev * S.end : nullptr, xch);
        __syncthreads();   // phi, bsh and xch are rewritten for the next unit
    }
}

// Batched form: one workgroup per work unit {item, column block, first and end
// plane}.  The tile size follows from the item's ny, so one launch serves the
// units of every tile size (the work list puts the largest tiles first and the
// small units fill the last round).
#define RF_YB_UNIT(Lv)                                                                                    \
    case Lv:                                                                                              \
        y_planes<Lv, ADJ>(in, out, T, KY, LM, PHI, nx, ny, blk, pa, pb, 1 << 30, phi, bsh);               \
        break;

template <bool ADJ>
__global__ __launch_bounds__(64 * kYWaves, 1) void k_rf3y_batch(const BatchEntry *__restrict__ E,
                                                               const BatchUnit *__restrict__ U, int src_out)
{
    __shared__ float phi[2][kYWaves][kYCols * 9];
    __shared__ float bsh[2 * kYWaves * 2 * kYCols * 3];
    const BatchUnit *up = U + blockIdx.x;
    const int item = uni(up->item);
    if (item < 0) return;
    const BatchEntry *e = E + item;
    const float *in = uni(src_out ? (const float *)e->out : e->in);
    float *out = uni(e->out);
    const float4 *T = uni(e->T[1]);
    const float *KY = uni(e->KY);
    const uint64_t *LM = uni(e->LM[1]);
    const float *PHI = uni(e->PHI[1]);
    const int nx = uni(e->nx), ny = uni(e->ny), blk = uni(up->a), pa = uni(up->b), pb = uni(up->c);
    switch (tile_ly(ny)) {
        RF_YB_UNIT(1) RF_YB_UNIT(2) RF_YB_UNIT(3) RF_YB_UNIT(4) RF_YB_UNIT(6) RF_YB_UNIT(8) RF_YB_UNIT(12)
        RF_YB_UNIT(16) RF_YB_UNIT(20) RF_YB_UNIT(24) RF_YB_UNIT(28) RF_YB_UNIT(32) RF_YB_UNIT(36) RF_YB_UNIT(40)
        RF_YB_UNIT(45) RF_YB_UNIT(48) RF_YB_UNIT(56) RF_YB_UNIT(64)
    default: break;
    }
}
#undef RF_YB_UNIT

// ---------------------------------------------------------------- setup
// 3x3 transfer matrix of one chunk of n points, FP64 from the FP32 table.
// kind 0 forward ascending, 1 forward descending, 2 adjoint ascending,
// 3 adjoint descending.  Forward kinds zero the state before the step at a
// segment start (0) / end (1); adjoint kinds after the step at a segment end
// (2) / start (3).  cf(i), cd(i): coefficients and code of chunk point i
// (ascending position).
template <class CF, class CD>
__device__ void chunk_transfer_d(int kind, int n, CF cf, CD cd, double *A)
{
    const bool desc = kind & 1;
    const uint8_t flag = kind == 0 ? CODE_FRESET : kind == 1 ? CODE_BRESET : kind == 2 ? CODE_BRESET : CODE_FRESET;
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
}
template <class CF, class CD>
__device__ void chunk_transfer(int kind, int n, CF cf, CD cd, float *dst)
{
    double A[9];
    chunk_transfer_d(kind, n, cf, cd, A);
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

// y kernel's local passes: K vectors.  The state a sweep leaves at the end of
// chunk w, from a zero state, is sum_i K_i v_i over the chunk's rows, with K_i
// the response of that end state to a unit input at row i: the state right
// after row i's step, carried through the later steps of the chunk (resets
// included: a reset after row i zeroes K_i).  Forward causal: the input is s
// and the step injects (beta, beta, 0); forward anti-causal: the input is
// beta u, injection (1, 1, 0); adjoint: injection (1 - gamma, -c2, -c3), then
// the reset after the step.  Kinds and reset flags as in chunk_transfer; rows
// past the grid reset and carry nothing.  KY[kind][r][col][3], FP64 from the
// FP32 table; one thread per (column, chunk, kind).
__global__ void k_kvec_y(const float4 *__restrict__ T, const uint8_t *__restrict__ code, float *__restrict__ KY,
                         int nx, int ny, int L, int nblk)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nblk * kYCols * kYWaves * 4) return;
    const int j = (int)(t % kYCols);
    const int w = (int)((t / kYCols) % kYWaves);
    const int kind = (int)((t / (kYCols * kYWaves)) % 4);
    const int blk = (int)(t / (kYCols * kYWaves * 4));
    const int col = blk * kYCols + j;
    if (col >= nx) return;
    const bool desc = kind & 1, adj = kind >= 2;
    const uint8_t flag = kind == 0 ? CODE_FRESET : kind == 1 ? CODE_BRESET : kind == 2 ? CODE_BRESET : CODE_FRESET;
    double P[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};   // steps after the current one, composed
    for (int k = L - 1; k >= 0; --k) {             // sweep steps, last first
        const int i = desc ? L - 1 - k : k;
        const int r = w * L + i;
        const bool in = r < ny;
        const float4 c = in ? T[(long)r * nx + col] : make_float4(0.f, 0.f, 0.f, 0.f);
        const bool rs = in ? (code[(long)r * nx + col] & flag) != 0 : true;
        const double bt = c.x, gm = c.y, c2 = c.z, c3 = c.w;
        double u[3];
        if (!adj) {
            const double s = desc ? 1.0 : bt;
            u[0] = s; u[1] = s; u[2] = 0.0;
        } else {
            u[0] = rs ? 0.0 : 1.0 - gm; u[1] = rs ? 0.0 : -c2; u[2] = rs ? 0.0 : -c3;
        }
        if (in) {
            float *dst = KY + (((long)kind * ny + r) * nx + col) * 3;
#pragma unroll
            for (int e = 0; e < 3; ++e) dst[e] = (float)(P[3 * e] * u[0] + P[3 * e + 1] * u[1] + P[3 * e + 2] * u[2]);
        }
        // P <- P * (this step's map with zero input); a reset makes it zero
        double M[9];
        if (rs) {
            for (int e = 0; e < 9; ++e) M[e] = 0.0;
        } else if (!adj) {   // (p, d1, d2) -> (p + t, t, d1), t = -gm p - c2 d1 - c3 d2
            const double m[9] = {1 - gm, -c2, -c3, -gm, -c2, -c3, 0, 1, 0};
            for (int e = 0; e < 9; ++e) M[e] = m[e];
        } else {             // (a, b, c) -> (a - gm u, c - c2 u, -c3 u), u = a + b
            const double m[9] = {1 - gm, -gm, 0, -c2, -c2, 1, -c3, -c3, 0};
            for (int e = 0; e < 9; ++e) M[e] = m[e];
        }
        double N[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) N[3 * a + b] = P[3 * a] * M[b] + P[3 * a + 1] * M[3 + b] + P[3 * a + 2] * M[6 + b];
        for (int e = 0; e < 9; ++e) P[e] = N[e];
    }
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

// periodic rows, x kernel's cyclic scan: PER[row][kind][kPerXEntries][12], one
// thread per (row, kind), FP64 products of FP64 chunk transfers (see rf3_internal.h)
__device__ inline void m3_mul_d(const double *A, const double *B, double *C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
__global__ void k_per_x(const float4 *__restrict__ T, const uint8_t *__restrict__ code, float *__restrict__ PER,
                        int nx, int ny, int L)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)ny * 4) return;
    const int row = (int)(t / 4), kind = (int)(t % 4);
    const int clast = (nx - 1) / L, slast = (nx - 1) % L;
    const float4 *tr = T + (long)row * nx;
    const uint8_t *cr = code + (long)row * nx;
    float *dst = PER + t * kPerXEntries * 12;
    auto chunk = [&](int c, int n, double *A) {
        auto cf = [&](int i) -> float4 {
            const int x = c * L + i;
            return x < nx ? tr[x] : make_float4(0.f, 0.f, 0.f, 0.f);
        };
        auto cd = [&](int i) -> uint8_t {
            const int x = c * L + i;
            return x < nx ? cr[x] : (uint8_t)(CODE_FRESET | CODE_BRESET);
        };
        chunk_transfer_d(kind, n, cf, cd, A);
    };
    auto put = [&](int e, const double *A) {
        for (int q = 0; q < 9; ++q) dst[e * 12 + q] = A ? (float)A[q] : 0.f;
        dst[e * 12 + 9] = dst[e * 12 + 10] = dst[e * 12 + 11] = 0.f;
    };
    for (int e = 0; e < kPerXEntries; ++e) put(e, nullptr);
    const double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double P[9], A[9], N[9], cyc[9];
    for (int e = 0; e < 9; ++e) P[e] = I[e];
    if (!(kind & 1)) {   // ascending: P_c = Phi_{c-1} .. Phi_0
        for (int c = 0; c <= clast; ++c) {
            put(c, P);
            if (c < clast) {
                chunk(c, L, A);
                m3_mul_d(A, P, N);
                for (int e = 0; e < 9; ++e) P[e] = N[e];
            }
        }
        chunk(clast, slast + 1, A);
        put(65, A);
        m3_mul_d(A, P, cyc);
    } else {             // descending: P_c = Phi_{c+1} .. Phi_{c_last - 1} Phi_last, P_{c_last} = I
        put(clast, I);
        chunk(clast, slast + 1, P);
        for (int c = clast - 1; c >= 0; --c) {
            put(c, P);
            chunk(c, L, A);
            m3_mul_d(A, P, N);
            for (int e = 0; e < 9; ++e) P[e] = N[e];
        }
        for (int e = 0; e < 9; ++e) cyc[e] = P[e];
    }
    // W = (I - cyc)^-1 (adjugate)
    double B[9];
    for (int e = 0; e < 9; ++e) B[e] = I[e] - cyc[e];
    const double c00 = B[4] * B[8] - B[5] * B[7], c01 = B[5] * B[6] - B[3] * B[8], c02 = B[3] * B[7] - B[4] * B[6];
    const double det = B[0] * c00 + B[1] * c01 + B[2] * c02;
    const double W[9] = {c00 / det, (B[2] * B[7] - B[1] * B[8]) / det, (B[1] * B[5] - B[2] * B[4]) / det,
                         c01 / det, (B[0] * B[8] - B[2] * B[6]) / det, (B[2] * B[3] - B[0] * B[5]) / det,
                         c02 / det, (B[1] * B[6] - B[0] * B[7]) / det, (B[0] * B[4] - B[1] * B[3]) / det};
    put(64, W);
}

// ---------------------------------------------------------------- dispatch
// compute units of the current device (cached per device)
static int cu_count()
{
    static int cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// groups per row for the x kernel (workgroups sharing one row's planes): more
// only while the rows alone give fewer than two workgroups per CU (a
// workgroup's setup, the row's coefficients and scan matrices, is paid once
// per group), at least two lines per wave, at most gmax
int x_groups(int ny, int nplanes, int gmax)
{
    const long target = 2L * cu_count();
    int groups = 1;
    while (groups * 2 <= gmax && (long)((ny + 7) / 8) * 8 * groups < target && groups * kXWaves * 2 <= nplanes)
        groups *= 2;
    return groups;
}

template <int L, bool ADJ>
static hipError_t launch_x(const float *in, float *out, const float4 *T, const uint64_t *LM, const float *PHI,
                           int nx, int ny, int nplanes, const float *PERT, const float *ENDT, const LevTabs *lv,
                           hipStream_t st)
{
    if (lv) {   // depth-dependent tables: one wave per (level, row)
        if ((PERT && ENDT) || lv->nlev < 1 || nplanes % lv->nlev) return hipErrorNotSupported;
        const unsigned nb = (unsigned)(((long)lv->nlev * ny + kXWaves - 1) / kXWaves);
        const int nf = nplanes / lv->nlev;
        if (PERT)
            k_rf3x_lev<L, ADJ, true, false><<<nb, 64 * kXWaves, 0, st>>>(in, out, T, LM, PHI, nx, ny, nf, *lv, PERT,
                                                                         nullptr);
        else if (ENDT)
            k_rf3x_lev<L, ADJ, false, true><<<nb, 64 * kXWaves, 0, st>>>(in, out, T, LM, PHI, nx, ny, nf, *lv,
                                                                         nullptr, ENDT);
        else
            k_rf3x_lev<L, ADJ, false, false><<<nb, 64 * kXWaves, 0, st>>>(in, out, T, LM, PHI, nx, ny, nf, *lv,
                                                                          nullptr, nullptr);
        return hipGetLastError();
    }
    const int groups = x_groups(ny, nplanes, 8);
    const unsigned nb = (unsigned)(((ny + 7) / 8) * 8 * groups);
    if (PERT && ENDT) return hipErrorNotSupported;   // periodic rows with exact ends: sequential kernels
    if (PERT)
        k_rf3x<L, ADJ, true, false><<<nb, 64 * kXWaves, 0, st>>>(in, out, T, LM, PHI, nx, ny, nplanes, groups, PERT,
                                                                 nullptr);
    else if (ENDT)
        k_rf3x<L, ADJ, false, true><<<nb, 64 * kXWaves, 0, st>>>(in, out, T, LM, PHI, nx, ny, nplanes, groups,
                                                                 nullptr, ENDT);
    else
        k_rf3x<L, ADJ, false, false><<<nb, 64 * kXWaves, 0, st>>>(in, out, T, LM, PHI, nx, ny, nplanes, groups,
                                                                  nullptr, nullptr);
    return hipGetLastError();
}


// time of a one-plane y unit relative to a two-plane one with every CU busy
// (measured on 1440 x 720 grids: the memory phases dominate both)
constexpr double kYSingleCost = 0.85;

// cost of a y workgroup with n planes, in two-plane units
static double y_range_cost(int n, int pm)
{
    return pm == 2 ? n / 2 + (n & 1) * kYSingleCost : n;
}

template <int L, bool ADJ>
static hipError_t launch_y(const float *in, float *out, const float4 *T, const float *KY, const uint64_t *LM,
                           const float *PHI, int nx, int ny, int nplanes, const float *ENDT, const LevTabs *lv,
                           hipStream_t st)
{
    static_assert(y_planes_per_lane(L) == 1 || y_planes_per_lane(L) == 2, "planes per lane");
    if (lv && (lv->nlev < 1 || nplanes % lv->nlev)) return hipErrorNotSupported;
    // depth-dependent tables: units of (field pair, level), counted as one-plane units here
    const int nfields = lv ? nplanes / lv->nlev : 0;
    const int nunits = lv ? lv->nlev * ((nfields + y_planes_per_lane(L) - 1) / y_planes_per_lane(L)) : 0;
    const int PM = lv ? 1 : y_planes_per_lane(L);
    const int nwork = lv ? nunits : nplanes;
    const int nblk = (nx + kYCols - 1) / kYCols;
    // slots (workgroups) per column block: one workgroup per CU at a time, so
    // minimise (rounds of workgroups) x (cost of the largest plane range)
    const int cus = cu_count(), nb8 = ((nblk + 7) / 8) * 8;
    int best = 1;
    double best_cost = -1;
    for (int sl = 1; sl <= nwork; ++sl) {
        const long rounds = ((long)nb8 * sl + cus - 1) / cus;
        const double cost = rounds * y_range_cost((nwork + sl - 1) / sl, PM);
        if (best_cost < 0 || cost < best_cost - 1e-9) { best_cost = cost; best = sl; }
    }
    const unsigned nb = (unsigned)(nb8 * best);
    if (lv) {
        if (ENDT)
            k_rf3y_lev<L, ADJ, true><<<nb, 64 * kYWaves, 0, st>>>(in, out, T, KY, LM, PHI, nx, ny, nfields, nunits,
                                                                  nblk, best, *lv, ENDT);
        else
            k_rf3y_lev<L, ADJ, false><<<nb, 64 * kYWaves, 0, st>>>(in, out, T, KY, LM, PHI, nx, ny, nfields, nunits,
                                                                   nblk, best, *lv, nullptr);
        return hipGetLastError();
    }
    if (ENDT)
        k_rf3y<L, ADJ, true><<<nb, 64 * kYWaves, 0, st>>>(in, out, T, KY, LM, PHI, nx, ny, nplanes, nblk, best, ENDT);
    else
        k_rf3y<L, ADJ, false><<<nb, 64 * kYWaves, 0, st>>>(in, out, T, KY, LM, PHI, nx, ny, nplanes, nblk, best,
                                                          nullptr);
    return hipGetLastError();
}

#define RF_X_CASE(Lv)                                                                                     \
    case Lv:                                                                                              \
        return adj ? launch_x<Lv, true>(in, out, T, LM, PHI, nx, ny, nplanes, PERT, ENDT, lv, st)         \
                   : launch_x<Lv, false>(in, out, T, LM, PHI, nx, ny, nplanes, PERT, ENDT, lv, st);
#define RF_Y_CASE(Lv)                                                                                     \
    case Lv:                                                                                              \
        return adj ? launch_y<Lv, true>(in, out, T, KY, LM, PHI, nx, ny, nplanes, ENDT, lv, st)           \
                   : launch_y<Lv, false>(in, out, T, KY, LM, PHI, nx, ny, nplanes, ENDT, lv, st);

hipError_t fast_rf3_x(const float *in, float *out, const float4 *T, const uint64_t *LM, const float *PHI, int lx,
                      int nx, int ny, int nplanes, bool adj, const float *PERT, const float *ENDT, const LevTabs *lv,
                      hipStream_t st)
{
    switch (lx) {
        RF_X_CASE(1) RF_X_CASE(3) RF_X_CASE(5) RF_X_CASE(7) RF_X_CASE(9) RF_X_CASE(11) RF_X_CASE(13)
        RF_X_CASE(15) RF_X_CASE(17) RF_X_CASE(19) RF_X_CASE(21) RF_X_CASE(23) RF_X_CASE(25) RF_X_CASE(27)
        RF_X_CASE(29) RF_X_CASE(31) RF_X_CASE(33)
    default: return hipErrorNotSupported;
    }
}

hipError_t fast_rf3_y(const float *in, float *out, const float4 *T, const float *KY, const uint64_t *LM,
                      const float *PHI, int ly, int nx, int ny, int nplanes, bool adj, const float *ENDT,
                      const LevTabs *lv, hipStream_t st)
{
    // scalar row offsets into the coefficient table are 32-bit
    if ((long)nx * ny * 16 >= (1L << 31)) return hipErrorNotSupported;
    switch (ly) {
        RF_Y_CASE(1) RF_Y_CASE(2) RF_Y_CASE(3) RF_Y_CASE(4) RF_Y_CASE(6) RF_Y_CASE(8) RF_Y_CASE(12)
        RF_Y_CASE(16) RF_Y_CASE(20) RF_Y_CASE(24) RF_Y_CASE(28) RF_Y_CASE(32) RF_Y_CASE(36) RF_Y_CASE(40)
        RF_Y_CASE(45) RF_Y_CASE(48) RF_Y_CASE(56) RF_Y_CASE(64)
    default: return hipErrorNotSupported;
    }
}

template <int LMAX, bool ALL>
static void launch_x_batch(const BatchEntry *E, const BatchUnit *U, int nunits, bool adj, bool src_out,
                           hipStream_t st)
{
    if (adj) k_rf3x_batch<LMAX, true, ALL><<<nunits, 64 * kXWaves, 0, st>>>(E, U, src_out);
    else k_rf3x_batch<LMAX, false, ALL><<<nunits, 64 * kXWaves, 0, st>>>(E, U, src_out);
}

hipError_t fast_rf3_x_batch(const BatchEntry *E, const BatchUnit *U, int nunits, int cls, bool adj, bool src_out,
                            bool all_classes, hipStream_t st)
{
    if (nunits <= 0) return hipSuccess;
    switch (cls) {
    case 3: launch_x_batch<3, false>(E, U, nunits, adj, src_out, st); break;   // the smallest class: no others
    case 11:
        if (all_classes) launch_x_batch<11, true>(E, U, nunits, adj, src_out, st);
        else launch_x_batch<11, false>(E, U, nunits, adj, src_out, st);
        break;
    case 23:
        if (all_classes) launch_x_batch<23, true>(E, U, nunits, adj, src_out, st);
        else launch_x_batch<23, false>(E, U, nunits, adj, src_out, st);
        break;
    case 33:
        if (all_classes) launch_x_batch<33, true>(E, U, nunits, adj, src_out, st);
        else launch_x_batch<33, false>(E, U, nunits, adj, src_out, st);
        break;
    default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

hipError_t fast_rf3_y_batch(const BatchEntry *E, const BatchUnit *U, int nunits, bool adj, bool src_out,
                            hipStream_t st)
{
    if (nunits <= 0) return hipSuccess;
    if (adj) k_rf3y_batch<true><<<nunits, 64 * kYWaves, 0, st>>>(E, U, src_out);
    else k_rf3y_batch<false><<<nunits, 64 * kYWaves, 0, st>>>(E, U, src_out);
    return hipGetLastError();
}

hipError_t setup_phi_x(const float4 *T, const uint8_t *code, float *PHI, int nx, int ny, int lx, hipStream_t st)
{
    const long n = (long)ny * 4 * 64;
    k_phi_x<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(T, code, PHI, nx, ny, lx);
    return hipGetLastError();
}

hipError_t setup_ky_y(const float4 *T, const uint8_t *code, float *KY, int nx, int ny, int ly, hipStream_t st)
{
    const int nblk = (nx + kYCols - 1) / kYCols;
    const long n = (long)nblk * kYCols * kYWaves * 4;
    k_kvec_y<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(T, code, KY, nx, ny, ly, nblk);
    return hipGetLastError();
}

hipError_t setup_per_x(const float4 *T, const uint8_t *code, float *PER, int nx, int ny, int lx, hipStream_t st)
{
    const long n = (long)ny * 4;
    k_per_x<<<(unsigned)((n + 63) / 64), 64, 0, st>>>(T, code, PER, nx, ny, lx);
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
