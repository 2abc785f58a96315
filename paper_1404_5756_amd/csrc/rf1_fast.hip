// Fused 1st-RF (eqs. "proc1-1", "proc1-2" with the Hayden relation, eq.
// "crucial"): all K iterations of one direction in one kernel, the lines
// staying on chip between iterations, FP32 or FP64.  It is the fast form of the
// paper's baseline filter, beside the plain one (one launch per iteration,
// sweep_seq.hip), so that the 3rd-RF is compared with a 1st-RF that moves the
// field through HBM once per direction (8 B per point and direction in FP32,
// 16 B in FP64) rather than once per iteration.
//
// Each sweep is the first-order recurrence p_i = beta_i s_i + alpha_i p_{i-1}
// (descending: s_i = beta_i p_i + alpha_i s_{i+1}), zero before a segment start
// (end).  A line is cut into chunks; a chunk maps its incoming value x to
// A x + b (A = product of its alphas after its last reset, b its value from a
// zero start), the chunks' maps are composed by a scan, and every chunk reruns
// from its true incoming value.  Imaginary points keep their values between
// iterations; inputs are taken at sea points only and outputs are zero off sea.
//
// x: one wave per line (a row of one plane), lane c owns points [cL, cL+L),
// lines staged through LDS for coalesced loads and stores; the scan runs over
// the 64 lanes with cross-lane shuffles.  y: 16 waves per block of 64 columns,
// wave w owns rows [wL, wL+L), lane = column; the chunk maps pass between the
// waves through LDS.  Coefficients: the block's FP64 1st-RF table (alpha, beta),
// kept in registers for a row (x) and read per pass (y).
#include "rf3_internal.h"
#include "sweeps.h"

namespace rf {

namespace {

constexpr int kR1XWaves = 4;

template <class T>
__device__ __forceinline__ T sel0(T x, bool reset) { return reset ? T(0) : x; }

// inclusive scan over the 64 lanes of the chunk maps (A, b): after it, b is the
// value leaving my chunk from a zero value entering chunk 0 (ascending) or 63
// (descending); the carry into my chunk is the previous lane's b
template <class T, bool DESC>
__device__ __forceinline__ T lane_carry(T A, T b, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T Ap = DESC ? __shfl_down(A, d, 64) : __shfl_up(A, d, 64);
        const T bp = DESC ? __shfl_down(b, d, 64) : __shfl_up(b, d, 64);
        const bool has = DESC ? lane + d < 64 : lane >= d;
        if (has) {
            b = b + A * bp;
            A = A * Ap;
        }
    }
    const T c = DESC ? __shfl_down(b, 1, 64) : __shfl_up(b, 1, 64);
    return (DESC ? lane < 63 : lane > 0) ? c : T(0);
}

template <class T, int L>
__global__ __launch_bounds__(64 * kR1XWaves) void k_rf1x(const T *in, T *out, const double2 *__restrict__ C,
                                                          const uint64_t *__restrict__ LM, int nx, int ny,
                                                          int nplanes, int K)
{
    __shared__ T stage[kR1XWaves][64 * L];
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int row = slot * 8 + xcd;   // XCD-aware: neighbouring rows on different XCDs
    if (row >= ny) return;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int x0 = lane * L;
    constexpr int LP = (L + 7) & ~7;
    const uint64_t *lm = LM + (long)row * kLaneMasks * LP;   // FRESET, BRESET, not-SEA per step
    T al[L], be[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int x = x0 + i;
        const double2 c = x < nx ? C[(long)row * nx + x] : make_double2(0.0, 0.0);
        al[i] = (T)c.x;
        be[i] = (T)c.y;
    }
    T *stg = stage[wave];
    const long plane = (long)nx * ny;
    for (int pl = wave; pl < nplanes; pl += kR1XWaves) {
        const T *src = in + pl * plane + (long)row * nx;
        T *dst = out + pl * plane + (long)row * nx;
        // coalesced load of the line into LDS, then my chunk
        for (int x = lane; x < 64 * L; x += 64) stg[x] = x < nx ? src[x] : T(0);
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS writes done
        __builtin_amdgcn_wave_barrier();
        T v[L];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const bool sea = !((lm[2 * LP + i] >> lane) & 1);
            v[i] = sea ? stg[x0 + i] : T(0);   // input only at sea points
        }
        for (int k = 0; k < K; ++k) {
            // ascending sweep (eq. "proc1-1"): zero before a segment start
            T A = T(1), b = T(0);
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const bool r = (lm[i] >> lane) & 1;
                b = fma(al[i], sel0(b, r), be[i] * v[i]);
                A = al[i] * sel0(A, r);
            }
            T p = lane_carry<T, false>(A, b, lane);
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const bool r = (lm[i] >> lane) & 1;
                p = fma(al[i], sel0(p, r), be[i] * v[i]);
                v[i] = p;
            }
            // descending sweep (eq. "proc1-2"): zero before a segment end
            A = T(1);
            b = T(0);
#pragma unroll
            for (int i = L - 1; i >= 0; --i) {
                const bool r = (lm[LP + i] >> lane) & 1;
                b = fma(al[i], sel0(b, r), be[i] * v[i]);
                A = al[i] * sel0(A, r);
            }
            T s = lane_carry<T, true>(A, b, lane);
#pragma unroll
            for (int i = L - 1; i >= 0; --i) {
                const bool r = (lm[LP + i] >> lane) & 1;
                s = fma(al[i], sel0(s, r), be[i] * v[i]);
                v[i] = s;
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const bool sea = !((lm[2 * LP + i] >> lane) & 1);
            stg[x0 + i] = sea ? v[i] : T(0);   // output zero off sea
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        for (int x = lane; x < nx; x += 64) dst[x] = stg[x];
        __builtin_amdgcn_wave_barrier();
    }
}

// One y pass over my chunk of L rows (lane = column): DESC selects the sweep
// direction, LOCAL the chunk's map from a zero value (A, and the returned b)
// instead of the rerun that overwrites v.  Coefficients stream through a window
// of WIN rows loaded ahead of their use; the compiler fence after each row keeps
// the loads from being hoisted further (hoisted, the whole pass's coefficients
// would not fit in the registers).
template <class T, int L, bool DESC, bool LOCAL>
__device__ __forceinline__ T y_pass(T (&v)[L], T x, T &A, const double2 *C, const uint64_t *rm, int lane, int r0,
                                    int ny, int nx, int col)
{
    constexpr int WIN = 4;
    // running row of the next coefficient load (rows past the grid read the last
    // row: they are reset by their masks and carry nothing)
    int rn = DESC ? r0 + L - 1 : r0;
    auto coef = [&]() -> double2 {
        const double2 c = C[(long)min(rn, ny - 1) * nx + col];
        rn += DESC ? -1 : 1;
        asm volatile("" : "+s"(rn));
        return c;
    };
    double2 win[WIN];
#pragma unroll
    for (int q = 0; q < WIN; ++q)
        if (q < L) win[q] = coef();
    A = T(1);
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int i = DESC ? L - 1 - t : t;
        const double2 c = win[t % WIN];
        if (t + WIN < L) win[t % WIN] = coef();
        const bool r = (rm[i] >> lane) & 1;
        x = fma((T)c.x, sel0(x, r), (T)c.y * v[i]);
        if (LOCAL) A = (T)c.x * sel0(A, r);
        else v[i] = x;
        asm volatile("" ::: "memory");
    }
    return x;
}

template <class T, int L>
__global__ __launch_bounds__(64 * kYWaves) void k_rf1y(const T *in, T *out, const double2 *__restrict__ C,
                                                       const uint64_t *__restrict__ LM, int nx, int ny, int nplanes,
                                                       int nblk, int nslot, int K)
{
    __shared__ T sh[2][kYWaves][2][kYCols];   // (A, b) of every wave's chunk, per sweep direction
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int blk = (slot / nslot) * 8 + xcd, j = slot % nslot;
    if (blk >= nblk) return;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool cok = blk * kYCols + lane < nx;
    const int col = cok ? blk * kYCols + lane : nx - 1;   // columns past the grid: not-sea, never stored
    const int lys = lmy_stride(L);
    const uint64_t *lm = LM + (long)blk * kLaneMasks * lys + 8;   // entry r = row r
    const int r0 = w * L;
    const long plane = (long)nx * ny;
    const uint64_t *fm = lm + r0, *bm = lm + lys + r0;             // FRESET, BRESET of my rows
    for (int pl = j; pl < nplanes; pl += nslot) {
        const T *src = in + pl * plane;
        T *dst = out + pl * plane;
        T v[L];
        {
            int rn = r0;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const bool sea = !((lm[2 * lys + r0 + i] >> lane) & 1);   // false past the grid
                const T val = src[(long)min(rn, ny - 1) * nx + col];
                v[i] = sea ? val : T(0);
                rn += 1;
                asm volatile("" : "+s"(rn));
            }
        }
        for (int k = 0; k < K; ++k) {
            // ascending: my chunk's map, the chain over the chunks above, rerun
            T A;
            T b = y_pass<T, L, false, true>(v, T(0), A, C, fm, lane, r0, ny, nx, col);
            sh[0][w][0][lane] = A;
            sh[0][w][1][lane] = b;
            __syncthreads();
            T p = T(0);
            for (int q = 0; q < w; ++q) p = sh[0][q][1][lane] + sh[0][q][0][lane] * p;
            y_pass<T, L, false, false>(v, p, A, C, fm, lane, r0, ny, nx, col);
            // descending
            b = y_pass<T, L, true, true>(v, T(0), A, C, bm, lane, r0, ny, nx, col);
            sh[1][w][0][lane] = A;
            sh[1][w][1][lane] = b;
            __syncthreads();
            T s = T(0);
            for (int q = kYWaves - 1; q > w; --q) s = sh[1][q][1][lane] + sh[1][q][0][lane] * s;
            y_pass<T, L, true, false>(v, s, A, C, bm, lane, r0, ny, nx, col);
        }
        {
            int rn = r0;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const bool sea = !((lm[2 * lys + r0 + i] >> lane) & 1);
                if (cok && rn < ny) dst[(long)rn * nx + col] = sea ? v[i] : T(0);
                rn += 1;
                asm volatile("" : "+s"(rn));
            }
        }
        __syncthreads();   // sh is rewritten by the next plane
    }
}

int cu_count_r1()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

template <class T>
hipError_t launch_x(const T *in, T *out, const double2 *C, const uint64_t *LM, int lx, int nx, int ny, int nplanes,
                    int K, hipStream_t st)
{
    const unsigned nb = (unsigned)(((ny + 7) / 8) * 8);
#define RF1_X(Lv)                                                                                         \
    case Lv:                                                                                              \
        k_rf1x<T, Lv><<<nb, 64 * kR1XWaves, 0, st>>>(in, out, C, LM, nx, ny, nplanes, K);                 \
        break;
    switch (lx) {
        RF1_X(1) RF1_X(3) RF1_X(5) RF1_X(7) RF1_X(9) RF1_X(11) RF1_X(13) RF1_X(15) RF1_X(17) RF1_X(19) RF1_X(21)
        RF1_X(23) RF1_X(25) RF1_X(27) RF1_X(29) RF1_X(31) RF1_X(33)
    default: return hipErrorNotSupported;
    }
#undef RF1_X
    return hipGetLastError();
}

template <class T>
hipError_t launch_y(const T *in, T *out, const double2 *C, const uint64_t *LM, int ly, int nx, int ny, int nplanes,
                    int K, hipStream_t st)
{
    const int nblk = (nx + kYCols - 1) / kYCols, nb8 = ((nblk + 7) / 8) * 8;
    // one workgroup per CU at a time: enough plane slots to fill the chip
    const int cus = cu_count_r1();
    int nslot = (cus + nb8 - 1) / nb8;
    nslot = nslot < 1 ? 1 : (nslot > nplanes ? nplanes : nslot);
    const unsigned nb = (unsigned)(nb8 * nslot);
#define RF1_Y(Lv)                                                                                         \
    case Lv:                                                                                              \
        k_rf1y<T, Lv><<<nb, 64 * kYWaves, 0, st>>>(in, out, C, LM, nx, ny, nplanes, nblk, nslot, K);      \
        break;
    switch (ly) {
        RF1_Y(1) RF1_Y(2) RF1_Y(3) RF1_Y(4) RF1_Y(6) RF1_Y(8) RF1_Y(12) RF1_Y(16) RF1_Y(20) RF1_Y(24) RF1_Y(28)
        RF1_Y(32) RF1_Y(36) RF1_Y(40) RF1_Y(45) RF1_Y(48) RF1_Y(56) RF1_Y(64)
    default: return hipErrorNotSupported;
    }
#undef RF1_Y
    return hipGetLastError();
}

}  // namespace

hipError_t fused_rf1(const void *in, void *out, bool fp64, const double2 *C, const uint64_t *LM, int dir, int l,
                     int nx, int ny, int nplanes, int K, hipStream_t st)
{
    if (dir == 0)
        return fp64 ? launch_x<double>((const double *)in, (double *)out, C, LM, l, nx, ny, nplanes, K, st)
                    : launch_x<float>((const float *)in, (float *)out, C, LM, l, nx, ny, nplanes, K, st);
    return fp64 ? launch_y<double>((const double *)in, (double *)out, C, LM, l, nx, ny, nplanes, K, st)
                : launch_y<float>((const float *)in, (float *)out, C, LM, l, nx, ny, nplanes, K, st);
}

}  // namespace rf
