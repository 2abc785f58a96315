// Vector steps of the conjugate-gradient minimiser of the 3D-VAR harness
// (Sec. 2.1 solves its preconditioned system by CG).  The scalars of the
// iteration stay in device memory (double s[kCgSlots]) so a whole iteration is
// a sequence of kernel launches with no host round trip.  Dot products are
// deterministic: a fixed grid of blocks writes per-block partial sums (FP64)
// into the caller's work array, and one block adds them in a fixed order.
#include "rf3_internal.h"

namespace {

constexpr int kCgBlocks = 1024, kCgThreads = 256;

// vectors are streamed once per kernel: non-temporal accesses, so that they do
// not evict the covariance operator's coefficient tables from L2
template <class T>
__device__ __forceinline__ T ld(const T *p) { return __builtin_nontemporal_load(p); }
template <class T>
__device__ __forceinline__ void st(T *p, T v) { __builtin_nontemporal_store(v, p); }

__device__ double block_sum(double v, double *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kCgThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    return sh[0];
}

// partial[b] = sum over this block's grid-stride share of a[i] * b[i]
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_dot(const T *__restrict__ a, const T *__restrict__ b,
                                                   double *__restrict__ partial, long n)
{
    __shared__ double sh[kCgThreads];
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += (long)kCgBlocks * kCgThreads)
        acc += (double)ld(a + i) * (double)ld(b + i);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// q = p + w (not stored when q is null); partial sums of p.q
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_q_dot(const T *__restrict__ p, const T *__restrict__ w,
                                                     T *__restrict__ q, double *__restrict__ partial, long n)
{
    __shared__ double sh[kCgThreads];
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += (long)kCgBlocks * kCgThreads) {
        const T pi = ld(p + i), qi = pi + ld(w + i);
        if (q) st(q + i, qi);
        acc += (double)pi * (double)qi;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// a = s[RR] / s[PQ]; v += a p; r -= a q; partial sums of r.r
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_step(const T *__restrict__ p, const T *__restrict__ q,
                                                    T *__restrict__ v, T *__restrict__ r,
                                                    const double *__restrict__ s, double *__restrict__ partial,
                                                    long n)
{
    __shared__ double sh[kCgThreads];
    const double pq = s[RF_CG_PQ];
    const T a = pq > 0.0 ? (T)(s[RF_CG_RR] / pq) : (T)0;
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += (long)kCgBlocks * kCgThreads) {
        st(v + i, ld(v + i) + a * ld(p + i));
        const T ri = ld(r + i) - a * ld(q + i);
        st(r + i, ri);
        acc += (double)ri * (double)ri;
    }
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// a = s[RR] / s[PQ]; v += a p; r -= a (p + w); partial sums of r.r
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_step_pw(const T *__restrict__ p, const T *__restrict__ w,
                                                       T *__restrict__ v, T *__restrict__ r,
                                                       const double *__restrict__ s, double *__restrict__ partial,
                                                       long n)
{
    __shared__ double sh[kCgThreads];
    const double pq = s[RF_CG_PQ];
    const T a = pq > 0.0 ? (T)(s[RF_CG_RR] / pq) : (T)0;
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += (long)kCgBlocks * kCgThreads) {
        const T pi = ld(p + i);
        st(v + i, ld(v + i) + a * pi);
        const T ri = ld(r + i) - a * (pi + ld(w + i));
        st(r + i, ri);
        acc += (double)ri * (double)ri;
    }
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// p = r + (s[RR_NEW] / s[RR]) p
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_dir(const T *__restrict__ r, T *__restrict__ p,
                                                   const double *__restrict__ s, long n)
{
    const double rr = s[RF_CG_RR];
    const T b = rr > 0.0 ? (T)(s[RF_CG_RR_NEW] / rr) : (T)0;
    for (long i = (long)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += (long)kCgBlocks * kCgThreads)
        st(p + i, ld(r + i) + b * ld(p + i));
}

// s[slot] = sum of the partials in a fixed order
__global__ __launch_bounds__(kCgThreads) void k_finish(const double *__restrict__ partial, double *__restrict__ s,
                                                       int slot)
{
    __shared__ double sh[kCgThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < kCgBlocks; i += kCgThreads) acc += partial[i];
    const double v = block_sum(acc, sh);
    if (threadIdx.x == 0) s[slot] = v;
}

__global__ void k_set(double *s, int to, int from) { s[to] = s[from]; }

// y += a x
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_axpy(T a, const T *__restrict__ x, T *__restrict__ y, long n)
{
    for (long i = (long)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += (long)kCgBlocks * kCgThreads)
        st(y + i, ld(y + i) + a * ld(x + i));
}

bool args_ok(int prec, long n, const void *a, const void *b)
{
    return (prec == RF_FP32 || prec == RF_FP64) && n >= 1 && a && b;
}

}  // namespace

extern "C" size_t rf_cg_work_bytes(void) { return (size_t)kCgBlocks * sizeof(double); }

extern "C" int rf_dot(rf_prec prec, int64_t n, const void *a, const void *b, void *work, double *s, int32_t slot,
                      void *stream)
{
    if (!args_ok(prec, n, a, b) || !work || !s || slot < 0 || slot >= RF_CG_SLOTS) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(work);
    if (prec == RF_FP32)
        k_dot<float><<<kCgBlocks, kCgThreads, 0, st>>>((const float *)a, (const float *)b, part, n);
    else
        k_dot<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)a, (const double *)b, part, n);
    k_finish<<<1, kCgThreads, 0, st>>>(part, s, slot);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_cg_q_dot(rf_prec prec, int64_t n, const void *p, const void *w, void *q, void *work, double *s,
                           void *stream)
{
    if (!args_ok(prec, n, p, w) || !work || !s) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(work);
    if (prec == RF_FP32)
        k_q_dot<float><<<kCgBlocks, kCgThreads, 0, st>>>((const float *)p, (const float *)w, (float *)q, part, n);
    else
        k_q_dot<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)p, (const double *)w, (double *)q, part, n);
    k_finish<<<1, kCgThreads, 0, st>>>(part, s, RF_CG_PQ);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_cg_step(rf_prec prec, int64_t n, const void *p, const void *q, void *v, void *r, void *work,
                          double *s, void *stream)
{
    if (!args_ok(prec, n, p, q) || !v || !r || !work || !s) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(work);
    if (prec == RF_FP32)
        k_step<float><<<kCgBlocks, kCgThreads, 0, st>>>((const float *)p, (const float *)q, (float *)v, (float *)r, s,
                                                       part, n);
    else
        k_step<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)p, (const double *)q, (double *)v,
                                                        (double *)r, s, part, n);
    k_finish<<<1, kCgThreads, 0, st>>>(part, s, RF_CG_RR_NEW);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_cg_dir(rf_prec prec, int64_t n, const void *r, void *p, double *s, void *stream)
{
    if (!args_ok(prec, n, r, p) || !s) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (prec == RF_FP32)
        k_dir<float><<<kCgBlocks, kCgThreads, 0, st>>>((const float *)r, (float *)p, s, n);
    else
        k_dir<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)r, (double *)p, s, n);
    // rr <- rr_new for the next iteration (after k_dir has read both)
    k_set<<<1, 1, 0, st>>>(s, RF_CG_RR, RF_CG_RR_NEW);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_axpy(rf_prec prec, int64_t n, double a, const void *x, void *y, void *stream)
{
    if (!args_ok(prec, n, x, y)) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (prec == RF_FP32)
        k_axpy<float><<<kCgBlocks, kCgThreads, 0, st>>>((float)a, (const float *)x, (float *)y, n);
    else
        k_axpy<double><<<kCgBlocks, kCgThreads, 0, st>>>(a, (const double *)x, (double *)y, n);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_cg_step_pw(rf_prec prec, int64_t n, const void *p, const void *w, void *v, void *r, void *work,
                             double *s, void *stream)
{
    if (!args_ok(prec, n, p, w) || !v || !r || !work || !s) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(work);
    if (prec == RF_FP32)
        k_step_pw<float><<<kCgBlocks, kCgThreads, 0, st>>>((const float *)p, (const float *)w, (float *)v,
                                                           (float *)r, s, part, n);
    else
        k_step_pw<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)p, (const double *)w, (double *)v,
                                                            (double *)r, s, part, n);
    k_finish<<<1, kCgThreads, 0, st>>>(part, s, RF_CG_RR_NEW);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}
