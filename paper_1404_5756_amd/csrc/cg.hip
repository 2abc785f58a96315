// Vector steps of the conjugate-gradient minimiser of the 3D-VAR harness
// (Sec. 2.1 solves its preconditioned system by CG).  The scalars of the
// iteration stay in device memory (double s[kCgSlots]) so a whole iteration is
// a sequence of kernel launches with no host round trip.  Dot products are
// deterministic: a fixed grid of blocks writes per-block partial sums (FP64)
// into the caller's work array, and one block adds them in a fixed order.
#include <initializer_list>
#include <mutex>

#include "rf3_internal.h"

namespace {

constexpr int kCgBlocks = 1024, kCgThreads = 256;
constexpr long kCgStride = (long)kCgBlocks * kCgThreads;

// vectors are streamed once per kernel: non-temporal accesses, so that they do
// not evict the covariance operator's coefficient tables from L2
template <class E>
__device__ __forceinline__ E ld(const E *p) { return __builtin_nontemporal_load(p); }
template <class E>
__device__ __forceinline__ void st(E *p, E v) { __builtin_nontemporal_store(v, p); }

// The bulk of each vector is streamed as 16-byte elements (one access per lane
// and stream; the bytes in flight per lane set the bandwidth a streaming kernel
// reaches).  The host passes nv, the number of 16-byte elements, which is 0 when
// a pointer is not 16-byte aligned; a scalar loop takes the remaining entries.
template <class T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <class T>
using vec16 = typename Vec16<T>::type;
template <class T>
constexpr int kVecLanes = 16 / sizeof(T);

// products summed in FP64 (vector components in order)
__device__ __forceinline__ double prod(float a, float b) { return (double)a * (double)b; }
__device__ __forceinline__ double prod(double a, double b) { return a * b; }
template <class V>
__device__ __forceinline__ double prod(V a, V b)
{
    double s = 0.0;
    for (int c = 0; c < (int)(sizeof(V) / sizeof(a[0])); ++c) s += (double)a[c] * (double)b[c];
    return s;
}

// this thread's first index in the vector part and in the scalar tail
__device__ __forceinline__ long first_index() { return (long)blockIdx.x * kCgThreads + threadIdx.x; }

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

template <class E>
__device__ double dot_run(const E *a, const E *b, long i, long end)
{
    double acc = 0.0;
    for (; i < end; i += kCgStride) acc += prod(ld(a + i), ld(b + i));
    return acc;
}

// partial[b] = sum over this block's grid-stride share of a[i] * b[i]
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_dot(const T *__restrict__ a, const T *__restrict__ b,
                                                   double *__restrict__ partial, long n, long nv)
{
    __shared__ double sh[kCgThreads];
    using V = vec16<T>;
    const long t0 = first_index();
    double acc = dot_run((const V *)a, (const V *)b, t0, nv);
    acc += dot_run(a, b, nv * kVecLanes<T> + t0, n);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <class E>
__device__ double q_dot_run(const E *p, const E *w, E *q, long i, long end)
{
    double acc = 0.0;
    for (; i < end; i += kCgStride) {
        const E pi = ld(p + i), qi = pi + ld(w + i);
        if (q) st(q + i, qi);
        acc += prod(pi, qi);
    }
    return acc;
}

// q = p + w (not stored when q is null); partial sums of p.q
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_q_dot(const T *__restrict__ p, const T *__restrict__ w,
                                                     T *__restrict__ q, double *__restrict__ partial, long n, long nv)
{
    __shared__ double sh[kCgThreads];
    using V = vec16<T>;
    const long t0 = first_index();
    double acc = q_dot_run((const V *)p, (const V *)w, (V *)q, t0, nv);
    acc += q_dot_run(p, w, q, nv * kVecLanes<T> + t0, n);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// the step length a = s[RR] / s[PQ] (0 when p.Ap is not positive)
template <class T>
__device__ __forceinline__ T step_length(const double *s)
{
    const double pq = s[RF_CG_PQ];
    return pq > 0.0 ? (T)(s[RF_CG_RR] / pq) : (T)0;
}

template <class T, class E>
__device__ double step_run(T a, const E *p, const E *q, E *v, E *r, long i, long end)
{
    double acc = 0.0;
    for (; i < end; i += kCgStride) {
        st(v + i, ld(v + i) + a * ld(p + i));
        const E ri = ld(r + i) - a * ld(q + i);
        st(r + i, ri);
        acc += prod(ri, ri);
    }
    return acc;
}

// a = s[RR] / s[PQ]; v += a p; r -= a q; partial sums of r.r
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_step(const T *__restrict__ p, const T *__restrict__ q,
                                                    T *__restrict__ v, T *__restrict__ r,
                                                    const double *__restrict__ s, double *__restrict__ partial,
                                                    long n, long nv)
{
    __shared__ double sh[kCgThreads];
    using V = vec16<T>;
    const T a = step_length<T>(s);
    const long t0 = first_index();
    double acc = step_run(a, (const V *)p, (const V *)q, (V *)v, (V *)r, t0, nv);
    acc += step_run(a, p, q, v, r, nv * kVecLanes<T> + t0, n);
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

template <class T, class E>
__device__ double step_pw_run(T a, const E *p, const E *w, E *v, E *r, long i, long end)
{
    double acc = 0.0;
    for (; i < end; i += kCgStride) {
        const E pi = ld(p + i);
        st(v + i, ld(v + i) + a * pi);
        const E ri = ld(r + i) - a * (pi + ld(w + i));
        st(r + i, ri);
        acc += prod(ri, ri);
    }
    return acc;
}

// a = s[RR] / s[PQ]; v += a p; r -= a (p + w); partial sums of r.r
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_step_pw(const T *__restrict__ p, const T *__restrict__ w,
                                                       T *__restrict__ v, T *__restrict__ r,
                                                       const double *__restrict__ s, double *__restrict__ partial,
                                                       long n, long nv)
{
    __shared__ double sh[kCgThreads];
    using V = vec16<T>;
    const T a = step_length<T>(s);
    const long t0 = first_index();
    double acc = step_pw_run(a, (const V *)p, (const V *)w, (V *)v, (V *)r, t0, nv);
    acc += step_pw_run(a, p, w, v, r, nv * kVecLanes<T> + t0, n);
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// p = r + b p over one range
template <class T, class E>
__device__ void dir_run(T b, const E *r, E *p, long i, long end)
{
    for (; i < end; i += kCgStride) st(p + i, ld(r + i) + b * ld(p + i));
}

// p = r + (s[RR_NEW] / s[RR]) p
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_dir(const T *__restrict__ r, T *__restrict__ p,
                                                   const double *__restrict__ s, long n, long nv)
{
    using V = vec16<T>;
    const double rr = s[RF_CG_RR];
    const T b = rr > 0.0 ? (T)(s[RF_CG_RR_NEW] / rr) : (T)0;
    const long t0 = first_index();
    dir_run(b, (const V *)r, (V *)p, t0, nv);
    dir_run(b, r, p, nv * kVecLanes<T> + t0, n);
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

template <class T, class E>
__device__ void axpy_run(T a, const E *x, E *y, long i, long end)
{
    for (; i < end; i += kCgStride) st(y + i, ld(y + i) + a * ld(x + i));
}

// y += a x
template <class T>
__global__ __launch_bounds__(kCgThreads) void k_axpy(T a, const T *__restrict__ x, T *__restrict__ y, long n,
                                                    long nv)
{
    using V = vec16<T>;
    const long t0 = first_index();
    axpy_run(a, (const V *)x, (V *)y, t0, nv);
    axpy_run(a, x, y, nv * kVecLanes<T> + t0, n);
}

// number of 16-byte elements of n entries of `es` bytes when every non-null
// pointer is 16-byte aligned, else 0
long vec_count(long n, int es, std::initializer_list<const void *> ptrs)
{
    for (const void *q : ptrs)
        if (q && reinterpret_cast<uintptr_t>(q) % 16) return 0;
    return n / (16 / es);
}

bool args_ok(int prec, long n, const void *a, const void *b)
{
    return (prec == RF_FP32 || prec == RF_FP64) && n >= 1 && a && b;
}

// Scratch of the allocation-free dot product (rf_dot_noalloc): the per-block
// FP64 partial sums of the fixed reduction grid.  Every device holds its own
// copy at its own address; host code never uses the name below as an address,
// only the pointer hipGetSymbolAddress returns for the current device.
constexpr int kScratchDoubles = kCgBlocks;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;

// device address of this device's scratch, looked up once per device (with
// that device current); null if the lookup fails
double *scratch_ptr()
{
    static std::mutex mu;
    static double *ptr[kMaxDevices];
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        ptr[dev] = static_cast<double *>(p);
    }
    return ptr[dev];
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
        k_dot<float><<<kCgBlocks, kCgThreads, 0, st>>>((const float *)a, (const float *)b, part, n, vec_count(n, 4, {a, b}));
    else
        k_dot<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)a, (const double *)b, part, n,
                                                  vec_count(n, 8, {a, b}));
    k_finish<<<1, kCgThreads, 0, st>>>(part, s, slot);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" size_t rf_dot_noalloc_scratch_bytes(void) { return sizeof(scratch); }

extern "C" int rf_dot_noalloc(rf_prec prec, int64_t n, const void *a, const void *b, double *s, int32_t slot,
                              void *stream)
{
    if (!args_ok(prec, n, a, b) || !s || slot < 0 || slot >= RF_CG_SLOTS) return RF_E_ARG;
    // the reduction grid writes one partial per block: kCgBlocks must fit the scratch
    static_assert(kCgBlocks <= kScratchDoubles, "scratch smaller than the reduction grid");
    if (rf_cg_work_bytes() > sizeof(scratch)) return RF_E_UNSUPPORTED;
    double *part = scratch_ptr();
    if (!part) return RF_E_HIP;
    return rf_dot(prec, n, a, b, part, s, slot, stream);
}

extern "C" int rf_cg_q_dot(rf_prec prec, int64_t n, const void *p, const void *w, void *q, void *work, double *s,
                           void *stream)
{
    if (!args_ok(prec, n, p, w) || !work || !s) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(work);
    if (prec == RF_FP32)
        k_q_dot<float><<<kCgBlocks, kCgThreads, 0, st>>>((const float *)p, (const float *)w, (float *)q, part, n,
                                                   vec_count(n, 4, {p, w, q}));
    else
        k_q_dot<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)p, (const double *)w, (double *)q, part, n,
                                                    vec_count(n, 8, {p, w, q}));
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
                                                       part, n, vec_count(n, 4, {p, q, v, r}));
    else
        k_step<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)p, (const double *)q, (double *)v,
                                                        (double *)r, s, part, n, vec_count(n, 8, {p, q, v, r}));
    k_finish<<<1, kCgThreads, 0, st>>>(part, s, RF_CG_RR_NEW);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_cg_dir(rf_prec prec, int64_t n, const void *r, void *p, double *s, void *stream)
{
    if (!args_ok(prec, n, r, p) || !s) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (prec == RF_FP32)
        k_dir<float><<<kCgBlocks, kCgThreads, 0, st>>>((const float *)r, (float *)p, s, n, vec_count(n, 4, {r, p}));
    else
        k_dir<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)r, (double *)p, s, n, vec_count(n, 8, {r, p}));
    // rr <- rr_new for the next iteration (after k_dir has read both)
    k_set<<<1, 1, 0, st>>>(s, RF_CG_RR, RF_CG_RR_NEW);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_axpy(rf_prec prec, int64_t n, double a, const void *x, void *y, void *stream)
{
    if (!args_ok(prec, n, x, y)) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (prec == RF_FP32)
        k_axpy<float><<<kCgBlocks, kCgThreads, 0, st>>>((float)a, (const float *)x, (float *)y, n, vec_count(n, 4, {x, y}));
    else
        k_axpy<double><<<kCgBlocks, kCgThreads, 0, st>>>(a, (const double *)x, (double *)y, n, vec_count(n, 8, {x, y}));
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
                                                           (float *)r, s, part, n, vec_count(n, 4, {p, w, v, r}));
    else
        k_step_pw<double><<<kCgBlocks, kCgThreads, 0, st>>>((const double *)p, (const double *)w, (double *)v,
                                                            (double *)r, s, part, n, vec_count(n, 8, {p, w, v, r}));
    k_finish<<<1, kCgThreads, 0, st>>>(part, s, RF_CG_RR_NEW);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}
