// Bilinear observation operator H and its adjoint H^T for the 3D-VAR harness
// (the conjugate-gradient minimiser of Sec. 2.1 applies H^T R^-1 H and the
// covariance factors every iteration).  Observation o sits at level lev[o] and position (x[o], y[o]) in
// grid units; it reads the four surrounding grid points with bilinear weights.
//
// H is a gather (one thread per observation).  H^T is a gather too, over the
// list of distinct grid points that observations touch, each with its own
// (observation, corner) entries in increasing observation order: no atomics,
// so the result does not depend on scheduling.  A fill kernel (not a memset,
// so the call can be captured into a graph) zeroes the rest of the field.
#include <algorithm>
#include <math.h>
#include <numeric>
#include <string.h>
#include <vector>

#include "rf3_internal.h"

namespace {

constexpr uint32_t kObsMagic = 0x5346424fu;   // "OBFS"

struct ObsPlanHeader {
    uint32_t magic, version;
    int32_t nobs, nuniq;
    int64_t npts;
    uint64_t off_idx, off_w, off_upt, off_uptr, off_ent, total_bytes;
    uint64_t pad;
};
static_assert(sizeof(ObsPlanHeader) <= 256, "header fits before the tables");

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    uint64_t off_idx, off_w, off_upt, off_uptr, off_ent, total;
};

Layout obs_layout(int32_t nobs, int32_t nuniq)
{
    Layout L;
    L.off_idx = 256;
    L.off_w = a256(L.off_idx + (size_t)nobs * 4 * 4);
    L.off_upt = a256(L.off_w + (size_t)nobs * 4 * 8);
    L.off_uptr = a256(L.off_upt + (size_t)nuniq * 4);
    L.off_ent = a256(L.off_uptr + ((size_t)nuniq + 1) * 4);
    L.total = a256(L.off_ent + (size_t)nobs * 4 * 4);
    return L;
}

// corner point indices and weights of observation o; false if outside the grid
bool corners(const rf_grid *g, int32_t lev, double x, double y, int32_t idx[4], double w[4])
{
    if (!(lev >= 0 && lev < g->nlev)) return false;
    if (!(x >= 0.0 && x <= g->nx - 1 && y >= 0.0 && y <= g->ny - 1)) return false;
    int i = (int)floor(x), j = (int)floor(y);
    if (i > g->nx - 2) i = std::max(g->nx - 2, 0);
    if (j > g->ny - 2) j = std::max(g->ny - 2, 0);
    const int i1 = std::min(i + 1, g->nx - 1), j1 = std::min(j + 1, g->ny - 1);
    const double fx = g->nx > 1 ? x - i : 0.0, fy = g->ny > 1 ? y - j : 0.0;
    const long base = (long)lev * g->nx * g->ny;
    idx[0] = (int32_t)(base + (long)j * g->nx + i);
    idx[1] = (int32_t)(base + (long)j * g->nx + i1);
    idx[2] = (int32_t)(base + (long)j1 * g->nx + i);
    idx[3] = (int32_t)(base + (long)j1 * g->nx + i1);
    w[0] = (1 - fx) * (1 - fy);
    w[1] = fx * (1 - fy);
    w[2] = (1 - fx) * fy;
    w[3] = fx * fy;
    return true;
}

struct HostObs {
    std::vector<int32_t> idx, upt, uptr, ent;
    std::vector<double> w;
};

int build(const rf_grid *g, int32_t nobs, const int32_t *lev, const double *x, const double *y, HostObs &H)
{
    if (!g || nobs < 1 || !lev || !x || !y) return RF_E_ARG;
    if (g->nx < 1 || g->ny < 1 || g->nlev < 1) return RF_E_SHAPE;
    if ((long)g->nx * g->ny * g->nlev >= (1L << 31) || (long)nobs * 4 >= (1L << 31)) return RF_E_SHAPE;
    H.idx.resize((size_t)nobs * 4);
    H.w.resize((size_t)nobs * 4);
    for (int32_t o = 0; o < nobs; ++o)
        if (!corners(g, lev[o], x[o], y[o], &H.idx[4 * (size_t)o], &H.w[4 * (size_t)o])) return RF_E_ARG;
    // entries sorted by (point, observation, corner): a stable sort keeps the observation order
    std::vector<int32_t> order((size_t)nobs * 4);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return H.idx[a] < H.idx[b]; });
    H.ent = order;
    H.upt.clear();
    H.uptr.clear();
    for (size_t k = 0; k < order.size(); ++k) {
        if (k == 0 || H.idx[order[k]] != H.idx[order[k - 1]]) {
            H.upt.push_back(H.idx[order[k]]);
            H.uptr.push_back((int32_t)k);
        }
    }
    H.uptr.push_back((int32_t)order.size());
    return RF_OK;
}

// the plan's own sizes must equal the launch sizes; otherwise nothing past the
// plan header is read and every output is set to NaN (a visible failure rather
// than a silently zero or partial result)
__device__ inline bool plan_matches(const ObsPlanHeader *hd, int32_t nobs, int32_t nuniq, int64_t npts)
{
    return hd->magic == kObsMagic && hd->nobs == nobs && hd->nuniq == nuniq && hd->npts == npts;
}
template <class T>
__device__ inline T nan_value() { return (T)__builtin_nan(""); }

template <class T>
__global__ void k_obs_apply(const ObsPlanHeader *__restrict__ hd, const int32_t *__restrict__ idx,
                            const double *__restrict__ w, const T *__restrict__ f, T *__restrict__ out, int32_t nobs,
                            int32_t nuniq, int64_t npts)
{
    const int32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nobs) return;
    if (!plan_matches(hd, nobs, nuniq, npts)) {
        out[o] = nan_value<T>();
        return;
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += (T)w[4 * o + c] * f[idx[4 * o + c]];
    out[o] = s;
}

// d = H f - y (a missing term is 0), rd = scale * rinv o d (rinv missing: 1)
template <class T>
__global__ void k_obs_innov(const ObsPlanHeader *__restrict__ hd, const int32_t *__restrict__ idx,
                            const double *__restrict__ w, const T *__restrict__ f, const T *__restrict__ y,
                            const T *__restrict__ rinv, T scale, T *__restrict__ d, T *__restrict__ rd,
                            int32_t nobs, int32_t nuniq, int64_t npts)
{
    const int32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nobs) return;
    if (!plan_matches(hd, nobs, nuniq, npts)) {
        if (d) d[o] = nan_value<T>();
        rd[o] = nan_value<T>();
        return;
    }
    T s = 0;
    if (f) {
#pragma unroll
        for (int c = 0; c < 4; ++c) s += (T)w[4 * o + c] * f[idx[4 * o + c]];
    }
    if (y) s -= y[o];
    if (d) d[o] = s;
    rd[o] = (rinv ? rinv[o] : (T)1) * scale * s;
}

// f[0, n) = 0: 16-byte stores over the first nv 16-byte elements (nv is 0 when
// f is not 16-byte aligned), then single entries.  Streamed once, so the stores
// are non-temporal and leave L2 to the covariance operator's tables.
// (NaN instead of 0 when the plan does not match the launch sizes)
template <class T>
__global__ void k_fill(T *__restrict__ f, long n, long nv, const ObsPlanHeader *__restrict__ hd, int32_t nobs,
                       int32_t nuniq)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const long t0 = (long)blockIdx.x * blockDim.x + threadIdx.x, stride = (long)gridDim.x * blockDim.x;
    const T val = plan_matches(hd, nobs, nuniq, n) ? (T)0 : nan_value<T>();
    u32x4 *fv = reinterpret_cast<u32x4 *>(f);
    T vv[16 / sizeof(T)];
    for (int q = 0; q < (int)(16 / sizeof(T)); ++q) vv[q] = val;
    const u32x4 z = *reinterpret_cast<const u32x4 *>(vv);
    for (long i = t0; i < nv; i += stride) __builtin_nontemporal_store(z, fv + i);
    for (long i = nv * (long)(16 / sizeof(T)) + t0; i < n; i += stride) __builtin_nontemporal_store(val, f + i);
}

template <class T>
__global__ void k_obs_adjoint(const ObsPlanHeader *__restrict__ hd, const int32_t *__restrict__ upt,
                              const int32_t *__restrict__ uptr, const int32_t *__restrict__ ent,
                              const double *__restrict__ w, const T *__restrict__ obs, T *__restrict__ f,
                              int32_t nobs, int32_t nuniq, int64_t npts)
{
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nuniq || !plan_matches(hd, nobs, nuniq, npts)) return;
    T s = 0;
    for (int32_t k = uptr[u]; k < uptr[u + 1]; ++k) {
        const int32_t e = ent[k];   // observation * 4 + corner
        s += (T)w[e] * obs[e >> 2];
    }
    f[upt[u]] = s;
}

}  // namespace

extern "C" size_t rf_obs_plan_bytes(const rf_grid *g, int32_t nobs, const int32_t *lev, const double *x,
                                    const double *y, int32_t *nuniq_out)
{
    HostObs H;
    if (build(g, nobs, lev, x, y, H) != RF_OK) return 0;
    if (nuniq_out) *nuniq_out = (int32_t)H.upt.size();
    return obs_layout(nobs, (int32_t)H.upt.size()).total;
}

extern "C" int rf_obs_plan(const rf_grid *g, int32_t nobs, const int32_t *lev, const double *x, const double *y,
                           void *plan, size_t plan_bytes)
{
    HostObs H;
    const int rc = build(g, nobs, lev, x, y, H);
    if (rc) return rc;
    const int32_t nuniq = (int32_t)H.upt.size();
    const Layout L = obs_layout(nobs, nuniq);
    if (!plan || plan_bytes != L.total) return RF_E_ARG;
    char *p = static_cast<char *>(plan);
    memset(p, 0, plan_bytes);
    ObsPlanHeader hd{};
    hd.magic = kObsMagic;
    hd.version = 1;
    hd.nobs = nobs;
    hd.nuniq = nuniq;
    hd.npts = (int64_t)g->nx * g->ny * g->nlev;
    hd.off_idx = L.off_idx;
    hd.off_w = L.off_w;
    hd.off_upt = L.off_upt;
    hd.off_uptr = L.off_uptr;
    hd.off_ent = L.off_ent;
    hd.total_bytes = L.total;
    memcpy(p, &hd, sizeof(hd));
    memcpy(p + L.off_idx, H.idx.data(), H.idx.size() * 4);
    memcpy(p + L.off_w, H.w.data(), H.w.size() * 8);
    memcpy(p + L.off_upt, H.upt.data(), H.upt.size() * 4);
    memcpy(p + L.off_uptr, H.uptr.data(), H.uptr.size() * 4);
    memcpy(p + L.off_ent, H.ent.data(), H.ent.size() * 4);
    return RF_OK;
}

// The launch sizes come from the caller (nobs, nuniq, npts as returned with the
// plan); the kernels check them against the plan's header before reading it.
extern "C" int rf_obs_apply(const void *plan_dev, int32_t nobs, int32_t nuniq, int64_t npts, rf_prec prec,
                            const void *field, void *obs, void *stream)
{
    if (!plan_dev || !field || !obs || nobs < 1 || nuniq < 1 || npts < 1) return RF_E_ARG;
    if (prec != RF_FP32 && prec != RF_FP64) return RF_E_ARG;
    if (reinterpret_cast<uintptr_t>(plan_dev) % 256) return RF_E_ARG;
    const Layout L = obs_layout(nobs, nuniq);
    const char *p = static_cast<const char *>(plan_dev);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned nb = (unsigned)((nobs + 255) / 256);
    const int32_t *idx = reinterpret_cast<const int32_t *>(p + L.off_idx);
    const double *w = reinterpret_cast<const double *>(p + L.off_w);
    const ObsPlanHeader *hd = static_cast<const ObsPlanHeader *>(plan_dev);
    if (prec == RF_FP32)
        k_obs_apply<float><<<nb, 256, 0, st>>>(hd, idx, w, (const float *)field, (float *)obs, nobs, nuniq, npts);
    else
        k_obs_apply<double><<<nb, 256, 0, st>>>(hd, idx, w, (const double *)field, (double *)obs, nobs, nuniq, npts);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_obs_adjoint(const void *plan_dev, int32_t nobs, int32_t nuniq, int64_t npts, rf_prec prec,
                              const void *obs, void *field, void *stream)
{
    if (!plan_dev || !field || !obs || nobs < 1 || nuniq < 1 || npts < 1) return RF_E_ARG;
    if (prec != RF_FP32 && prec != RF_FP64) return RF_E_ARG;
    if (reinterpret_cast<uintptr_t>(plan_dev) % 256) return RF_E_ARG;
    const Layout L = obs_layout(nobs, nuniq);
    const char *p = static_cast<const char *>(plan_dev);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int32_t *upt = reinterpret_cast<const int32_t *>(p + L.off_upt);
    const int32_t *uptr = reinterpret_cast<const int32_t *>(p + L.off_uptr);
    const int32_t *ent = reinterpret_cast<const int32_t *>(p + L.off_ent);
    const double *w = reinterpret_cast<const double *>(p + L.off_w);
    const unsigned nf = (unsigned)std::min<long>((npts + 255) / 256, 8192);
    const unsigned nb = (unsigned)((nuniq + 255) / 256);
    const ObsPlanHeader *hd = static_cast<const ObsPlanHeader *>(plan_dev);
    const long es = prec == RF_FP32 ? 4 : 8;
    const long nv = reinterpret_cast<uintptr_t>(field) % 16 ? 0 : npts * es / 16;
    if (prec == RF_FP32) {
        k_fill<float><<<nf, 256, 0, st>>>((float *)field, npts, nv, hd, nobs, nuniq);
        k_obs_adjoint<float><<<nb, 256, 0, st>>>(hd, upt, uptr, ent, w, (const float *)obs, (float *)field, nobs,
                                                 nuniq, npts);
    } else {
        k_fill<double><<<nf, 256, 0, st>>>((double *)field, npts, nv, hd, nobs, nuniq);
        k_obs_adjoint<double><<<nb, 256, 0, st>>>(hd, upt, uptr, ent, w, (const double *)obs, (double *)field, nobs,
                                                  nuniq, npts);
    }
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf_obs_innovation(const void *plan_dev, int32_t nobs, int32_t nuniq, int64_t npts, rf_prec prec,
                                 const void *field, const void *yobs, const void *rinv, double scale, void *d,
                                 void *rd, void *stream)
{
    if (!plan_dev || !rd || nobs < 1 || nuniq < 1 || npts < 1) return RF_E_ARG;
    if (prec != RF_FP32 && prec != RF_FP64) return RF_E_ARG;
    if (reinterpret_cast<uintptr_t>(plan_dev) % 256) return RF_E_ARG;
    const Layout L = obs_layout(nobs, nuniq);
    const char *p = static_cast<const char *>(plan_dev);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned nb = (unsigned)((nobs + 255) / 256);
    const int32_t *idx = reinterpret_cast<const int32_t *>(p + L.off_idx);
    const double *w = reinterpret_cast<const double *>(p + L.off_w);
    const ObsPlanHeader *hd = static_cast<const ObsPlanHeader *>(plan_dev);
    if (prec == RF_FP32)
        k_obs_innov<float><<<nb, 256, 0, st>>>(hd, idx, w, (const float *)field, (const float *)yobs,
                                               (const float *)rinv, (float)scale, (float *)d, (float *)rd, nobs,
                                               nuniq, npts);
    else
        k_obs_innov<double><<<nb, 256, 0, st>>>(hd, idx, w, (const double *)field, (const double *)yobs,
                                                (const double *)rinv, scale, (double *)d, (double *)rd, nobs,
                                                nuniq, npts);
    return hipGetLastError() == hipSuccess ? RF_OK : RF_E_HIP;
}
