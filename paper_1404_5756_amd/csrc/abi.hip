// C-ABI entry points of librf3: argument checks, then kernel launches on the
// caller's stream.  No call allocates memory or synchronises, except
// rf_coeffs (coef.hip), which reports invalid sigma.
#include <stdlib.h>
#include <string.h>

#include "rf3_internal.h"
#include "sweeps.h"

using namespace rf;

namespace {

LineGeom geom(const rf_grid *g, int dir, int nlev, int nfields, const void *coef)
{
    LineGeom G;
    G.n = dir == 0 ? g->nx : g->ny;
    G.nlines = dir == 0 ? g->ny : g->nx;
    G.estride = dir == 0 ? 1 : g->nx;
    G.lstride = dir == 0 ? g->nx : 1;
    G.plane = (long)g->nx * g->ny;
    G.nplanes = nlev * nfields;
    G.nlev = nlev;
    G.mask_per_lev = g->mask_nlev > 1;
    G.coef_per_lev = g->sigma_nlev > 1;
    G.periodic = dir == 0 && (g->flags & RF_PERIODIC_X);
    G.per = nullptr;
    G.endd = nullptr;
    G.endf = nullptr;
    G.end_per_lev = 0;
    if (g->flags) {
        const BlockHeader h = layout(g);
        if (G.periodic) G.per = reinterpret_cast<const double *>(reinterpret_cast<const char *>(coef) + h.off_perseq);
        if (h.end_nlev) {
            G.endd = reinterpret_cast<const double *>(reinterpret_cast<const char *>(coef) + h.off_endd[dir]);
            G.endf = reinterpret_cast<const float *>(reinterpret_cast<const char *>(coef) + h.off_endf[dir]);
            G.end_per_lev = h.end_nlev > 1;
        }
    }
    return G;
}

}  // namespace

int rf::check_apply(const rf_grid *g, const void *coef, int prec, const void *in, const void *out,
                    int nlev, int nfields)
{
    if (!g || !coef || !in || !out) return RF_E_ARG;
    if (prec != RF_FP32 && prec != RF_FP64) return RF_E_ARG;
    if (!grid_ok(g)) return RF_E_SHAPE;
    if (nlev < 1 || nlev > g->nlev || nfields < 1) return RF_E_SHAPE;
    if ((long long)nlev * nfields > (1ll << 30)) return RF_E_SHAPE;
    if (reinterpret_cast<uintptr_t>(coef) % 256) return RF_E_ARG;
    const size_t es = prec == RF_FP32 ? 4 : 8;
    if (reinterpret_cast<uintptr_t>(in) % es || reinterpret_cast<uintptr_t>(out) % es) return RF_E_ARG;
    if (in != out) {
        const size_t bytes = (size_t)g->nx * g->ny * (size_t)nlev * nfields * es;
        const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
        if (a < b + bytes && b < a + bytes) return RF_E_ARG;
    }
    return RF_OK;
}

namespace {

template <class T>
const T *tab(const void *coef, uint64_t off)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(coef) + off);
}

}  // namespace

// RF3_SEQUENTIAL=1 in the environment selects the line-sequential FP32 kernels
// (a cross-check of the tiled kernels); read at every call.
bool rf::force_sequential()
{
    const char *e = getenv("RF3_SEQUENTIAL");
    return e && e[0] == '1';
}

// One direction of the 3rd-RF in FP32 (forward when adj is false).  The tiled
// kernels take one 2-D mask and sigma for all levels, or per-level tables when
// either depends on depth; other cases (tile sizes not covered, periodic rows with
// exact ends along x) run the line-sequential kernels.
static hipError_t rf3_dir_f32(const rf_grid *g, const BlockHeader &h, const void *coef, int dir,
                              bool adj, const float *in, float *out, int nlev, int nfields,
                              hipStream_t st)
{
    const bool depth = g->mask_nlev > 1 || g->sigma_nlev > 1;
    const bool tiled = !force_sequential();
    const int nplanes = nlev * nfields;
    const long plane = (long)g->nx * g->ny;
    LevTabs lt{};
    lt.nlev = nlev;
    lt.t = g->sigma_nlev > 1 ? plane : 0;
    lt.lm = g->mask_nlev > 1 ? (dir == 0 ? (long)g->ny * kLaneMasks * lmx_stride(h.lx)
                                         : (long)((g->nx + kYCols - 1) / kYCols) * kLaneMasks * lmy_stride(h.ly))
                             : 0;
    lt.phi = depth ? (dir == 0 ? phix_level_floats(g->ny) : phiy_level_floats(g->nx)) : 0;
    lt.ky = depth ? ky_level_floats(g->nx, g->ny) : 0;
    lt.end = h.end_nlev > 1 ? plane * 36 : 0;
    lt.per = depth ? perx_level_floats(g->ny) : 0;
    const LevTabs *lv = depth ? &lt : nullptr;
    if (tiled && dir == 0 && h.lx) {
        const float *pert = h.off_perx ? tab<float>(coef, h.off_perx) : nullptr;
        const float *endt = h.off_endf[0] ? tab<float>(coef, h.off_endf[0]) : nullptr;
        hipError_t e = fast_rf3_x(in, out, tab<float4>(coef, h.off_f32[0]), tab<uint64_t>(coef, h.off_lmx),
                                  tab<float>(coef, h.off_phix), h.lx, g->nx, g->ny, nplanes, adj, pert, endt, lv,
                                  st);
        if (e != hipErrorNotSupported) return e;
    }
    if (tiled && dir == 1 && h.ly) {
        const float *endt = h.off_endf[1] ? tab<float>(coef, h.off_endf[1]) : nullptr;
        hipError_t e = fast_rf3_y(in, out, tab<float4>(coef, h.off_f32[1]), tab<float>(coef, h.off_ky),
                                  tab<uint64_t>(coef, h.off_lmy), tab<float>(coef, h.off_phiy), h.ly, g->nx, g->ny,
                                  nplanes, adj, endt, lv, st);
        if (e != hipErrorNotSupported) return e;
    }
    const LineGeom G = geom(g, dir, nlev, nfields, coef);
    const float4 *T1 = tab<float4>(coef, adj ? h.off_a32[dir] : h.off_f32[dir]);
    const float4 *T2 = tab<float4>(coef, adj ? h.off_d32[dir] : h.off_f32[dir]);
    return seq_rf3_f32(in, out, T1, T2, tab<uint8_t>(coef, h.off_code[dir]), G, adj, st);
}

static hipError_t rf3_dir(const rf_grid *g, const BlockHeader &h, const void *coef, rf_prec prec, int dir,
                          bool adj, const void *in, void *out, int nlev, int nfields, hipStream_t st)
{
    if (prec == RF_FP32)
        return rf3_dir_f32(g, h, coef, dir, adj, (const float *)in, (float *)out, nlev, nfields, st);
    return seq_rf3_f64((const double *)in, (double *)out, tab<double4>(coef, h.off_f64[dir]),
                       tab<uint8_t>(coef, h.off_code[dir]), geom(g, dir, nlev, nfields, coef), adj, st);
}

int rf::rf3_run(const rf_grid *g, const void *coef, rf_prec prec, const void *in, void *out,
                int32_t nlev, int32_t nfields, void *stream, bool adj)
{
    const int rc = check_apply(g, coef, prec, in, out, nlev, nfields);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const BlockHeader h = layout(g);
    // forward: x then y;  adjoint: y then x.  The second pass runs in place on out.
    const int d0 = adj ? 1 : 0, d1 = adj ? 0 : 1;
    hipError_t e = rf3_dir(g, h, coef, prec, d0, adj, in, out, nlev, nfields, st);
    if (e == hipSuccess) e = rf3_dir(g, h, coef, prec, d1, adj, out, out, nlev, nfields, st);
    return e == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf3_apply_dir(const rf_grid *g, const void *coef, rf_prec prec, int32_t dir, int32_t adjoint,
                             const void *in, void *out, int32_t nlev, int32_t nfields, void *stream)
{
    const int rc = check_apply(g, coef, prec, in, out, nlev, nfields);
    if (rc) return rc;
    if (dir != 0 && dir != 1) return RF_E_ARG;
    const BlockHeader h = layout(g);
    const hipError_t e = rf3_dir(g, h, coef, prec, dir, adjoint != 0, in, out, nlev, nfields,
                                 reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf3_apply_xy(const rf_grid *g, const void *coef, rf_prec prec, const void *in,
                            void *out, int32_t nlev, int32_t nfields, void *stream)
{
    return rf3_run(g, coef, prec, in, out, nlev, nfields, stream, false);
}

extern "C" int rf3_adjoint_xy(const rf_grid *g, const void *coef, rf_prec prec, const void *in,
                              void *out, int32_t nlev, int32_t nfields, void *stream)
{
    return rf3_run(g, coef, prec, in, out, nlev, nfields, stream, true);
}

extern "C" int rf1_apply_xy(const rf_grid *g, const void *coef, rf_prec prec, int32_t K,
                            const void *in, void *out, int32_t nlev, int32_t nfields, void *stream)
{
    const int rc = check_apply(g, coef, prec, in, out, nlev, nfields);
    if (rc) return rc;
    if (K != g->k1 || K < 1) return RF_E_ARG;
    if (prec != RF_FP64) return RF_E_UNSUPPORTED;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const BlockHeader h = layout(g);
    hipError_t e = hipSuccess;
    for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
        const LineGeom G = geom(g, dir, nlev, nfields, coef);
        const double2 *C = tab<double2>(coef, h.off_r1[dir]);
        const uint8_t *code = tab<uint8_t>(coef, h.off_code[dir]);
        for (int k = 0; k < K && e == hipSuccess; ++k) {
            const double *src = (dir == 0 && k == 0) ? (const double *)in : (const double *)out;
            e = seq_rf1_f64(src, (double *)out, C, code, G, k == 0, k == K - 1, st);
        }
    }
    return e == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" int rf1_apply_xy_fused(const rf_grid *g, const void *coef, rf_prec prec, int32_t K, const void *in,
                                  void *out, int32_t nlev, int32_t nfields, void *stream)
{
    const int rc = check_apply(g, coef, prec, in, out, nlev, nfields);
    if (rc) return rc;
    if (K != g->k1 || K < 1) return RF_E_ARG;
    const BlockHeader h = layout(g);
    if (g->mask_nlev != 1 || g->sigma_nlev != 1 || !h.lx || !h.ly || (g->flags & RF_PERIODIC_X))
        return RF_E_UNSUPPORTED;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nplanes = nlev * nfields;
    hipError_t e = fused_rf1(in, out, prec == RF_FP64, tab<double2>(coef, h.off_r1[0]), tab<uint64_t>(coef, h.off_lmx),
                             0, h.lx, g->nx, g->ny, nplanes, K, st);
    if (e == hipSuccess)
        e = fused_rf1(out, out, prec == RF_FP64, tab<double2>(coef, h.off_r1[1]), tab<uint64_t>(coef, h.off_lmy), 1,
                      h.ly, g->nx, g->ny, nplanes, K, st);
    if (e == hipErrorNotSupported) return RF_E_UNSUPPORTED;
    return e == hipSuccess ? RF_OK : RF_E_HIP;
}

extern "C" const char *rf_strerror(int status)
{
    switch (status) {
    case RF_OK: return "success";
    case RF_E_ARG: return "invalid argument (null pointer, bad enum or count, misaligned or overlapping buffers)";
    case RF_E_SHAPE: return "invalid grid or level/field count";
    case RF_E_SIGMA: return "sigma not positive and finite at a sea or imaginary point";
    case RF_E_HIP: return "HIP runtime error";
    case RF_E_UNSUPPORTED: return "request not supported by the library";
    default: return "unknown status";
    }
}
