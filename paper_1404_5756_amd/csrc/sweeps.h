// Kernel launchers shared between the librf3 sources.
#pragma once
#include "rf3_internal.h"

namespace rf {

bool grid_ok(const rf_grid *g);
BlockHeader layout(const rf_grid *g);

// abi.hip: argument checks shared by the entry points, the RF3_SEQUENTIAL switch,
// and one whole V_H (or adjoint) application of one grid on a stream
int check_apply(const rf_grid *g, const void *coef, int prec, const void *in, const void *out, int nlev,
                int nfields);
bool force_sequential();
int rf3_run(const rf_grid *g, const void *coef, rf_prec prec, const void *in, void *out, int32_t nlev,
            int32_t nfields, void *stream, bool adj);

// line-sequential kernels (sweep_seq.hip)
hipError_t seq_rf3_f32(const float *in, float *out, const float4 *T1, const float4 *T2,
                       const uint8_t *code, const LineGeom &G, bool adj, hipStream_t st);
hipError_t seq_rf3_f64(const double *in, double *out, const double4 *C, const uint8_t *code,
                       const LineGeom &G, bool adj, hipStream_t st);
hipError_t seq_rf1_f64(const double *in, double *out, const double2 *C, const uint8_t *code,
                       const LineGeom &G, bool first, bool last, hipStream_t st);

}  // namespace rf

namespace rf {
// tiled FP32 kernels (sweep_fast.hip); hipErrorNotSupported when the tile size is not covered
// PERT: cyclic-scan tables of periodic rows, ENDT: exact-end tables (rf3_internal.h), or null;
// lv: per-level strides of depth-dependent tables (null: one table for every plane)
hipError_t fast_rf3_x(const float *in, float *out, const float4 *T, const uint64_t *LM, const float *PHI, int lx,
                      int nx, int ny, int nplanes, bool adj, const float *PERT, const float *ENDT, const LevTabs *lv,
                      hipStream_t st);
hipError_t fast_rf3_y(const float *in, float *out, const float4 *T, const float *KY, const uint64_t *LM,
                      const float *PHI, int ly, int nx, int ny, int nplanes, bool adj, const float *ENDT,
                      const LevTabs *lv, hipStream_t st);
// batched forms over a work list: x units of one launch share the occupancy
// class of their tile size (x_batch_class), or (all_classes) have any class up
// to cls; a y launch takes units of any tile size; each unit's tile size follows
// from its item's nx or ny
hipError_t fast_rf3_x_batch(const BatchEntry *E, const BatchUnit *U, int nunits, int cls, bool adj, bool src_out,
                            bool all_classes, hipStream_t st);
hipError_t fast_rf3_y_batch(const BatchEntry *E, const BatchUnit *U, int nunits, bool adj, bool src_out,
                            hipStream_t st);
int x_groups(int ny, int nplanes, int gmax);
hipError_t setup_phi_y(const float4 *T, const uint8_t *code, float *PHI, int nx, int ny, int ly, hipStream_t st);
hipError_t setup_ky_y(const float4 *T, const uint8_t *code, float *KY, int nx, int ny, int ly, hipStream_t st);
// fused 1st-RF (rf1_fast.hip): K iterations of one direction on chip; l = lx (dir 0) or ly (dir 1)
hipError_t fused_rf1(const void *in, void *out, bool fp64, const double2 *C, const uint64_t *LM, int dir, int l,
                     int nx, int ny, int nplanes, int K, hipStream_t st);
hipError_t setup_phi_x(const float4 *T, const uint8_t *code, float *PHI, int nx, int ny, int lx, hipStream_t st);
hipError_t setup_per_x(const float4 *T, const uint8_t *code, float *PER, int nx, int ny, int lx, hipStream_t st);
}  // namespace rf
