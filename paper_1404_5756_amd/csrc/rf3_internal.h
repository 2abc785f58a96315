// Internal layout of the coefficient block and helpers shared by the librf3
// sources.  Not part of the public ABI (include/rf3.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rf3.h"

namespace rf {

constexpr uint32_t kMagic = 0x52463321u;   // "RF3!"
constexpr uint32_t kVersion = 5;
constexpr size_t kHeaderBytes = 512;         // the tables start here

// Per-point coast code bits (one byte per point and direction).
enum : uint8_t {
    CODE_SEA = 1,      // sea point: input read, output written
    CODE_FRESET = 2,   // state is zero before this point in the ascending sweep
                       // (first point of a segment, or a point outside every segment)
    CODE_BRESET = 4,   // state is zero before this point in the descending sweep
                       // (last point of a segment, or outside every segment)
    CODE_ACTIVE = 8,   // sea or imaginary point (inside a segment)
};

// lane-mask slabs of the tiled kernels: FRESET, BRESET, not-SEA, segment end (ACTIVE and BRESET)
constexpr int kLaneMasks = 4;

// Tables per direction (0 = x, 1 = y).  Element index of every per-point table
// is (level * ny + y) * nx + x, where level is the sigma level for coefficient
// tables and the mask level for code tables.
struct BlockHeader {
    uint32_t magic, version;
    rf_grid g;
    uint64_t npts_c;          // sigma_nlev * ny * nx
    uint64_t npts_m;          // mask_nlev * ny * nx
    // FP32, forward:  (beta, gamma, c2, c3) with gamma = 1 - (a1+a2+a3), c2 = a2+a3, c3 = a3
    uint64_t off_f32[2];
    // FP32, adjoint ascending sweep: (beta, Ga, C2a, C3a) built from alpha_{j-k,k}
    uint64_t off_a32[2];
    // FP32, adjoint descending sweep: (beta, Gd, C2d, C3d) built from alpha_{j+k,k}
    uint64_t off_d32[2];
    // FP64, printed form: (beta, alpha1, alpha2, alpha3)
    uint64_t off_f64[2];
    // FP64 1st-RF: (alpha, beta)
    uint64_t off_r1[2];
    // uint8 coast codes
    uint64_t off_code[2];
    uint64_t total_bytes;
    int32_t sigma_error;      // device-written: number of active points with invalid sigma
    int32_t pad[3];
    // lane-mask tables of the tiled FP32 kernels (0 when the shape is not tiled)
    int32_t lx, ly;           // points per lane along x (64 lanes per row), per wave along y (16 waves)
    uint64_t off_lmx;         // uint64 [mask_nlev][ny][kLaneMasks][lxp]: FRESET, BRESET, not-SEA, end; bit c = chunk c
    uint64_t off_lmy;         // uint64 [mask_nlev][nblk][kLaneMasks][lys]: bit j = column 64*blk + j, entry 8+r = row r
    // per coefficient level (coef_levels: one, or nlev when the mask or sigma depends on depth):
    uint64_t off_phiy;        // float [clev][nblk][4][16][64][12]: y-chunk transfer matrices
    uint64_t off_phix;        // float [clev][ny][4][64][12]: x-chunk transfer matrices
    uint64_t off_ky;          // float [clev][4][ny][nx][3]: y local-pass K vectors
    // RF_PERIODIC_X (0 otherwise):
    uint64_t off_perx;        // float [clev][ny][4][kPerXEntries][12]: cyclic scan of the tiled x kernel
    uint64_t off_perseq;      // double [sigma_nlev][ny][kPerSeq]: one-lap fixed points of the sequential kernels
    // RF_EXACT_ENDS (0 otherwise): 3x3 end matrices at segment ends, zero elsewhere
    uint64_t off_endd[2];     // double [end_nlev][ny][nx][2][9]: forward J M, adjoint M^T J^T (on p and z)
    uint64_t off_endf[2];     // float [end_nlev][ny][nx][3][12]: the FP32 paths' maps on increment-form
                              // states: forward J M D^-1, tiled adjoint M^T D^T, sequential adjoint
                              // M^T J^T D^-1 (a row-major 3x3 in the first 9 floats of each 12)
    int32_t end_nlev;         // max(mask_nlev, sigma_nlev) when RF_EXACT_ENDS
    int32_t pad2;
};
static_assert(sizeof(BlockHeader) <= kHeaderBytes, "header must fit before the tables");

// Cyclic scan of the tiled x kernel on periodic rows, per row and kind
// (0 forward ascending, 1 forward descending, 2 adjoint ascending, 3 adjoint
// descending), 12 floats (a row-major 3x3, padded) per entry:
//   entries 0..63: P_c, the transfer from the wrap state to the state entering
//     chunk c (ascending: Phi_{c-1}..Phi_0; descending: Phi_{c+1}..Phi_{c_last}
//     with the last real chunk c_last taken from its last real point on);
//   entry 64: W = (I - Phi_lap)^-1 (Phi_lap: one lap of the row's real points);
//   entry 65: ascending kinds, the transfer of chunk c_last up to the row's
//     last point (its steps past nx are padding).
constexpr int kPerXEntries = 66;
// One-lap fixed points of the line-sequential kernels on periodic rows, per
// (sigma level, row), doubles: W = (I - Phi_lap)^-1 for the FP64 printed form
// (4 kinds x 9), for the FP32 increment form (4 kinds x 9), and the 1st-RF's
// scalar 1 / (1 - prod alpha) (ascending, descending); padded to 76.
constexpr int kPerSeq = 76;
constexpr int kPerSeqDelta = 36, kPerSeqRf1 = 72;

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Tiling of the FP32 kernels.  x: one wave per row, 64 lanes each own a chunk
// of lx consecutive points (lx odd, so that a chunk-major LDS layout is free
// of bank conflicts).  y: 16 waves per block of 64 columns, each wave owns a
// chunk of ly consecutive rows; lane = column, two planes per lane when ly <= 45.
constexpr int kLxMax = 33, kLyMax = 64, kYWaves = 16, kYCols = 64;
__host__ __device__ inline int tile_lx(int nx)
{
    const int need = (nx + 63) / 64;
    if (need > kLxMax) return 0;
    return need | 1;
}
// batched x launches group the tile sizes by occupancy: the class is its
// largest tile size (the x kernels' registers and LDS grow with the tile)
__host__ __device__ constexpr int x_batch_class(int lx) { return lx <= 3 ? 3 : lx <= 11 ? 11 : lx <= 23 ? 23 : 33; }
// padded per-row length of the x lane-mask arrays (whole 8-entry blocks)
__host__ __device__ inline int lmx_stride(int lx) { return (lx + 7) & ~7; }
// per-column-block length of the y lane-mask arrays: 8 guard entries before row
// 0, 16*ly rows (whole 8-entry blocks) and 8 guard entries after
__host__ __device__ inline int lmy_stride(int ly) { return 16 * ((ly + 7) & ~7) + 16; }
__host__ __device__ inline int tile_ly(int ny)
{
    const int need = (ny + kYWaves - 1) / kYWaves;
    const int opts[] = {1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 28, 32, 36, 40, 45, 48, 56, 64};
    for (int o : opts)
        if (o >= need) return o;
    return 0;
}
__host__ __device__ constexpr int y_planes_per_lane(int ly) { return ly <= 45 ? 2 : 1; }

// levels of the tiled kernels' scan tables: the scan matrices of a line follow from
// its coefficients and its coast codes, so they depend on depth when either does
inline int coef_levels(const rf_grid *g) { return g->mask_nlev > g->sigma_nlev ? g->mask_nlev : g->sigma_nlev; }
inline long phix_level_floats(int ny) { return (long)ny * 4 * 64 * 12; }
inline long phiy_level_floats(int nx) { return (long)((nx + kYCols - 1) / kYCols) * 4 * kYWaves * kYCols * 12; }
inline long ky_level_floats(int nx, int ny) { return 4L * nx * ny * 3; }
inline long perx_level_floats(int ny) { return (long)ny * 4 * kPerXEntries * 12; }

// Depth-dependent tables of the tiled kernels: plane p of [nfields][nlev] has
// level p % nlev, and each table of that level starts this many elements after
// level 0's (0: one table serves every level).
struct LevTabs {
    int nlev;
    long t;      // float4 coefficients (sigma level)
    long lm;     // uint64 lane masks (mask level)
    long phi;    // float chunk transfer matrices (coefficient level)
    long ky;     // float y K vectors (coefficient level; y only)
    long end;    // float exact-end maps (coefficient level)
    long per;    // float cyclic-scan tables of periodic rows (coefficient level; x only)
};

// Batched FP32 application (batch.hip builds these on the host).  One entry per
// item with its buffers and the tables of both directions; one unit per
// workgroup: x {item, row, group, groups}, y {item, column block, first plane,
// end plane}; item < 0 marks an idle unit.
struct BatchEntry {
    const float *in;
    float *out;
    const float4 *T[2];
    const float *KY;
    const uint64_t *LM[2];
    const float *PHI[2];
    const float *PER;         // cyclic x scan tables (periodic rows), or null
    const float *END[2];      // exact-end maps of the tiled kernels, or null (unused: such items run per item)
    int32_t nx, ny, nplanes, pad;
};
struct BatchUnit {
    int32_t item, a, b, c;
};

// Geometry of one direction's lines inside a [nplanes][ny][nx] field stack.
struct LineGeom {
    int n;            // points per line
    int nlines;       // lines per plane (level)
    long estride;     // element stride along a line
    long lstride;     // stride between neighbouring lines
    long plane;       // nx * ny
    int nplanes;      // nfields * nlev planes to process
    int nlev;         // levels per field (plane index % nlev = level)
    int mask_per_lev; // 1: code tables have one plane per level; 0: a single 2-D plane
    int coef_per_lev; // same for coefficient tables
    int periodic;     // lines are cycles (periodic rows)
    const double *per;// periodic: one-lap fixed points [coefficient level][line][kPerSeq]
    const double *endd;  // exact ends: [end level][ny][nx][2][9] end matrices, or null
    const float *endf;   // exact ends: [end level][ny][nx][3][12] FP32 maps, or null
    int end_per_lev;     // the end tables have one plane per level
};

__host__ __device__ inline long plane_offset(const LineGeom &G, int pl, int per_lev)
{
    return per_lev ? (long)(pl % G.nlev) * G.plane : 0;
}

}  // namespace rf
