// Batched application of V_H (or its adjoint) to many grids in one go: the
// fields, levels and uneven grids of all items become one work list of x rows
// and y column blocks, run by one work-list launch per occupancy class of the
// x tile sizes and one for all y units.  The work list ("plan") is built on the host from the items and
// the block layout alone; the caller copies it to device memory once.  Items
// whose mask or sigma vary with level, and items with periodic rows or exact
// ends, are applied one by one (rf3_run).
#include <algorithm>
#include <map>
#include <string.h>
#include <vector>

#include "rf3_internal.h"
#include "sweeps.h"

using namespace rf;

namespace {

constexpr uint32_t kPlanMagic = 0x50424652u;   // "RFBP"
constexpr uint32_t kPlanVersion = 3;
// default planes per y work unit: the unit's setup (transfer matrices into
// LDS) is shared by this many planes of its column block
constexpr int kYPlanesPerUnit = 8;
// default cap on the workgroups that share one x row of an item
constexpr int kXGroupsMax = 8;

struct Tuning {
    int x_groups_max, y_planes, x_one;
};

// the work-list shape: defaults for zero fields; false on values out of range
bool tuning_of(const rf_batch_tuning *t, Tuning &o)
{
    o = Tuning{kXGroupsMax, kYPlanesPerUnit, 0};
    if (!t) return true;
    if (t->x_groups_max < 0 || t->x_groups_max > 64 || t->y_planes < 0 || t->y_planes > 4096) return false;
    if (t->x_one_launch != 0 && t->x_one_launch != 1) return false;
    if (t->x_groups_max) o.x_groups_max = t->x_groups_max;
    if (t->y_planes) o.y_planes = t->y_planes;
    o.x_one = t->x_one_launch;
    return true;
}

struct PlanHeader {
    uint32_t magic, version;
    int32_t n_items, n_units;
    uint64_t off_entries, off_units, total_bytes;
    uint64_t pad[3];
};
static_assert(sizeof(PlanHeader) == 64, "plan header size");

struct Group {
    int dir, L, offset, count;
};

struct HostPlan {
    std::vector<BatchEntry> entries;
    std::vector<BatchUnit> units;
    std::vector<Group> groups;   // x groups first, then y groups
    std::vector<int> seq_items;  // items for the line-sequential path
    size_t off_entries = 0, off_units = 0, total_bytes = 0;
};

template <class T>
T *at(const void *base, uint64_t off)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(const_cast<void *>(base)) + off);
}

// Units of one cluster share data (a row's coefficients, a column block's
// tables); they get block ids of one residue mod 8, i.e. one XCD and its L2.
void emit_xcd(const std::vector<std::vector<BatchUnit>> &clusters, std::vector<BatchUnit> &out)
{
    std::vector<BatchUnit> q[8];
    for (const auto &c : clusters) {
        int best = 0;
        for (int x = 1; x < 8; ++x)
            if (q[x].size() < q[best].size()) best = x;
        q[best].insert(q[best].end(), c.begin(), c.end());
    }
    size_t len = 0;
    for (auto &v : q) len = std::max(len, v.size());
    for (size_t i = 0; i < len; ++i)
        for (int x = 0; x < 8; ++x) out.push_back(i < q[x].size() ? q[x][i] : BatchUnit{-1, 0, 0, 0});
}

int build(const rf_batch_item *items, int32_t n, const rf_batch_tuning *tuning, HostPlan &P)
{
    Tuning tu;
    if (!items || n < 1 || !tuning_of(tuning, tu)) return RF_E_ARG;
    std::map<int, std::vector<std::vector<BatchUnit>>> xc, yc;   // tile size -> clusters
    P.entries.assign(n, BatchEntry{});
    const bool seq_all = force_sequential();
    for (int i = 0; i < n; ++i) {
        const rf_batch_item &it = items[i];
        if (!it.g) return RF_E_ARG;
        const rf_grid *g = it.g;
        const int rc = check_apply(g, it.coef, RF_FP32, it.in, it.out, g->nlev, it.nfields);
        if (rc) return rc;
        const BlockHeader h = layout(g);
        const long nplanes = (long)g->nlev * it.nfields;
        BatchEntry &e = P.entries[i];
        e.in = static_cast<const float *>(it.in);
        e.out = static_cast<float *>(it.out);
        e.nx = g->nx;
        e.ny = g->ny;
        e.nplanes = (int32_t)nplanes;
        // periodic rows and exact ends: the per-item path (rf3_run) runs their own kernels
        const bool tiled = !seq_all && g->flags == 0 && g->mask_nlev == 1 && g->sigma_nlev == 1 && h.lx && h.ly &&
                           (long)g->nx * g->ny * 16 < (1L << 31);
        if (!tiled) {
            P.seq_items.push_back(i);
            continue;
        }
        for (int d = 0; d < 2; ++d) e.T[d] = at<const float4>(it.coef, h.off_f32[d]);
        e.KY = at<const float>(it.coef, h.off_ky);
        e.LM[0] = at<const uint64_t>(it.coef, h.off_lmx);
        e.LM[1] = at<const uint64_t>(it.coef, h.off_lmy);
        e.PHI[0] = at<const float>(it.coef, h.off_phix);
        e.PHI[1] = at<const float>(it.coef, h.off_phiy);
        // x: one cluster per row, its `groups` units take interleaved planes
        const int groups = x_groups(g->ny, (int)nplanes, tu.x_groups_max);
        auto &xl = xc[h.lx];
        for (int r = 0; r < g->ny; ++r) {
            std::vector<BatchUnit> c;
            for (int k = 0; k < groups; ++k) c.push_back(BatchUnit{i, r, k, groups});
            xl.push_back(std::move(c));
        }
        // y: one cluster per column block, units of up to tu.y_planes planes [b, c)
        const int nblk = (g->nx + kYCols - 1) / kYCols;
        auto &yl = yc[h.ly];
        for (int b = 0; b < nblk; ++b) {
            std::vector<BatchUnit> c;
            for (long p0 = 0; p0 < nplanes; p0 += tu.y_planes)
                c.push_back(BatchUnit{i, b, (int)p0, (int)std::min<long>(nplanes, p0 + tu.y_planes)});
            yl.push_back(std::move(c));
        }
    }
    // x groups per tile size, largest first; the groups of one occupancy class
    // run in one launch
    for (auto it = xc.rbegin(); it != xc.rend(); ++it) {
        const int off = (int)P.units.size();
        emit_xcd(it->second, P.units);
        P.groups.push_back(Group{0, it->first, off, (int)P.units.size() - off});
    }
    // y groups from the largest tile size down: their units run in one launch,
    // and the short units of small tiles fill its last round
    for (auto it = yc.rbegin(); it != yc.rend(); ++it) {
        const int off = (int)P.units.size();
        emit_xcd(it->second, P.units);
        P.groups.push_back(Group{1, it->first, off, (int)P.units.size() - off});
    }
    if (P.units.size() > (size_t)INT32_MAX / 2) return RF_E_SHAPE;
    P.off_entries = sizeof(PlanHeader);
    P.off_units = (P.off_entries + P.entries.size() * sizeof(BatchEntry) + 255) & ~size_t(255);
    P.total_bytes = (P.off_units + P.units.size() * sizeof(BatchUnit) + 255) & ~size_t(255);
    return RF_OK;
}

}  // namespace

extern "C" size_t rf3_batch_plan_bytes_ex(const rf_batch_item *items, int32_t n, const rf_batch_tuning *t)
{
    HostPlan P;
    if (build(items, n, t, P) != RF_OK) return 0;
    return P.total_bytes;
}

extern "C" size_t rf3_batch_plan_bytes(const rf_batch_item *items, int32_t n)
{
    return rf3_batch_plan_bytes_ex(items, n, nullptr);
}

extern "C" int rf3_batch_plan_ex(const rf_batch_item *items, int32_t n, const rf_batch_tuning *t, void *plan,
                                 size_t plan_bytes)
{
    HostPlan P;
    const int rc = build(items, n, t, P);
    if (rc) return rc;
    if (!plan || plan_bytes != P.total_bytes) return RF_E_ARG;
    memset(plan, 0, plan_bytes);
    PlanHeader hd{};
    hd.magic = kPlanMagic;
    hd.version = kPlanVersion;
    hd.n_items = n;
    hd.n_units = (int32_t)P.units.size();
    hd.off_entries = P.off_entries;
    hd.off_units = P.off_units;
    hd.total_bytes = P.total_bytes;
    memcpy(plan, &hd, sizeof(hd));
    memcpy(at<char>(plan, P.off_entries), P.entries.data(), P.entries.size() * sizeof(BatchEntry));
    if (!P.units.empty()) memcpy(at<char>(plan, P.off_units), P.units.data(), P.units.size() * sizeof(BatchUnit));
    return RF_OK;
}

extern "C" int rf3_batch_plan(const rf_batch_item *items, int32_t n, void *plan, size_t plan_bytes)
{
    return rf3_batch_plan_ex(items, n, nullptr, plan, plan_bytes);
}

extern "C" int rf3_apply_batch_ex(const rf_batch_item *items, int32_t n, const rf_batch_tuning *t, rf_prec prec,
                                  int32_t adjoint, const void *plan_dev, size_t plan_bytes, void *stream)
{
    const bool adj = adjoint != 0;
    Tuning tu;
    if ((prec != RF_FP32 && prec != RF_FP64) || !tuning_of(t, tu)) return RF_E_ARG;
    if (prec == RF_FP64) {   // no FP64 tiled kernels: one application per item
        if (!items || n < 1) return RF_E_ARG;
        for (int i = 0; i < n; ++i) {
            if (!items[i].g) return RF_E_ARG;
            const int rc = check_apply(items[i].g, items[i].coef, prec, items[i].in, items[i].out, items[i].g->nlev,
                                       items[i].nfields);
            if (rc) return rc;
        }
        for (int i = 0; i < n; ++i) {
            const int rc = rf3_run(items[i].g, items[i].coef, prec, items[i].in, items[i].out, items[i].g->nlev,
                                   items[i].nfields, stream, adj);
            if (rc) return rc;
        }
        return RF_OK;
    }
    HostPlan P;
    const int rc = build(items, n, t, P);
    if (rc) return rc;
    if (!plan_dev || plan_bytes != P.total_bytes || reinterpret_cast<uintptr_t>(plan_dev) % 256) return RF_E_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const BatchEntry *E = at<const BatchEntry>(plan_dev, P.off_entries);
    const BatchUnit *U = at<const BatchUnit>(plan_dev, P.off_units);
    // the y groups follow the x groups in the work list, one after another
    int y_off = (int)P.units.size();
    for (const Group &gr : P.groups)
        if (gr.dir == 1) y_off = std::min(y_off, gr.offset);
    // forward: all x groups, then all y units reading the x output; adjoint: y first
    for (int pass = 0; pass < 2; ++pass) {
        const int dir = adj ? 1 - pass : pass;
        hipError_t e = hipSuccess;
        if (dir == 1) {
            e = fast_rf3_y_batch(E, U + y_off, (int)P.units.size() - y_off, adj, pass == 1, st);
        } else {
            // consecutive x groups of one occupancy class make one launch; with
            // x_one, all x groups (contiguous, largest tiles first) make one launch
            // of the largest class present
            for (size_t k = 0; k < P.groups.size() && e == hipSuccess;) {
                const Group &gr = P.groups[k];
                if (gr.dir != 0) { ++k; continue; }
                const int cls = x_batch_class(gr.L);
                int count = 0;
                for (; k < P.groups.size() && P.groups[k].dir == 0 &&
                       (tu.x_one || x_batch_class(P.groups[k].L) == cls);
                     ++k)
                    count += P.groups[k].count;
                e = fast_rf3_x_batch(E, U + gr.offset, count, cls, adj, pass == 1, tu.x_one != 0, st);
            }
        }
        if (e != hipSuccess) return RF_E_HIP;
    }
    for (int i : P.seq_items) {
        const int r = rf3_run(items[i].g, items[i].coef, prec, items[i].in, items[i].out, items[i].g->nlev,
                              items[i].nfields, stream, adj);
        if (r) return r;
    }
    return RF_OK;
}

extern "C" int rf3_apply_batch(const rf_batch_item *items, int32_t n, rf_prec prec, int32_t adjoint,
                               const void *plan_dev, size_t plan_bytes, void *stream)
{
    return rf3_apply_batch_ex(items, n, nullptr, prec, adjoint, plan_dev, plan_bytes, stream);
}
