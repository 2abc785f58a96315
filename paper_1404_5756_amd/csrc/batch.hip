// Batched application over many grids (placeholder).
#include "rf3_internal.h"
#include "sweeps.h"

extern "C" size_t rf3_batch_plan_bytes(const rf_batch_item *, int32_t) { return 0; }
extern "C" int rf3_batch_plan(const rf_batch_item *, int32_t, void *, size_t) { return RF_E_UNSUPPORTED; }
extern "C" int rf3_apply_batch(const rf_batch_item *, int32_t, rf_prec, int32_t, const void *, size_t, void *)
{
    return RF_E_UNSUPPORTED;
}
