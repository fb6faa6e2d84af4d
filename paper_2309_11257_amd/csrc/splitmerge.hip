// Vertical splitting, per-cell merge and per-column cap.
#include "rt_internal.h"

rt_status do_split_merge(rt_ctx ctx, double alpha, int32_t nmax, int32_t mode, rt_stats *out)
{
    (void)alpha;
    (void)nmax;
    (void)mode;
    (void)out;
    return rt_fail(ctx, RT_E_UNSUPPORTED, "split/merge not built yet");
}
