// Batched step over many solves (placeholder until the persistent kernel lands).
#include "lbm3d_api_impl.h"

extern "C" int32_t lbm3d_batch_step(lbm3d_t* hs, int32_t count, const int64_t* nsteps)
{
    if (!hs || !nsteps || count < 1) return LBM3D_E_INVAL;
    for (int32_t k = 0; k < count; k++) {
        if (!hs[k] || nsteps[k] < 0) return LBM3D_E_INVAL;
        int32_t rc = lbm3d_step(hs[k], nsteps[k]);
        if (rc) return rc;
    }
    for (int32_t k = 0; k < count; k++) {
        int32_t rc = lbm3d_sync(hs[k]);
        if (rc) return rc;
    }
    return LBM3D_OK;
}
