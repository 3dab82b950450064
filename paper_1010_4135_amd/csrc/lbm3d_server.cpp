// Continuous-batching server (placeholder).
#include "lbm3d_api_impl.h"

extern "C" {
int32_t lbm3d_server_create(size_t, int32_t, lbm3d_server_t* out) { if (out) *out = nullptr; return LBM3D_E_STATE; }
int32_t lbm3d_server_submit(lbm3d_server_t, const lbm3d_params*, const double*, const double*, const double*,
                            const double*, const double*, int64_t, uint64_t*) { return LBM3D_E_STATE; }
int32_t lbm3d_server_poll(lbm3d_server_t, uint64_t, int32_t*) { return LBM3D_E_STATE; }
int32_t lbm3d_server_wait(lbm3d_server_t, uint64_t, double*, double*, double*, double*, double*, lbm3d_timing*) { return LBM3D_E_STATE; }
int32_t lbm3d_server_cancel(lbm3d_server_t, uint64_t) { return LBM3D_E_STATE; }
int32_t lbm3d_server_destroy(lbm3d_server_t) { return LBM3D_OK; }
}
