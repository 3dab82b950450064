// Streaming-bandwidth diagnostic: the practical ceiling of an HBM-bound
// kernel on this device, measured as a plain copy that alternates between
// two buffers like the time step does (level n is read from the buffer the
// previous launch wrote), so that no launch finds its input in a cache.
#include "lbm3d_api_impl.h"

namespace lbm3d {

// One float4 per thread; the stores bypass the caches' allocation like the
// step kernel's.
__global__ void __launch_bounds__(256) k_stream_copy(const float4* __restrict__ a, float4* __restrict__ b, int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const float4 v = a[i];
    __builtin_nontemporal_store(v.x, &b[i].x);
    __builtin_nontemporal_store(v.y, &b[i].y);
    __builtin_nontemporal_store(v.z, &b[i].z);
    __builtin_nontemporal_store(v.w, &b[i].w);
}

}  // namespace lbm3d

using namespace lbm3d;

extern "C" int32_t lbm3d_stream_copy_rate(int64_t bytes, int32_t launches, double* gbs)
{
    if (bytes < 4096 || launches < 1 || !gbs) return LBM3D_E_INVAL;
    const int64_t n4 = bytes / 16;
    const size_t nb = (size_t)n4 * 16;
    void* a = nullptr;
    void* b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = nullptr;
    hipError_t e = hipMalloc(&a, nb);
    if (e == hipSuccess) e = hipMalloc(&b, nb);
    if (e == hipSuccess) e = hipMemset(a, 0, nb);
    if (e == hipSuccess) e = hipMemset(b, 0, nb);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const unsigned grid = (unsigned)((n4 + 255) / 256);
    auto pair = [&]() {
        hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, s, (const float4*)a, (float4*)b, n4);
        hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, s, (const float4*)b, (float4*)a, n4);
        return hipGetLastError();
    };
    for (int w = 0; w < 2 && e == hipSuccess; w++) e = pair();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int k = 0; k < launches && e == hipSuccess; k++) e = pair();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) *gbs = 2.0 * (double)nb * 2.0 * launches / ((double)ms * 1e-3) / 1e9;
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return e == hipSuccess ? LBM3D_OK : (e == hipErrorOutOfMemory ? LBM3D_E_NOMEM : LBM3D_E_DEVICE);
}
