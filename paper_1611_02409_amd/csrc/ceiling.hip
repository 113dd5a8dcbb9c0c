// Measured bandwidth ceiling of the step kernels' access pattern: an in-place
// read-modify-write stream over 74 planes, with no collision arithmetic.
#include <vector>

#include "runtime.hpp"

namespace esbgk {
namespace {

template <int NP>
__global__ __launch_bounds__(256) void k_stream_rw(char *p, uint32_t ncell, uint32_t set_bytes) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const Sets R(p, p + set_bytes, ncell * 4u, set_bytes);
    float v[NP];
#pragma unroll
    for (int i = 0; i < NP; i++) v[i] = ld<ST_F32>(i < NP / 2 ? R.f : R.g, c * 4u, R.so(i % (NP / 2)));
    float s = 0;
#pragma unroll
    for (int i = 0; i < NP; i++) s += v[i];
#pragma unroll
    for (int i = 0; i < NP; i++) st<ST_F32>(v[i] + s * 1e-30f, i < NP / 2 ? R.f : R.g, c * 4u, R.so(i % (NP / 2)));
}

}  // namespace
}  // namespace esbgk

using namespace esbgk;

extern "C" int esbgk_stream_ceiling(int64_t cells, int reps, double *gbps) {
    clear_error();
    if (cells < 256 || cells > (int64_t)14000000 * 2 || reps < 1 || !gbps) {
        set_error("need 256 <= cells <= 2.8e7, reps >= 1 and gbps");
        return ESBGK_EINVAL;
    }
    const uint32_t n = (uint32_t)cells;
    const uint32_t set_bytes = 37u * n * 4u;
    char *p = nullptr;
    ESBGK_HIP(hipMalloc(&p, 2ull * set_bytes));
    hipEvent_t e0, e1;
    int rc = ESBGK_OK;
    if (hipMemset(p, 0, 2ull * set_bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        set_error("setup failed");
        (void)hipFree(p);
        return ESBGK_EDEVICE;
    }
    const uint32_t nb = (n + 255) / 256;
    for (int w = 0; w < 2; w++) k_stream_rw<74><<<nb, 256>>>(p, n, set_bytes);
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; r++) k_stream_rw<74><<<nb, 256>>>(p, n, set_bytes);
    (void)hipEventRecord(e1, nullptr);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        set_error("stream kernel failed");
        rc = ESBGK_EDEVICE;
    } else {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        *gbps = 2.0 * 2.0 * set_bytes * reps / (ms * 1e-3) / 1e9;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(p);
    return rc;
}
