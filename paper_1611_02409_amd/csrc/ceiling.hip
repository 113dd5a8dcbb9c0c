// Measured bandwidth ceiling of the step kernels' access patterns: the read
// and write streams of their planes (in place or between two buffers), no
// arithmetic.
#include <algorithm>
#include <vector>

#include "runtime.hpp"

namespace esbgk {
namespace {

// Reads NP planes of 4-byte values of each cell from src and writes them to
// dst (dst == src: in place, as A-A does; another buffer: as two-copy pull
// does).  The planes form NSET sets of NP / NSET planes (two sets: f and g
// stored apart; one set: FP16/BF16 (f, g) pairs, or a single population).
// `lds` bytes of dynamic LDS per work-group only limit how many work-groups
// share a CU (the pattern streams best at a few waves per SIMD); touch is 0.
// SCP: cache-policy bits of the stores (0 default, 2 non-temporal).
template <int NP, int NSET, int SCP>
__global__ __launch_bounds__(256) void k_stream_rw(char *src, char *dst, uint32_t ncell, uint32_t plane_bytes,
                                                   uint32_t set_bytes, int touch) {
    constexpr int PP = NP / NSET;
    static_assert(PP * NSET == NP && NSET <= 2, "planes split evenly over one or two sets");
    extern __shared__ float occupancy_lds[];
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const Sets R(src, NSET == 2 ? src + set_bytes : nullptr, plane_bytes, set_bytes);
    const Sets W(dst, NSET == 2 ? dst + set_bytes : nullptr, plane_bytes, set_bytes);
    float v[NP];
#pragma unroll
    for (int i = 0; i < NP; i++) v[i] = ld<ST_F32>(i < PP ? R.f : R.g, c * 4u, R.so(i % PP));
    float s = 0;
#pragma unroll
    for (int i = 0; i < NP; i++) s += v[i];
    if (touch) occupancy_lds[threadIdx.x] = s;
#pragma unroll
    for (int i = 0; i < NP; i++) st<ST_F32, SCP>(v[i] + s * 1e-30f, i < PP ? W.f : W.g, c * 4u, W.so(i % PP));
}

using StreamKernel = void (*)(char *, char *, uint32_t, uint32_t, uint32_t, int);

template <int NP, int NSET>
StreamKernel stream_kernel(int policy) {
    return policy ? k_stream_rw<NP, NSET, 2> : k_stream_rw<NP, NSET, 0>;
}

// The kernel for a (planes, sets) pattern the step kernels have, or null.
StreamKernel pick_stream_kernel(int planes, int sets, int policy) {
    if (sets == 2) {
        if (planes == 74) return stream_kernel<74, 2>(policy);   // D2Q37, FP32 f and g
        if (planes == 78) return stream_kernel<78, 2>(policy);   // D3Q39
        if (planes == 66) return stream_kernel<66, 2>(policy);   // D2Q33
    } else if (sets == 1) {
        if (planes == 37) return stream_kernel<37, 1>(policy);   // D2Q37, (f, g) pairs or f alone
        if (planes == 39) return stream_kernel<39, 1>(policy);   // D3Q39
        if (planes == 33) return stream_kernel<33, 1>(policy);   // D2Q33
    }
    return nullptr;
}

}  // namespace
}  // namespace esbgk

using namespace esbgk;

// Best of three placements of the pattern (in place on each of two buffers
// allocated one after the other, and a copy from one to the other: where a
// buffer lands in HBM moves such streams by a few per cent), of four
// occupancies (1, 2, 3 and up to 8 work-groups of 256 per CU), of two
// store policies (default and non-temporal, the two the step kernels use)
// and of two plane strides (unpadded, and 16 KiB of padding per plane).
extern "C" int esbgk_stream_ceiling_planes(int64_t cells, int planes, int sets, int reps, double *gbps) {
    clear_error();
    if (!pick_stream_kernel(planes, sets, 0)) {
        set_error("no stream pattern of %d planes in %d sets (74, 78, 66 in two sets; 37, 39, 33 in one)", planes,
                  sets);
        return ESBGK_EINVAL;
    }
    const int pp = planes / sets;
    if (cells < 256 || (uint64_t)pp * ((uint64_t)cells * 4 + 16384) >= ((uint64_t)1 << 32) || reps < 1 || !gbps) {
        set_error("need 256 <= cells, a set of at most 4 GiB, reps >= 1 and gbps");
        return ESBGK_EINVAL;
    }
    const uint32_t n = (uint32_t)cells;
    const uint64_t data_bytes = (uint64_t)planes * n * 4u;         // all planes' values
    const uint64_t alloc_set = (uint64_t)pp * (n * 4ull + 16384);   // room for the padded layout
    char *p[2] = {nullptr, nullptr};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ESBGK_OK;
    for (int k = 0; k < 2 && rc == ESBGK_OK; k++) {
        if (hipMalloc(&p[k], sets * alloc_set) != hipSuccess || hipMemset(p[k], 0, sets * alloc_set) != hipSuccess) {
            set_error("allocation of the stream buffers failed");
            rc = ESBGK_ENOMEM;
        }
    }
    if (rc == ESBGK_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        set_error("event creation failed");
        rc = ESBGK_EDEVICE;
    }
    const uint32_t nb = (n + 255) / 256;
    double best = 0;
    // LDS per CU is 160 KiB: a work-group asking for a bit over 160/(k+1) KiB
    // leaves room for at most k of them
    const size_t lds_for[4] = {96 * 1024, 60 * 1024, 44 * 1024, 0};
    for (uint32_t pad : {0u, 16384u}) {
        const uint32_t plane = n * 4u + pad, set_bytes = (uint32_t)pp * plane;
        for (int pass = 0; pass < 3 && rc == ESBGK_OK; pass++) {
            char *src = p[pass == 1 ? 1 : 0], *dst = p[pass == 0 ? 0 : 1];
            for (int pol = 0; pol < 2 && rc == ESBGK_OK; pol++) {
                const StreamKernel kern = pick_stream_kernel(planes, sets, pol);
                for (size_t lds : lds_for) {
                    for (int w = 0; w < 2; w++) kern<<<nb, 256, lds>>>(src, dst, n, plane, set_bytes, 0);
                    (void)hipEventRecord(e0, nullptr);
                    for (int r = 0; r < reps; r++) kern<<<nb, 256, lds>>>(src, dst, n, plane, set_bytes, 0);
                    (void)hipEventRecord(e1, nullptr);
                    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        set_error("stream kernel failed");
                        rc = ESBGK_EDEVICE;
                        break;
                    }
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    best = std::max(best, 2.0 * data_bytes * reps / (ms * 1e-3) / 1e9);
                }
            }
        }
    }
    if (rc == ESBGK_OK) *gbps = best;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (char *q : p)
        if (q) (void)hipFree(q);
    return rc;
}

// The pattern of the FP32 D2Q37 step with both populations.
extern "C" int esbgk_stream_ceiling(int64_t cells, int reps, double *gbps) {
    clear_error();
    if (cells > (int64_t)28000000) {
        set_error("need 256 <= cells <= 2.8e7, reps >= 1 and gbps");
        return ESBGK_EINVAL;
    }
    return esbgk_stream_ceiling_planes(cells, 74, 2, reps, gbps);
}
