// A streaming kernel that measures the HBM ceiling of this device for the stencils'
// access mix: R nontemporal read streams and one nontemporal write stream of float4,
// four per lane in flight, over arrays far larger than the caches.  The benchmark
// prices its kernels against the published peak and reports this measured ceiling
// beside it.
#include "wv_internal.h"

namespace wv {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

template <int R>
__global__ __launch_bounds__(256) void stream_kernel(const f4v *__restrict__ in, f4v *__restrict__ out, long long n4)
{
    constexpr int U = 4;
    const long long stride = (long long)gridDim.x * 256 * U;
    for (long long i0 = blockIdx.x * 256LL * U + threadIdx.x; i0 < n4; i0 += stride) {
        f4v acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = min(i0 + 256LL * u, n4 - 1);
            acc[u] = __builtin_nontemporal_load(in + i);
#pragma unroll
            for (int r = 1; r < R; ++r) acc[u] += __builtin_nontemporal_load(in + (long long)r * n4 + i);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = i0 + 256LL * u;
            if (i < n4) __builtin_nontemporal_store(acc[u], out + i);
        }
    }
}

}  // namespace

}  // namespace wv

using namespace wv;

extern "C" int wv_stream_ceiling(int reads, size_t stream_bytes, void *ws, size_t ws_bytes, int reps, double *gbs,
                                 void *stream)
{
    if (reads < 1 || reads > 4 || reps < 1 || !gbs || !ws || (((uintptr_t)ws) & 255)) return WV_EINVAL;
    const long long n4 = (long long)(stream_bytes / 16);
    if (n4 < 1 || ws_bytes < (size_t)(reads + 1) * (size_t)n4 * 16) return WV_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const f4v *in = reinterpret_cast<const f4v *>(ws);
    f4v *out = reinterpret_cast<f4v *>(ws) + (long long)reads * n4;
    auto launch = [&]() -> hipError_t {
        const dim3 grid(8192), block(256);
        switch (reads) {
        case 1: hipLaunchKernelGGL(stream_kernel<1>, grid, block, 0, s, in, out, n4); break;
        case 2: hipLaunchKernelGGL(stream_kernel<2>, grid, block, 0, s, in, out, n4); break;
        case 3: hipLaunchKernelGGL(stream_kernel<3>, grid, block, 0, s, in, out, n4); break;
        default: hipLaunchKernelGGL(stream_kernel<4>, grid, block, 0, s, in, out, n4); break;
        }
        return hipGetLastError();
    };
    // inputs hold zeros (a fill kernel), so the sums stay finite
    hipError_t e = launch_fill_f32(reinterpret_cast<float *>(ws), (long long)(reads + 1) * n4 * 4, 0.0f, s);
    if (e != hipSuccess) return WV_EHIP;
    if ((e = launch()) != hipSuccess) return WV_EHIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return WV_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return WV_EHIP;
    }
    double best = 0.0;
    int rc = WV_OK;
    for (int r = 0; r < reps && rc == WV_OK; ++r) {
        float ms = 0.0f;
        if (hipEventRecord(e0, s) != hipSuccess || launch() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = WV_EHIP;
            break;
        }
        const double rate = (double)(reads + 1) * (double)n4 * 16.0 / (ms * 1e-3);
        best = rate > best ? rate : best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *gbs = best / 1e9;
    return rc;
}
