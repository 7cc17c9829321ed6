// A streaming kernel that measures the HBM ceiling of this device for the stencils'
// access mix: R read streams of float4, the first through the caches (as the stencils
// read their marched field) and the others nontemporal (their pointwise operands), and
// one nontemporal write stream, four loads per lane in flight, over arrays far larger
// than the caches.  The mix matters: on MI355X a 2-nontemporal + 1-cached read mix
// streams about a quarter faster than three nontemporal reads or three cached ones.
// The benchmark prices its kernels against the published peak and reports this
// measured ceiling beside it.
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
            acc[u] = in[i];
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

// Inputs of the streams: values in [0, 1) from a hash of the index, so that the sums
// stay finite and the arrays hold varied bits (on this chip a stream over zeros ran
// faster than the same stream over varied data).
__global__ void hash_fill_kernel(float *p, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        unsigned h = (unsigned)i * 2654435761u ^ (unsigned)(i >> 32);
        h ^= h >> 15;
        h *= 0x2c1b3c6du;
        h ^= h >> 12;
        p[i] = (float)(h & 0xffffffu) * (1.0f / 16777216.0f);
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
    hipLaunchKernelGGL(hash_fill_kernel, dim3(4096), dim3(256), 0, s, reinterpret_cast<float *>(ws),
                       (long long)(reads + 1) * n4 * 4);
    hipError_t e = hipGetLastError();
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
