// Device building blocks of the stencil kernels shared by the per-step kernels and the
// batched 2-D solver: one definition of each point update, so that a shot gives the same
// bits whichever kernel advances it.
#pragma once

#include "wv_internal.h"

namespace wv {

namespace {

constexpr int kNumXcd = 8;

__device__ __forceinline__ int xcd_remap(int bid, int nwg)
{
    // hardware dispatches workgroup i to XCD i % 8; give XCD j a contiguous range
    int xcd = bid % kNumXcd, loc = bid / kNumXcd;
    int q = nwg / kNumXcd, r = nwg % kNumXcd;
    return xcd * q + (xcd < r ? xcd : r) + loc;
}

__device__ __forceinline__ int layer_depth(int i, int lo, int hi)
{
    int a = lo - i, b = i - hi;
    return a > 0 ? a : (b > 0 ? b : 0);
}

__device__ __forceinline__ float damping(const Grid &g, int x, int y, int z)
{
    int dx = layer_depth(x, g.ix0[0], g.ix1[0]);
    int dy = layer_depth(y, g.ix0[1], g.ix1[1]);
    int dz = layer_depth(z, g.ix0[2], g.ix1[2]);
    return g.dampx * (float)(dx * dx) + g.dampy * (float)(dy * dy) + g.dampz * (float)(dz * dz);
}

// what a stencil launch does with the Laplacian (see stencil3d)
constexpr int kOT2 = 0, kLapW = 1, kOT4 = 2;

// One point (x, z) of the 2-D step, p its index.  q: the 2K+1 values of the marched
// field's column around z (q[K] the point itself); rowc: the point in the field's row z,
// staged with its K neighbours on either side (rowc[-K..K]).  MODE as for stencil3d:
//   kOT2: fout = c + ((1-a)(c - prev) + w L)/(1+a), in binary32 with the damping
//         division skipped where a = 0; GRAD adds gscale u^k (w L) to G in binary64;
//   kLapW: fout = w L;  kOT4: the second pass of an OT4 step.
// The Laplacian takes the k = 1 term from differences and the far terms as a plain sum
// folded once against the centre.
template <int K, bool GRAD, int MODE>
__device__ __forceinline__ void point2d(const Grid &g, const float *q, const float *rowc, int x, int z, long long p,
                                        const float *__restrict__ w, const float *prev, float *fout,
                                        const float *__restrict__ uk, const float *__restrict__ xtra,
                                        const float *__restrict__ xtra2, double *__restrict__ G, double gscale)
{
    const float c = q[K];
    float sx = g.cx[1] * ((rowc[1] - c) + (rowc[-1] - c));
    float sz = g.cz[1] * ((q[K + 1] - c) + (q[K - 1] - c));
    if constexpr (K > 1) {
        float fx = 0.0f, fz = 0.0f;
#pragma unroll
        for (int k = 2; k <= K; ++k) {
            fx = fmaf(g.cx[k], rowc[k] + rowc[-k], fx);
            fz = fmaf(g.cz[k], q[K + k] + q[K - k], fz);
        }
        sx += fmaf(-g.cf2[0], c, fx);
        sz += fmaf(-g.cf2[2], c, fz);
    }
    const float lap = sx + sz;
    const float wp = __builtin_nontemporal_load(&w[p]);
    if constexpr (MODE == kLapW) {
        __builtin_nontemporal_store(wp * lap, &fout[p]);
    } else {
        const float ctr = MODE == kOT4 ? __builtin_nontemporal_load(&xtra[p]) : c;
        const float wl = MODE == kOT4 ? fmaf(wp * (1.0f / 12.0f), lap, c) : wp * lap;
        const float a = damping(g, x, 0, z);
        const float d = ctr - __builtin_nontemporal_load(&prev[p]);
        const float dn = (a == 0.0f) ? d + wl : ((1.0f - a) * d + wl) / (1.0f + a);
        __builtin_nontemporal_store(ctr + dn, &fout[p]);
        if constexpr (GRAD && MODE == kOT4)
            G[p] += gscale * ((double)__builtin_nontemporal_load(&uk[p]) * (double)wl +
                              (double)c * (double)__builtin_nontemporal_load(&xtra2[p]) * (1.0 / 12.0));
        else if constexpr (GRAD)
            G[p] += gscale * (double)__builtin_nontemporal_load(&uk[p]) * (double)wl;
    }
}

// The 2-D march of one workgroup: the 256-wide x strip tix over rows [z0, z1), the
// column around each point in a register queue, the row with its x halo in LDS (row:
// 256 + 2K floats).  Every lane of the workgroup calls it (it holds barriers).
template <int K, bool GRAD, int MODE>
__device__ __forceinline__ void march2d(const Grid &g, const float *__restrict__ fin, const float *prev, float *fout,
                                        const float *__restrict__ w, const float *__restrict__ uk,
                                        const float *__restrict__ xtra, const float *__restrict__ xtra2,
                                        double *__restrict__ G, double gscale, int tix, int z0, int z1, float *row)
{
    constexpr int TX = 256;
    const int nx = g.nx, nz = g.nz;
    const int tid = threadIdx.x;
    const int x = tix * TX + tid;
    const bool in = x < nx;
    const float *col = fin + (in ? x : 0);
    float q[2 * K + 1];
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) {
        const int z = z0 - K + j;
        q[j] = (in && z >= 0 && z < nz) ? col[(long long)z * nx] : 0.0f;
    }
    for (int z = z0; z < z1; ++z) {
        const int zf = z + K;
        q[2 * K] = (in && zf < nz) ? col[(long long)zf * nx] : 0.0f;
        row[tid + K] = q[K];
        const float *plane = fin + (long long)z * nx;
        if (tid < K) {
            const int gl = tix * TX - K + tid;
            row[tid] = (gl >= 0 && gl < nx) ? plane[gl] : 0.0f;
            const int gr = tix * TX + TX + tid;
            row[TX + K + tid] = (gr < nx) ? plane[gr] : 0.0f;
        }
        __syncthreads();
        if (in)
            point2d<K, GRAD, MODE>(g, q, &row[tid + K], x, z, (long long)z * nx + x, w, prev, fout, uk, xtra, xtra2,
                                   G, gscale);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2 * K; ++j) q[j] = q[j + 1];
    }
}

// Source (or residual) injection at one unique point p of the scatter table entry i:
// fout[p] += w s / (1+a), s the weighted sum of its samples; GRAD adds the gradient term
// of the injected value.  (x, y, z): the point's coordinates.
template <bool GRAD>
__device__ __forceinline__ void inject_point(const Grid &g, const Sparse &sp, int i, int p, int x, int y, int z,
                                             const float *__restrict__ vals, const float *__restrict__ w,
                                             float *__restrict__ fout, const float *__restrict__ uk,
                                             double *__restrict__ G, long long pg, double gscale)
{
    float s = 0.0f;
    for (int e = sp.s_start[i]; e < sp.s_start[i + 1]; ++e) s = fmaf(sp.s_wt[e], vals[sp.s_col[e]], s);
    const float a = damping(g, x, y, z);
    const float wi = w[p] * s;
    const float inj = (a == 0.0f) ? wi : wi / (1.0f + a);
    fout[p] += inj;
    if constexpr (GRAD) G[pg] += gscale * (double)uk[p] * (double)wi;
}

// Receiver r of the gather table: (R f)_r.
__device__ __forceinline__ float gather_point(const Sparse &sp, int r, const float *__restrict__ f)
{
    float s = 0.0f;
    for (int c = 0; c < sp.nc; ++c) s = fmaf(sp.g_wt[r * sp.nc + c], f[sp.g_idx[r * sp.nc + c]], s);
    return s;
}

}  // namespace

}  // namespace wv
