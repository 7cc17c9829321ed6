// Stencil kernels of the forward and adjoint acoustic solver (gfx950, wave64).
//
// The discrete problem is eq. (7) of the paper with the OT2 (second order in time)
// leapfrog on two time levels, updated in place (u^{n+1} overwrites u^{n-1}):
//   u^{n+1} = [2u^n - (1-a)u^{n-1} + w(lap u^n + s^n)]/(1+a),   w = dt^2 c^2,
// so a step moves exactly three reads and one write per point.  It is evaluated as
//   u^{n+1} = u^n + [(1-a)(u^n - u^{n-1}) + w lap u^n]/(1+a)
// (the source term is added by the injection kernel): the small per-step change is
// formed first and added once, which keeps binary32 rounding near 5e-6 relative over
// thousands of steps.  The adjoint of the recursion has the same form run backward
// in time (lam^{k-1} overwrites lam^{k+1}) with the residual injected at the
// receivers; the gradient of the misfit with respect to m accumulates
// -(1/dt^2) u^k w (lap lam^k + R^T r^k), which equals
// -(1/dt^2) u^k [(1+a)lam^{k-1} - 2lam^k + (1-a)lam^{k+1}].
//
// Operands read or written once per step (u^{n-1}, w, u^k, the new level) use
// nontemporal loads and stores, so they stream past the caches and leave L2 to the
// centre field, whose halos are re-read by neighbouring tiles.  The binary64 gradient
// takes two 16-byte accesses per lane; it is cached normally, so that a line is
// fetched and written once although each access covers only half of it.
//
// Laplacian along one axis, in binary32 without the cancellation of a direct sum:
//   c_1 ((u_{+1} - u) + (u_{-1} - u)) + [sum_{k>=2} c_k (u_{+k} + u_{-k}) - 2 (sum_{k>=2} c_k) u].
// The dominant k = 1 term is formed from differences, which are small and nearly
// exact for smooth fields; the far weights are small (|c_k| <= 0.18 c_1 for k >= 2 at
// every order up to 16, falling fast), so their plain sum, folded once against u, adds only
// a fraction of an ulp of the result.  In a 3000-step binary32 run this matches the
// all-difference form (about 5e-6 against binary64; a direct sum of all terms loses
// about two digits) at 20 instead of 32 operations per axis for order 16.
//
// Workgroup ids are remapped so that every XCD (each has its own L2) receives a
// contiguous run of neighbouring tiles, whose halos then hit the same L2.
//
// Field arrays are pitched (rows of px >= nx elements, px a multiple of 32 in 3-D):
// a 32-wide tile row is then exactly one 128-byte line.  With a row length that is
// not a multiple of 32 (e.g. 400), every other tile row straddles two lines, which
// measured 10-15 % slower.  The binary64 gradient belongs to the caller and is dense.
#include <hip/hip_ext.h>

#include "wv_stencil_dev.h"

namespace wv {

namespace {


typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 ntload4(const float *p)
{
    const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
    return make_float4(t.x, t.y, t.z, t.w);
}

__device__ __forceinline__ void ntstore4(float *p, float a, float b, float c, float d)
{
    f4v t = {a, b, c, d};
    __builtin_nontemporal_store(t, reinterpret_cast<f4v *>(p));
}

// 3-D step.  A workgroup owns a 32 x 32 tile of the x-y plane and marches down z
// over a chunk of planes; each lane owns four consecutive x points of one row.
//   * z neighbours: a register queue of 2K+1 planes per point, shifted once per plane;
//   * x, y neighbours: the centre plane staged in LDS with its halos (x halo padded to
//     a multiple of four columns so that every LDS access is an aligned float4),
//     double buffered, one barrier per plane;
//   * software pipeline: the global loads a plane needs (its point operands, its
//     halo and the queue front K planes further on) are issued into a register
//     stage AHEAD planes before the plane is computed (two where a third stage fits
//     in the registers, else one);
//   * the halo of plane z+1 goes from its stage straight into the next LDS buffer;
//   * interior LDS values come from the queue, so HBM is read once per value
//     (plus the 2K-plane warm-up of each z chunk); halos are lines the neighbouring
//     tiles of the same XCD read as their interior.
// VEC: nx % 4 == 0, every float4 of a row is either inside or outside the grid.
// `prev` (u^{n-1}) and `fout` (u^{n+1}) may be the same array: each point of it is
// read and then written by the same lane only.
//
// MODE selects what is done with the Laplacian L of the marched field `fin`:
//   kOT2:  the OT2 step above: out = c + ((1-a)(c - prev) + w L)/(1+a), c = fin's
//          centre; GRAD adds gscale u^k (w L) to G.
//   kLapW: out = w L (the first pass of an OT4 step; no gradient).
//   kOT4:  the second pass of an OT4 step: fin is v = w lap u^n, the centre
//          c = u^n comes pointwise from xtra, and
//          out = c + ((1-a)(c - prev) + v + (w/12) L)/(1+a);
//          GRAD adds both OT4 gradient terms in one update,
//          gscale [u^k (v + (w/12) L) + v vu / 12], where vu = w lap u^k comes pointwise
//          from xtra2 (the second is the term of the m inside the OT4 operator).
// GM selects how the gradient term t = u^k (w L) of an OT2 step reaches G:
//   kGNone: no gradient;  kGAdd: G += gscale t;
//   kGCarryOut: cr = t rounded to binary32, G untouched;
//   kGCarryIn:  G += gscale (t + cr), cr from the kGCarryOut step before.
// A pair of adjoint steps thus reads and writes the binary64 gradient once.
template <int K, int GM, bool VEC, int MODE>
__global__ __launch_bounds__(256, 2) void stencil3d(const Grid g, const float *__restrict__ fin,
                                                 const float *prev, float *fout, const float *__restrict__ w,
                                                 const float *__restrict__ uk, const float *__restrict__ xtra,
                                                 const float *__restrict__ xtra2, double *__restrict__ G,
                                                 float *__restrict__ cr, double gscale, int tiles_x, int tiles_y,
                                                 int zchunks, int zlen)
{
    constexpr bool GRAD = GM != kGNone;                    // u^k is read
    constexpr bool GRW = GM == kGAdd || GM == kGCarryIn;    // G is read and written
    static_assert(!(GRAD && MODE == kLapW), "the w lap pass carries no gradient term");
    static_assert(MODE == kOT2 || GM == kGNone || GM == kGAdd, "carried gradient terms are OT2 only");
    constexpr int TX = 32, TY = 32;
    constexpr int HX = (K + 3) / 4 * 4;          // x halo columns (>= K, multiple of 4)
    constexpr int LX = TX + 2 * HX, LY = TY + 2 * K;
    constexpr int NXV = 1 + 2 * ((K + 3) / 4);   // float4 reads for the x neighbours
    constexpr int XC = 4 * ((K + 3) / 4);        // index of the lane's first point in them
    constexpr int NHX = 2 * TY * (HX / 4);        // x-halo float4s per plane
    constexpr int NH = NHX + 2 * K * (TX / 4);    // all halo float4s per plane (<= 256)
    static_assert(NH <= 256, "one halo float4 per lane at most");
    // planes between a stage's loads and its use: two where three stages fit in 256
    // registers without spilling (no gradient, aligned rows, not the OT4 update)
    constexpr int AHEAD = (!GRAD && VEC && MODE != kOT4) ? 2 : 1;
    __shared__ __align__(16) float tile[2][LY][LX];

    const int nwg = tiles_x * tiles_y * zchunks;
    const int lid = xcd_remap(blockIdx.x, nwg);
    const int tix = lid % tiles_x;
    const int tiy = (lid / tiles_x) % tiles_y;
    const int zc = lid / (tiles_x * tiles_y);
    const int z0 = zc * zlen;
    const int z1 = min(z0 + zlen, g.nz);

    const int tid = threadIdx.x;
    const int tx4 = tid & 7, ty = tid >> 3;
    const int nx = g.nx, ny = g.ny, nz = g.nz, px = g.px;
    const long long sxy = (long long)px * ny;     // pitched field plane
    const int x0 = tix * TX + 4 * tx4;
    const int y = tiy * TY + ty;
    const bool rowin = y < ny;
    const bool ptin = rowin && x0 < nx;
    const long long rowoff = (long long)(rowin ? y : 0) * px;

    // halo float4 of this lane: source in the plane and place in the tile
    int hrow = 0, hcol = 0, hgx = -1, hgy = -1;
    if (tid < NHX) {
        const int side = tid / (TY * (HX / 4));
        const int rem = tid - side * (TY * (HX / 4));
        const int r = rem / (HX / 4), c4 = rem - (rem / (HX / 4)) * (HX / 4);
        hrow = r + K;
        hcol = side ? (TX + HX + 4 * c4) : (4 * c4);
        hgx = tix * TX - HX + hcol;
        hgy = tiy * TY + r;
    } else if (tid < NH) {
        const int e = tid - NHX;
        const int side = e / (K * (TX / 4));
        const int rem = e - side * (K * (TX / 4));
        const int r = rem / (TX / 4), c4 = rem - (rem / (TX / 4)) * (TX / 4);
        hrow = side ? (TY + K + r) : r;
        hcol = HX + 4 * c4;
        hgx = tix * TX + 4 * c4;
        hgy = tiy * TY - K + hrow;
    }
    const bool hact = tid < NH && hgy >= 0 && hgy < ny;

    // Branch-free float4 load of (gx..gx+3, yy, z): the address is clamped into the
    // grid and the value zeroed outside, so every lane issues its load and no wait
    // is forced at a control-flow join (the pipeline depends on that).
    auto load4 = [&](const float *base, int z, int yy, int gx, bool ok) -> float4 {
        const bool in = ok && z >= 0 && z < nz && yy >= 0 && yy < ny;
        const int zc = min(max(z, 0), nz - 1), yc = min(max(yy, 0), ny - 1);
        const float *row = base + (long long)zc * sxy + (long long)yc * px;
        float4 v;
        if constexpr (VEC) {
            const bool inx = in && gx >= 0 && gx < nx;
            const float4 t = *reinterpret_cast<const float4 *>(row + min(max(gx, 0), nx - 4));
            v.x = inx ? t.x : 0.0f;
            v.y = inx ? t.y : 0.0f;
            v.z = inx ? t.z : 0.0f;
            v.w = inx ? t.w : 0.0f;
        } else {
            const float t0 = row[min(max(gx + 0, 0), nx - 1)], t1 = row[min(max(gx + 1, 0), nx - 1)];
            const float t2 = row[min(max(gx + 2, 0), nx - 1)], t3 = row[min(max(gx + 3, 0), nx - 1)];
            v.x = (in && gx + 0 >= 0 && gx + 0 < nx) ? t0 : 0.0f;
            v.y = (in && gx + 1 >= 0 && gx + 1 < nx) ? t1 : 0.0f;
            v.z = (in && gx + 2 >= 0 && gx + 2 < nx) ? t2 : 0.0f;
            v.w = (in && gx + 3 >= 0 && gx + 3 < nx) ? t3 : 0.0f;
        }
        return v;
    };

    struct Stage {
        float4 p, w, u, c, h, f, t;
        double g[GRW ? 4 : 1];
    };
    // loads that computing plane z needs: its point operands (with GRAD also u^k and
    // the gradient), the halo of plane z+1+K and the queue front of plane z+1+K
    // point operands feed only values stored under the same in-range predicate, so
    // they are loaded from the clamped address without zeroing
    auto load4p = [&](const float *base, int z, int gx) -> float4 {
        const int zc = min(z, nz - 1), yc = min(y, ny - 1);
        const float *row = base + (long long)zc * sxy + (long long)yc * px;
        if constexpr (VEC) return ntload4(row + min(gx, nx - 4));
        return make_float4(row[min(gx + 0, nx - 1)], row[min(gx + 1, nx - 1)], row[min(gx + 2, nx - 1)],
                           row[min(gx + 3, nx - 1)]);
    };
    auto fill = [&](Stage &S, int z) {
        if constexpr (MODE != kLapW) S.p = load4p(prev, z, x0);
        S.w = load4p(w, z, x0);
        if constexpr (MODE == kOT4) S.c = load4p(xtra, z, x0);
        if constexpr (GRAD) S.u = load4p(uk, z, x0);
        if constexpr (GM == kGCarryIn) S.t = load4p(cr, z, x0);
        if constexpr (GRW) {
            const long long pg = ((long long)min(z, nz - 1) * ny + min(y, ny - 1)) * nx;   // dense
            if constexpr (VEC) {
                // two 16-byte loads per lane, normally cached: the line a lane pair shares
                // stays in L2 between them
                const double2 g0 = *reinterpret_cast<const double2 *>(&G[pg + min(x0, nx - 4)]);
                const double2 g1 = *reinterpret_cast<const double2 *>(&G[pg + min(x0, nx - 4) + 2]);
                S.g[0] = g0.x; S.g[1] = g0.y; S.g[2] = g1.x; S.g[3] = g1.y;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) S.g[i] = G[pg + min(x0 + i, nx - 1)];
            }
        }
        const bool more = z + 1 < z1;
        S.h = load4(fin, z + 1, hgy, hgx, hact && more);
        S.f = load4(fin, z + 1 + K, y, x0, more && rowin);
    };

    // register queue: q[i][j] = u(x0+i, y, z-K+j)
    float q[4][2 * K + 1];
#pragma unroll
    for (int j = 0; j < 2 * K + 1; ++j) {
        const float4 v = load4(fin, z0 - K + j, y, x0, rowin);
        q[0][j] = v.x; q[1][j] = v.y; q[2][j] = v.z; q[3][j] = v.w;
    }
    Stage A, B, C;
    fill(A, z0);
    if constexpr (AHEAD == 2) fill(B, z0 + 1);
    {
        const float4 hv = load4(fin, z0, hgy, hgx, hact);
        *reinterpret_cast<float4 *>(&tile[0][ty + K][HX + 4 * tx4]) = make_float4(q[0][K], q[1][K], q[2][K], q[3][K]);
        if (tid < NH) *reinterpret_cast<float4 *>(&tile[0][hrow][hcol]) = hv;
    }
    __syncthreads();

    const float c1 = g.cy[0], c2 = g.cz[0];   // h_x^2/h_y^2, h_x^2/h_z^2
    auto step = [&](int z, Stage &S, Stage &N) {
        // the binary64 gradient of this plane arrived with the stage (clamped address,
        // no branch; only in-range lanes store the update)
        double gold[4] = {0.0, 0.0, 0.0, 0.0};
        if constexpr (GRW) {
#pragma unroll
            for (int i = 0; i < 4; ++i) gold[i] = S.g[i];
        }
        // OT4 adjoint: w lap u^k of this plane, loaded here rather than staged (a staged
        // copy would not fit the registers); the Laplacian below covers its latency
        float4 vu4 = make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (MODE == kOT4 && GRAD) vu4 = load4p(xtra2, z, x0);
        fill(N, z + AHEAD);
        const int cur = (z - z0) & 1;
        // x neighbours: NXV aligned float4 around the lane's four points
        float xr[4 * NXV];
        const float *trow = &tile[cur][ty + K][0];
#pragma unroll
        for (int v = 0; v < NXV; ++v) {
            const float4 t = *reinterpret_cast<const float4 *>(trow + HX + 4 * tx4 - XC + 4 * v);
            xr[4 * v + 0] = t.x; xr[4 * v + 1] = t.y; xr[4 * v + 2] = t.z; xr[4 * v + 3] = t.w;
        }
        // per axis: near (k = 1, differences) + far (k >= 2, plain sum) - cf2 * centre;
        // the 3-D kernel applies cx on every axis and scales y and z afterwards
        const float cf2 = g.cf2[0];
        float lap[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float c = q[i][K];
            float sx = g.cx[1] * ((xr[XC + i + 1] - c) + (xr[XC + i - 1] - c));
            float sz = g.cx[1] * ((q[i][K + 1] - c) + (q[i][K - 1] - c));
            if constexpr (K > 1) {
                float fx = 0.0f, fz = 0.0f;
#pragma unroll
                for (int k = 2; k <= K; ++k) {
                    fx = fmaf(g.cx[k], xr[XC + i + k] + xr[XC + i - k], fx);
                    fz = fmaf(g.cx[k], q[i][K + k] + q[i][K - k], fz);
                }
                sx += fmaf(-cf2, c, fx);
                sz += fmaf(-cf2, c, fz);
            }
            lap[i] = fmaf(c2, sz, sx);
        }
        float sy[4];
        {
            const float4 a = *reinterpret_cast<const float4 *>(&tile[cur][ty + K + 1][HX + 4 * tx4]);
            const float4 b = *reinterpret_cast<const float4 *>(&tile[cur][ty + K - 1][HX + 4 * tx4]);
            sy[0] = g.cx[1] * ((a.x - q[0][K]) + (b.x - q[0][K]));
            sy[1] = g.cx[1] * ((a.y - q[1][K]) + (b.y - q[1][K]));
            sy[2] = g.cx[1] * ((a.z - q[2][K]) + (b.z - q[2][K]));
            sy[3] = g.cx[1] * ((a.w - q[3][K]) + (b.w - q[3][K]));
        }
        if constexpr (K > 1) {
            float fy[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 2; k <= K; ++k) {
                const float4 a = *reinterpret_cast<const float4 *>(&tile[cur][ty + K + k][HX + 4 * tx4]);
                const float4 b = *reinterpret_cast<const float4 *>(&tile[cur][ty + K - k][HX + 4 * tx4]);
                fy[0] = fmaf(g.cx[k], a.x + b.x, fy[0]);
                fy[1] = fmaf(g.cx[k], a.y + b.y, fy[1]);
                fy[2] = fmaf(g.cx[k], a.z + b.z, fy[2]);
                fy[3] = fmaf(g.cx[k], a.w + b.w, fy[3]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) sy[i] += fmaf(-cf2, q[i][K], fy[i]);
        }
        // damping a = dampx dx^2 + dampy dy^2 + dampz dz^2; the change of this step is
        // formed from the two levels and added once
        const int dy_ = layer_depth(y, g.ix0[1], g.ix1[1]);
        const int dz_ = layer_depth(z, g.ix0[2], g.ix1[2]);
        const float ayz = g.dampy * (float)(dy_ * dy_) + g.dampz * (float)(dz_ * dz_);
        const float pin[4] = {S.p.x, S.p.y, S.p.z, S.p.w};
        const float win[4] = {S.w.x, S.w.y, S.w.z, S.w.w};
        const float uin[4] = {S.u.x, S.u.y, S.u.z, S.u.w};
        const float cin[4] = {S.c.x, S.c.y, S.c.z, S.c.w};
        const float c2in[4] = {vu4.x, vu4.y, vu4.z, vu4.w};
        float on[4], wl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float l = fmaf(c1, sy[i], lap[i]);
            if constexpr (MODE == kLapW) {
                on[i] = win[i] * l;
            } else {
                // wl: w B u^n, the whole spatial term of the step
                const float ctr = MODE == kOT4 ? cin[i] : q[i][K];
                wl[i] = MODE == kOT4 ? fmaf(win[i] * (1.0f / 12.0f), l, q[i][K]) : win[i] * l;
                const int dx_ = layer_depth(x0 + i, g.ix0[0], g.ix1[0]);
                const float a = fmaf(g.dampx, (float)(dx_ * dx_), ayz);
                const float r = __builtin_amdgcn_rcpf(1.0f + a);
                on[i] = ctr + ((1.0f - a) * (ctr - pin[i]) + wl[i]) * r;
            }
        }
        if (ptin) {
            const long long p0 = (long long)z * sxy + rowoff + x0;
            const long long p0g = ((long long)z * ny + y) * nx + x0;   // dense gradient
            if constexpr (VEC) {
                ntstore4(fout + p0, on[0], on[1], on[2], on[3]);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (x0 + i < nx) fout[p0 + i] = on[i];
            }
            if constexpr (GM == kGCarryOut) {
                float t[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) t[i] = uin[i] * wl[i];
                if constexpr (VEC) {
                    ntstore4(cr + p0, t[0], t[1], t[2], t[3]);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (x0 + i < nx) cr[p0 + i] = t[i];
                }
            }
            if constexpr (GRW) {
                const float tin[4] = {S.t.x, S.t.y, S.t.z, S.t.w};
                double gn[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if constexpr (MODE == kOT4)   // v vu / 12 rounded once in binary32
                        gn[i] = gold[i] + gscale * ((double)uin[i] * (double)wl[i] +
                                                    (double)(q[i][K] * c2in[i] * (1.0f / 12.0f)));
                    else if constexpr (GM == kGCarryIn)
                        gn[i] = gold[i] + gscale * ((double)uin[i] * (double)wl[i] + (double)tin[i]);
                    else
                        gn[i] = gold[i] + gscale * (double)uin[i] * (double)wl[i];
                }
                if constexpr (VEC) {
                    *reinterpret_cast<double2 *>(&G[p0g]) = make_double2(gn[0], gn[1]);
                    *reinterpret_cast<double2 *>(&G[p0g + 2]) = make_double2(gn[2], gn[3]);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (x0 + i < nx) G[p0g + i] = gn[i];
                }
            }
        }
        // stage plane z+1 (after the last plane this buffer is simply not read)
        *reinterpret_cast<float4 *>(&tile[cur ^ 1][ty + K][HX + 4 * tx4]) =
            make_float4(q[0][K + 1], q[1][K + 1], q[2][K + 1], q[3][K + 1]);
        if (tid < NH) *reinterpret_cast<float4 *>(&tile[cur ^ 1][hrow][hcol]) = S.h;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int j = 0; j < 2 * K; ++j) q[i][j] = q[i][j + 1];
        }
        q[0][2 * K] = S.f.x; q[1][2 * K] = S.f.y; q[2][2 * K] = S.f.z; q[3][2 * K] = S.f.w;
    };
    // AHEAD = 2: three stages in rotation, six planes per trip; otherwise without the
    // binary64 gradient two stages, four planes per trip (the wait pass drains
    // outstanding loads at the back-edge); with it, whose stage also carries u^k and
    // the gradient, one plane per trip and the stage handed over by copy, which keeps
    // it within 256 registers without spilling
    int z = z0;
    if constexpr (AHEAD == 2) {
        for (; z + 5 < z1; z += 6) {
            step(z, A, C);
            step(z + 1, B, A);
            step(z + 2, C, B);
            step(z + 3, A, C);
            step(z + 4, B, A);
            step(z + 5, C, B);
        }
        for (; z + 2 < z1; z += 3) {
            step(z, A, C);
            step(z + 1, B, A);
            step(z + 2, C, B);
        }
        if (z < z1) step(z, A, C);
        if (z + 1 < z1) step(z + 1, B, A);
    } else if constexpr (!GRW) {
        (void)C;
        for (; z + 3 < z1; z += 4) {
            step(z, A, B);
            step(z + 1, B, A);
            step(z + 2, A, B);
            step(z + 3, B, A);
        }
        for (; z + 1 < z1; z += 2) {
            step(z, A, B);
            step(z + 1, B, A);
        }
        if (z < z1) step(z, A, B);
    } else {
        (void)C;
        for (; z < z1; ++z) {
            step(z, A, B);
            A = B;
        }
    }
}

// 2-D: a workgroup owns 256 consecutive x and marches down z (the second axis).
// `prev` and `fout` may be the same array (read, then written, by the same lane).
// MODE as for the 3-D kernel.
// With inj_vals set (an OT2 step), the workgroup then injects the scatter table's points
// inside its strip and rows into the level it has just written, as the separate injection
// kernel would after the step (the same arithmetic in the same order): a 2-D step is
// short, and a launch saved is a good part of it.  With gout set, one workgroup more
// gathers the receivers of gin (the level the previous step wrote) into gout.
template <int K, bool GRAD, int MODE>
__global__ __launch_bounds__(256) void stencil2d(Grid g, const float *__restrict__ fin, const float *prev,
                                                 float *fout, const float *__restrict__ w,
                                                 const float *__restrict__ uk, const float *__restrict__ xtra,
                                                 const float *__restrict__ xtra2, double *__restrict__ G,
                                                 double gscale, int tiles_x, int zchunks, int zlen, Sparse sp,
                                                 const float *__restrict__ inj_vals, Sparse gsp,
                                                 const float *__restrict__ gin, float *__restrict__ gout)
{
    static_assert(!(GRAD && MODE == kLapW), "the w lap pass carries no gradient term");
    __shared__ float row[256 + 2 * K];
    const int nwg = tiles_x * zchunks;
    if (gout && (int)blockIdx.x == nwg) {
        for (int r = threadIdx.x; r < gsp.n; r += 256) gout[r] = gather_point(gsp, r, gin);
        return;
    }
    const int lid = xcd_remap(blockIdx.x, nwg);
    const int tix = lid % tiles_x, zc = lid / tiles_x;
    const int z0 = zc * zlen, z1 = min(z0 + zlen, g.nz);
    march2d<K, GRAD, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, gscale, tix, z0, z1, row);
    if constexpr (MODE == kOT2) {
        if (inj_vals) {
            __syncthreads();
            const int nx = g.nx, x0 = tix * 256, x1 = min(x0 + 256, nx);
            for (int i = threadIdx.x; i < sp.npts; i += 256) {
                const int p = sp.s_pts[i];
                const int z = p / nx, x = p - z * nx;
                if (z < z0 || z >= z1 || x < x0 || x >= x1) continue;
                inject_point<GRAD>(g, sp, i, p, x, 0, z, inj_vals, w, fout, uk, G, p, gscale);
            }
        }
    }
}

// Adds w s / (1+a) at the source (or receiver) points of the level just written.
template <bool GRAD>
__global__ void inject_kernel(Grid g, Sparse sp, const float *__restrict__ vals, const float *__restrict__ w,
                              float *__restrict__ fout, const float *__restrict__ uk, double *__restrict__ G,
                              double gscale)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sp.npts) return;
    const int p = sp.s_pts[i];
    const long long sxy = (long long)g.px * g.ny;   // p indexes the pitched field arrays
    const int z = (int)(p / sxy);
    const int rem = (int)(p - z * sxy);
    const int y = rem / g.px, x = rem - (rem / g.px) * g.px;
    inject_point<GRAD>(g, sp, i, p, x, y, z, vals, w, fout, uk, G, ((long long)z * g.ny + y) * g.nx + x, gscale);
}

__global__ void gather_kernel(Sparse sp, const float *__restrict__ f, float *__restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= sp.n) return;
    out[r] = gather_point(sp, r, f);
}

__global__ void gather_sum_kernel(Sparse sp, const float *__restrict__ f, float *__restrict__ out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    float tot = 0.0f;
    for (int r = 0; r < sp.n; ++r) {
        float s = 0.0f;
        for (int c = 0; c < sp.nc; ++c) s = fmaf(sp.g_wt[r * sp.nc + c], f[sp.g_idx[r * sp.nc + c]], s);
        tot += s;
    }
    out[0] = tot;
}

// w over the pitched field array from the dense velocity; pad columns get 0
__global__ void setup_w_kernel(const float *__restrict__ vel, float *__restrict__ w, long long P, int nx, int px,
                               double dt, double vmax, unsigned *err)
{
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P;
         p += (long long)gridDim.x * blockDim.x) {
        const long long row = p / px;
        const int x = (int)(p - row * px);
        if (x >= nx) {
            w[p] = 0.0f;
            continue;
        }
        const float v = vel[row * nx + x];
        const double vd = (double)v;
        if (!(vd > 0.0) || !(vd <= vmax)) atomicOr(err, 1u);
        w[p] = (float)(dt * dt * vd * vd);
    }
}

template <typename T>
__global__ void fill_kernel(T *p, long long n, T v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void check_finite_kernel(const float *__restrict__ f, long long n, unsigned *err)
{
    bool bad = false;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        bad |= !isfinite(f[i]);
    if (bad) atomicOr(err, 8u);
}

constexpr int kRedThreads = 256;

__global__ __launch_bounds__(kRedThreads) void residual_kernel(const float *__restrict__ dsim,
                                                               const float *__restrict__ dobs,
                                                               float *__restrict__ res, long long n,
                                                               long long nrec, double *partials)
{
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (long long e = blockIdx.x * (long long)kRedThreads + threadIdx.x; e < n;
         e += (long long)gridDim.x * kRedThreads) {
        if (e < nrec) {
            res[e] = 0.0f;
            continue;
        }
        const double r = (double)dsim[e] - (double)dobs[e];
        res[e] = (float)r;
        acc += r * r;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void final_sum_kernel(const double *partials, int n, double *out)
{
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kRedThreads) acc += partials[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 0.5 * sh[0];
}

struct Dims3 { int n[3]; int N[3]; int nbl; int nd; };

__global__ void pad_kernel(Dims3 d, const float *__restrict__ vin, float *__restrict__ vout, long long P)
{
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P;
         p += (long long)gridDim.x * blockDim.x) {
        long long r = p;
        long long src = 0, stride = 1;
        for (int a = 0; a < d.nd; ++a) {
            int i = (int)(r % d.N[a]);
            r /= d.N[a];
            int j = i - d.nbl;
            j = j < 0 ? 0 : (j > d.n[a] - 1 ? d.n[a] - 1 : j);
            src += (long long)j * stride;
            stride *= d.n[a];
        }
        vout[p] = vin[src];
    }
}

__global__ void velgrad_kernel(Dims3 d, const float *__restrict__ vpad, const double *__restrict__ gm,
                               double *__restrict__ gv, long long Pint)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < Pint;
         q += (long long)gridDim.x * blockDim.x) {
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        long long r = q;
        for (int a = 0; a < d.nd; ++a) {
            int j = (int)(r % d.n[a]);
            r /= d.n[a];
            lo[a] = (j == 0) ? 0 : j + d.nbl;
            hi[a] = (j == d.n[a] - 1) ? d.N[a] - 1 : j + d.nbl;
        }
        double s = 0.0;
        const int z1 = d.nd == 3 ? hi[2] : 0, zl = d.nd == 3 ? lo[2] : 0;
        for (int k = zl; k <= z1; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    const long long p = ((long long)k * d.N[1] + j) * d.N[0] + i;
                    const double c = (double)vpad[p];
                    s += gm[p] * (-2.0 / (c * c * c));
                }
        gv[q] = s;
    }
}

int grid_for(long long n, int threads)
{
    long long b = (n + threads - 1) / threads;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

// z chunking: about `target` workgroups, chunks no shorter than min_len planes.
void choose_chunks(long long tiles, int nz, int min_len, int target, int &zchunks, int &zlen)
{
    long long want = target / tiles;
    long long maxc = nz / (min_len > 0 ? min_len : 1);
    if (maxc < 1) maxc = 1;
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    zlen = (int)((nz + want - 1) / want);
    zchunks = (nz + zlen - 1) / zlen;
}

// Workgroups that fit on the device at once for this kernel (occupancy x CUs).
template <typename Kern>
int resident_workgroups(Kern kern)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    return cus * per_cu;
}

// Kernel launch; with events, the dispatch itself records them around the kernel.
template <typename Kern, typename... Args>
void launch_timed(Kern kern, dim3 grid, hipStream_t s, LaunchEvents ev, Args... args)
{
    if (ev.start)
        hipExtLaunchKernelGGL(kern, grid, dim3(256), 0, s, ev.start, ev.stop, 0, args...);
    else
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, args...);
}

template <int K, int GM, bool VEC, int MODE>
hipError_t launch3d(const Grid &g, const float *fin, const float *prev, float *fout, const float *w,
                    const float *uk, const float *xtra, const float *xtra2, double *G, float *cr, double gscale,
                    hipStream_t s, LaunchEvents ev)
{
    auto kern = stencil3d<K, GM, VEC, MODE>;
    const int tiles_x = (g.nx + 31) / 32, tiles_y = (g.ny + 31) / 32;
    // one resident round of workgroups: z chunks as long as possible (the 2K-plane
    // warm-up of each chunk re-reads the field), but enough of them to fill the GPU
    int zchunks, zlen;
    choose_chunks((long long)tiles_x * tiles_y, g.nz, 4 * K, resident_workgroups(kern), zchunks, zlen);
    const int nwg = tiles_x * tiles_y * zchunks;
    launch_timed(kern, dim3(nwg), s, ev, g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, tiles_x, tiles_y,
                 zchunks, zlen);
    return hipGetLastError();
}

template <int K, int GM, int MODE>
hipError_t launch_k(const Grid &g, const float *fin, const float *prev, float *fout, const float *w,
                    const float *uk, const float *xtra, const float *xtra2, double *G, float *cr, double gscale,
                    hipStream_t s, LaunchEvents ev, const Sparse *inj, const float *inj_vals, const Sparse *gsp,
                    const float *gin, float *gout)
{
    if (g.ndim == 3) {
        if (g.nx % 4 == 0)
            return launch3d<K, GM, true, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev);
        return launch3d<K, GM, false, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev);
    }
    if constexpr (GM == kGCarryOut || GM == kGCarryIn) {
        return hipErrorInvalidValue;   // 2-D steps add their gradient term directly
    } else {
    // 2-D grids are small (a few MB): a step is bound by the latency of each workgroup's
    // plane-by-plane march, not by bandwidth, so chunks are short (down to K planes, whose
    // 2K-plane warm-up loads are issued together) and the workgroups many
    const int tiles_x = (g.nx + 255) / 256;
    int zchunks, zlen;
    choose_chunks(tiles_x, g.nz, K, 2048, zchunks, zlen);
    const int nwg = tiles_x * zchunks;
    const Sparse spv = inj ? *inj : Sparse{};
    const Sparse gv = (gsp && gout) ? *gsp : Sparse{};
    float *go = (gsp && gout) ? gout : nullptr;
    launch_timed(stencil2d<K, GM == kGAdd, MODE>, dim3(nwg + (go ? 1 : 0)), s, ev, g, fin, prev, fout, w, uk, xtra,
                 xtra2, G, gscale, tiles_x, zchunks, zlen, spv, inj ? inj_vals : (const float *)nullptr, gv, gin, go);
    return hipGetLastError();
    }
}

template <int GM, int MODE>
hipError_t launch_any(const Grid &g, const float *fin, const float *prev, float *fout, const float *w,
                      const float *uk, const float *xtra, const float *xtra2, double *G, double gscale, hipStream_t s,
                      LaunchEvents ev, float *cr = nullptr, const Sparse *inj = nullptr,
                      const float *inj_vals = nullptr, const Sparse *gsp = nullptr, const float *gin = nullptr,
                      float *gout = nullptr)
{
    if (gout && g.ndim != 2) return hipErrorInvalidValue;
    if (inj && g.ndim != 2) return hipErrorInvalidValue;   // 3-D steps inject in a launch of their own
    switch (g.K) {
    case 1:
        return launch_k<1, GM, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev, inj, inj_vals, gsp,
                                       gin, gout);
    case 2:
        return launch_k<2, GM, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev, inj, inj_vals, gsp,
                                       gin, gout);
    case 3:
        return launch_k<3, GM, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev, inj, inj_vals, gsp,
                                       gin, gout);
    case 4:
        return launch_k<4, GM, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev, inj, inj_vals, gsp,
                                       gin, gout);
    case 5:
        return launch_k<5, GM, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev, inj, inj_vals, gsp,
                                       gin, gout);
    case 6:
        return launch_k<6, GM, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev, inj, inj_vals, gsp,
                                       gin, gout);
    case 7:
        return launch_k<7, GM, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev, inj, inj_vals, gsp,
                                       gin, gout);
    case 8:
        return launch_k<8, GM, MODE>(g, fin, prev, fout, w, uk, xtra, xtra2, G, cr, gscale, s, ev, inj, inj_vals, gsp,
                                       gin, gout);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fwd_step(const Grid &g, const float *u_in, const float *u_prev, float *u_out, const float *w,
                           hipStream_t s, LaunchEvents ev, const Sparse *src, const float *q_n, const Sparse *rec,
                           float *row_prev)
{
    return launch_any<kGNone, kOT2>(g, u_in, u_prev, u_out, w, nullptr, nullptr, nullptr, nullptr, 0.0, s, ev,
                                    nullptr, src, q_n, rec, u_in, row_prev);
}

hipError_t launch_adj_step(const Grid &g, const float *lam_in, const float *lam_next, float *lam_out,
                           const float *w, const float *uk, double *G, double gscale, hipStream_t s,
                           LaunchEvents ev, float *carry, int gmode, const Sparse *rec, const float *r_row)
{
    if (!G) return launch_any<kGNone, kOT2>(g, lam_in, lam_next, lam_out, w, nullptr, nullptr, nullptr, nullptr, 0.0,
                                            s, ev, nullptr, rec, r_row);
    if (gmode != kGAdd && (g.ndim != 3 || !carry)) return hipErrorInvalidValue;
    switch (gmode) {
    case kGAdd:
        return launch_any<kGAdd, kOT2>(g, lam_in, lam_next, lam_out, w, uk, nullptr, nullptr, G, gscale, s, ev,
                                       nullptr, rec, r_row);
    case kGCarryOut:
        return launch_any<kGCarryOut, kOT2>(g, lam_in, lam_next, lam_out, w, uk, nullptr, nullptr, G, gscale, s, ev,
                                            carry);
    case kGCarryIn:
        return launch_any<kGCarryIn, kOT2>(g, lam_in, lam_next, lam_out, w, uk, nullptr, nullptr, G, gscale, s, ev,
                                           carry);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lapw(const Grid &g, const float *f, float *v_out, const float *w, hipStream_t s, LaunchEvents ev)
{
    return launch_any<kGNone, kLapW>(g, f, nullptr, v_out, w, nullptr, nullptr, nullptr, nullptr, 0.0, s, ev);
}

hipError_t launch_ot4_update(const Grid &g, const float *v, const float *u_in, const float *u_prev, float *u_out,
                             const float *w, const float *uk, const float *vu, double *G, double gscale, hipStream_t s,
                             LaunchEvents ev)
{
    if (G) return launch_any<kGAdd, kOT4>(g, v, u_prev, u_out, w, uk, u_in, vu, G, gscale, s, ev);
    return launch_any<kGNone, kOT4>(g, v, u_prev, u_out, w, nullptr, u_in, nullptr, nullptr, 0.0, s, ev);
}

hipError_t launch_inject_src(const Grid &g, const Sparse &sp, const float *q, int n, const float *w,
                             float *u_out, hipStream_t s)
{
    if (sp.npts == 0) return hipSuccess;
    hipLaunchKernelGGL((inject_kernel<false>), dim3((sp.npts + 63) / 64), dim3(64), 0, s, g, sp, q + n, w, u_out,
                       nullptr, nullptr, 0.0);
    return hipGetLastError();
}

hipError_t launch_inject_res(const Grid &g, const Sparse &sp, const float *r_row, const float *w, float *lam_out,
                             const float *uk, double *G, double gscale, hipStream_t s)
{
    if (sp.npts == 0) return hipSuccess;
    if (G)
        hipLaunchKernelGGL((inject_kernel<true>), dim3((sp.npts + 255) / 256), dim3(256), 0, s, g, sp, r_row, w,
                           lam_out, uk, G, gscale);
    else
        hipLaunchKernelGGL((inject_kernel<false>), dim3((sp.npts + 255) / 256), dim3(256), 0, s, g, sp, r_row, w,
                           lam_out, nullptr, nullptr, 0.0);
    return hipGetLastError();
}

hipError_t launch_gather(const Sparse &sp, const float *f, float *out, hipStream_t s)
{
    if (sp.n == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3((sp.n + 255) / 256), dim3(256), 0, s, sp, f, out);
    return hipGetLastError();
}

hipError_t launch_gather_sum(const Sparse &sp, const float *f, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(gather_sum_kernel, dim3(1), dim3(64), 0, s, sp, f, out);
    return hipGetLastError();
}

hipError_t launch_setup_w(const Grid &g, const float *vel, float *w, double dt, double vmax, unsigned *err,
                          hipStream_t s)
{
    hipLaunchKernelGGL(setup_w_kernel, dim3(grid_for(g.P, 256)), dim3(256), 0, s, vel, w, g.P, g.nx, g.px, dt,
                       vmax, err);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, long long n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((fill_kernel<float>), dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, long long n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((fill_kernel<double>), dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, long long n, uint64_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((fill_kernel<uint64_t>), dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float *f, long long n, unsigned *err, hipStream_t s)
{
    hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, f, n, err);
    return hipGetLastError();
}

hipError_t launch_residual_misfit(const float *dsim, const float *dobs, float *res, long long n, long long nrec,
                                  double *partials, int nparts, double *misfit, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3(nparts), dim3(kRedThreads), 0, s, dsim, dobs, res, n, nrec, partials);
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, nparts, misfit);
    return hipGetLastError();
}

hipError_t launch_pad_velocity(int ndim, const int *n, int nbl, const float *vin, float *vout, hipStream_t s)
{
    Dims3 d{};
    d.nd = ndim;
    d.nbl = nbl;
    long long P = 1;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = a < ndim ? n[a] : 1;
        d.N[a] = a < ndim ? n[a] + 2 * nbl : 1;
        P *= d.N[a];
    }
    hipLaunchKernelGGL(pad_kernel, dim3(grid_for(P, 256)), dim3(256), 0, s, d, vin, vout, P);
    return hipGetLastError();
}

hipError_t launch_velocity_gradient(int ndim, const int *n, int nbl, const float *vpad, const double *gm,
                                    double *gv, hipStream_t s)
{
    Dims3 d{};
    d.nd = ndim;
    d.nbl = nbl;
    long long Pint = 1;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = a < ndim ? n[a] : 1;
        d.N[a] = a < ndim ? n[a] + 2 * nbl : 1;
        Pint *= d.n[a];
    }
    hipLaunchKernelGGL(velgrad_kernel, dim3(grid_for(Pint, 256)), dim3(256), 0, s, d, vpad, gm, gv, Pint);
    return hipGetLastError();
}

}  // namespace wv
