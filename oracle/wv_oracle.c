/*
 * Oracle for the checkpointed adjoint acoustic solver and the ZFP-kind codec.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU reference that the GPU library is checked against.  Nothing in the
 * product path may link, load or call it; only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark do.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * Arithmetic is IEEE binary64 throughout, except the codec, which is defined
 * on binary32 fields (the paper's wavefields are single precision: one
 * 287x881x881 field is "just under 900MB", Sec. "Problem and test case") and
 * is integer work after an exact power-of-two scaling.
 *
 * Paper references (Kukreja et al., "Combining checkpointing and data
 * compression to accelerate adjoint-based optimization problems"):
 *   eq. (7)  acoustic wave equation  m u_tt - lap u = q,  m = 1/c^2
 *   eq. (8)  misfit  phi = 1/2 || d_sim - d_obs ||^2
 *   Sec. "Problem and test case": OT2 kernel, absorbing layer, adjoint-state
 *            gradient, Ricker source at the surface
 *   Sec. "Lossy Compression": ZFP in fixed-tolerance (absolute error) mode
 *
 * Discrete readings (the paper gives only the continuous problem):
 *   - centred 2K-th order second differences, closed-form coefficients;
 *   - interior grid n_a plus nbl absorbing cells on every side, zero halo
 *     (homogeneous Dirichlet) outside the padded grid;
 *   - damping eta = m*sigma, sigma = sum_a smax_a (delta_a/nbl)^2,
 *     smax_a = 3 vmax ln(1000) / (2 nbl h_a), a = sigma dt / 2;
 *   - time stepping residual
 *       E_n = m[(1+a)u^{n+1} - 2u^n + (1-a)u^{n-1}]/dt^2 - lap u^n - s^n = 0,
 *     u^0 = u^-1 = 0, data d^n = R u^n for n = 0..N;
 *   - multilinear source/receiver weights, no 1/h^d scaling;
 *   - OT4 (the paper's fourth-order-in-time kernel, Sec. "Problem and test case"):
 *     the modified-equation scheme, which adds the dt^2/12 u_tttt correction of
 *     the leapfrog and takes u_tttt from the PDE itself, so the spatial operator
 *     becomes B(m) u = lap u + (dt^2/12) lap((1/m) lap u) in E_n (source and
 *     damping as in OT2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ECAP (-3)
#define OR_ESTATE (-4)

/* ------------------------------------------------------------------ */
/* Discretisation                                                       */
/* ------------------------------------------------------------------ */

/* Centred 2K-th order coefficients of the second derivative on a unit grid:
 *   a_k = 2(-1)^(k+1) (K!)^2 / (k^2 (K-k)! (K+k)!),  a_0 = -2 sum_k a_k.   */
void or_fd_coeffs(int K, double *a)
{
    double fk = 1.0;
    for (int i = 2; i <= K; i++) fk *= i;
    double s = 0.0;
    for (int k = 1; k <= K; k++) {
        double fkm = 1.0, fkp = 1.0;
        for (int i = 2; i <= K - k; i++) fkm *= i;
        for (int i = 2; i <= K + k; i++) fkp *= i;
        double v = 2.0 * fk * fk / ((double)k * k * fkm * fkp);
        a[k] = (k % 2 == 1) ? v : -v;
        s += a[k];
    }
    a[0] = -2.0 * s;
}

/* von Neumann limit of the leapfrog scheme with this star stencil:
 *   c dt sqrt(sum_a S/h_a^2) <= 2,  S = |a_0| + 2 sum_k |a_k|.
 * With lam = c^2 dt^2 times the largest eigenvalue of -lap, OT2 needs lam <= 4;
 * OT4 advances u^{n+1} = 2u^n - u^{n-1} - (lam - lam^2/12) u^n per mode, which is
 * stable while 0 <= lam - lam^2/12 <= 4, i.e. lam <= 12: a limit sqrt(3) larger.   */
double or_cfl_dt_to(int ndim, const double *h, int order, double vmax, int time_order)
{
    double a[9];
    int K = order / 2;
    or_fd_coeffs(K, a);
    double S = fabs(a[0]);
    for (int k = 1; k <= K; k++) S += 2.0 * fabs(a[k]);
    double q = 0.0;
    for (int d = 0; d < ndim; d++) q += S / (h[d] * h[d]);
    return (time_order == 4 ? sqrt(12.0) : 2.0) / (vmax * sqrt(q));
}

double or_cfl_dt(int ndim, const double *h, int order, double vmax)
{
    double a[9];
    int K = order / 2;
    or_fd_coeffs(K, a);
    double S = fabs(a[0]);
    for (int k = 1; k <= K; k++) S += 2.0 * fabs(a[k]);
    double q = 0.0;
    for (int d = 0; d < ndim; d++) q += S / (h[d] * h[d]);
    return 2.0 / (vmax * sqrt(q));
}

typedef struct {
    int ndim;       /* 2 or 3 */
    int n[3];       /* interior points per axis, axis 0 fastest (x), last is depth */
    double h[3];    /* spacing per axis, metres */
    int nbl;        /* absorbing cells on each side */
    int order;      /* space order 2K */
    int nt;         /* number of time steps N */
    double dt;      /* seconds */
    double vmax;    /* m/s, sets the damping strength */
    int time_order; /* 2 (OT2) or 4 (OT4); 0 means 2 */
} or_model;

typedef struct {
    or_model m;
    int N[3];           /* padded extents, N[2] = 1 in 2-D */
    long P;
    int K;
    double a[9];        /* unit-grid coefficients */
    double *w;          /* dt^2 / m = dt^2 c^2 */
    double *damp;       /* a = sigma dt / 2 */
    int nsrc, nrec;
    long *src_idx;  double *src_wt;   /* [nsrc][8] */
    long *rec_idx;  double *rec_wt;   /* [nrec][8] */
    double *wavelet;    /* [nt] */
    int nthreads;
} or_ctx;

static int corners(int ndim) { return ndim == 3 ? 8 : 4; }

/* Multilinear weights of a point given in metres from the first interior
 * grid point; coordinates are ordered like the axes (x first, depth last). */
static int interp_point(const or_ctx *c, const double *xyz, long *idx, double *wt)
{
    int nd = c->m.ndim;
    int i0[3] = {0, 0, 0};
    double f[3] = {0, 0, 0};
    for (int d = 0; d < nd; d++) {
        double g = xyz[d] / c->m.h[d] + c->m.nbl;
        if (!(g >= 0.0) || g > (double)(c->N[d] - 1)) return OR_EINVAL;
        int i = (int)floor(g);
        if (i > c->N[d] - 2) i = c->N[d] - 2;
        i0[d] = i;
        f[d] = g - i;
    }
    int nc = corners(nd);
    for (int cc = 0; cc < nc; cc++) {
        long p = 0, stride = 1;
        double wv = 1.0;
        for (int d = 0; d < nd; d++) {
            int bit = (cc >> d) & 1;
            p += (long)(i0[d] + bit) * stride;
            stride *= c->N[d];
            wv *= bit ? f[d] : (1.0 - f[d]);
        }
        idx[cc] = p;
        wt[cc] = wv;
    }
    return OR_OK;
}

void or_destroy(or_ctx *c);

or_ctx *or_create(const or_model *m, const double *vel, int nsrc, const double *src_xyz,
                  const double *wavelet, int nrec, const double *rec_xyz, int nthreads, int *status)
{
    *status = OR_EINVAL;
    if (m->ndim != 2 && m->ndim != 3) return NULL;
    if (m->order < 2 || m->order > 16 || (m->order & 1)) return NULL;
    if (m->nbl < 0 || m->nt < 0 || !(m->dt > 0) || !(m->vmax > 0)) return NULL;
    if (m->time_order != 0 && m->time_order != 2 && m->time_order != 4) return NULL;
    or_ctx *c = calloc(1, sizeof(or_ctx));
    if (!c) { *status = OR_ENOMEM; return NULL; }
    c->m = *m;
    c->nthreads = nthreads > 0 ? nthreads : 1;
    c->K = m->order / 2;
    or_fd_coeffs(c->K, c->a);
    c->P = 1;
    for (int d = 0; d < 3; d++) {
        c->N[d] = d < m->ndim ? m->n[d] + 2 * m->nbl : 1;
        if (c->N[d] < 2 && d < m->ndim) { or_destroy(c); return NULL; }
        c->P *= c->N[d];
    }
    c->w = malloc(sizeof(double) * c->P);
    c->damp = malloc(sizeof(double) * c->P);
    c->nsrc = nsrc; c->nrec = nrec;
    int nc = corners(m->ndim);
    c->src_idx = malloc(sizeof(long) * (nsrc * nc + 1));
    c->src_wt = malloc(sizeof(double) * (nsrc * nc + 1));
    c->rec_idx = malloc(sizeof(long) * (nrec * nc + 1));
    c->rec_wt = malloc(sizeof(double) * (nrec * nc + 1));
    c->wavelet = malloc(sizeof(double) * (m->nt + 1));
    if (!c->w || !c->damp || !c->src_idx || !c->src_wt || !c->rec_idx || !c->rec_wt || !c->wavelet) {
        or_destroy(c); *status = OR_ENOMEM; return NULL;
    }
    for (long p = 0; p < c->P; p++) {
        if (!(vel[p] > 0) || !isfinite(vel[p])) { or_destroy(c); return NULL; }
        c->w[p] = m->dt * m->dt * vel[p] * vel[p];
    }
    /* damping profile, computed point by point from its definition */
    for (long p = 0; p < c->P; p++) {
        long r = p;
        double sigma = 0.0;
        for (int d = 0; d < m->ndim; d++) {
            int i = (int)(r % c->N[d]);
            r /= c->N[d];
            int lo = m->nbl - i;
            int hi = i - (m->nbl + m->n[d] - 1);
            int delta = lo > 0 ? lo : (hi > 0 ? hi : 0);
            if (delta > 0) {
                double smax = 3.0 * m->vmax * log(1000.0) / (2.0 * m->nbl * m->h[d]);
                double x = (double)delta / m->nbl;
                sigma += smax * x * x;
            }
        }
        c->damp[p] = 0.5 * sigma * m->dt;
    }
    for (int s = 0; s < nsrc; s++)
        if (interp_point(c, src_xyz + s * m->ndim, c->src_idx + s * nc, c->src_wt + s * nc)) {
            or_destroy(c); return NULL;
        }
    for (int r = 0; r < nrec; r++)
        if (interp_point(c, rec_xyz + r * m->ndim, c->rec_idx + r * nc, c->rec_wt + r * nc)) {
            or_destroy(c); return NULL;
        }
    for (int n = 0; n < m->nt; n++) c->wavelet[n] = wavelet[n];
    *status = OR_OK;
    return c;
}

void or_destroy(or_ctx *c)
{
    if (!c) return;
    free(c->w); free(c->damp); free(c->src_idx); free(c->src_wt);
    free(c->rec_idx); free(c->rec_wt); free(c->wavelet); free(c);
}

long or_npoints(const or_ctx *c) { return c->P; }
void or_get_w(const or_ctx *c, double *out) { memcpy(out, c->w, sizeof(double) * c->P); }
void or_get_damp(const or_ctx *c, double *out) { memcpy(out, c->damp, sizeof(double) * c->P); }
void or_get_interp(const or_ctx *c, int which, long *idx, double *wt)
{
    int nc = corners(c->m.ndim);
    int np = which ? c->nrec : c->nsrc;
    memcpy(idx, which ? c->rec_idx : c->src_idx, sizeof(long) * np * nc);
    memcpy(wt, which ? c->rec_wt : c->src_wt, sizeof(double) * np * nc);
}

/* out = lap_h u with a zero halo: sum over axes of (1/h^2)(a_0 u + sum_k a_k (u_{+k} + u_{-k})). */
void or_laplacian(const or_ctx *c, const double *u, double *out)
{
    const int nx = c->N[0], ny = c->N[1], nz = c->N[2];
    const int nd = c->m.ndim, K = c->K;
    const long sx = 1, sy = nx, sz = (long)nx * ny;
    int nout = nd == 3 ? nz : ny;   /* slowest axis used for threading */
    (void)nout;
#pragma omp parallel for schedule(static) num_threads(c->nthreads)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long p = x + y * sy + z * sz;
                int pos[3] = {x, y, z};
                long str[3] = {sx, sy, sz};
                int ext[3] = {nx, ny, nz};
                double acc = 0.0;
                for (int d = 0; d < nd; d++) {
                    /* in 2-D the axes are (x, depth) = array axes (0, 1) */
                    double s = c->a[0] * u[p];
                    for (int k = 1; k <= K; k++) {
                        double up = (pos[d] + k < ext[d]) ? u[p + k * str[d]] : 0.0;
                        double dn = (pos[d] - k >= 0) ? u[p - k * str[d]] : 0.0;
                        s += c->a[k] * (up + dn);
                    }
                    acc += s / (c->m.h[d] * c->m.h[d]);
                }
                out[p] = acc;
            }
}

static int is_ot4(const or_ctx *c) { return c->m.time_order == 4; }

/* out = B u: lap u for OT2; lap u + (1/12) lap(w lap u) for OT4, where
 * w = dt^2/m, so that (1/12) lap(w lap u) = (dt^2/12) lap((1/m) lap u). */
int or_apply_B(const or_ctx *c, const double *u, double *out)
{
    or_laplacian(c, u, out);
    if (!is_ot4(c)) return OR_OK;
    double *wl = malloc(sizeof(double) * c->P), *l2 = malloc(sizeof(double) * c->P);
    if (!wl || !l2) { free(wl); free(l2); return OR_ENOMEM; }
    for (long p = 0; p < c->P; p++) wl[p] = c->w[p] * out[p];
    or_laplacian(c, wl, l2);
    for (long p = 0; p < c->P; p++) out[p] += l2[p] / 12.0;
    free(wl); free(l2);
    return OR_OK;
}

/* Multilinear gather: val[r] = sum_c wt u[idx] */
static void gather(const or_ctx *c, int which, const double *u, double *val)
{
    int nc = corners(c->m.ndim);
    int np = which ? c->nrec : c->nsrc;
    const long *idx = which ? c->rec_idx : c->src_idx;
    const double *wt = which ? c->rec_wt : c->src_wt;
    for (int r = 0; r < np; r++) {
        double s = 0.0;
        for (int cc = 0; cc < nc; cc++) s += wt[r * nc + cc] * u[idx[r * nc + cc]];
        val[r] = s;
    }
}

/* Transposed gather (scatter-add): f[idx] += wt val[r] */
static void scatter(const or_ctx *c, int which, const double *val, double *f)
{
    int nc = corners(c->m.ndim);
    int np = which ? c->nrec : c->nsrc;
    const long *idx = which ? c->rec_idx : c->src_idx;
    const double *wt = which ? c->rec_wt : c->src_wt;
    for (int r = 0; r < np; r++)
        for (int cc = 0; cc < nc; cc++) f[idx[r * nc + cc]] += wt[r * nc + cc] * val[r];
}

/* One forward step, eq. (7) discretised: given u^n (cur) and u^{n-1} (prev),
 * solve E_n = 0 for u^{n+1} and write it to next. lap is scratch [P].
 *   E_n = m[(1+a)u^{n+1} - 2u^n + (1-a)u^{n-1}]/dt^2 - B u^n - s^n           */
void or_forward_step(const or_ctx *c, int n, const double *cur, const double *prev, double *next, double *lap)
{
    or_apply_B(c, cur, lap);
    double q = c->wavelet[n];
    double qv[64];
    for (int s = 0; s < c->nsrc && s < 64; s++) qv[s] = q;
    if (c->nsrc <= 64) scatter(c, 0, qv, lap);
    else {
        double *tmp = malloc(sizeof(double) * c->nsrc);
        for (int s = 0; s < c->nsrc; s++) tmp[s] = q;
        scatter(c, 0, tmp, lap);
        free(tmp);
    }
#pragma omp parallel for schedule(static) num_threads(c->nthreads)
    for (long p = 0; p < c->P; p++) {
        double a = c->damp[p];
        next[p] = (2.0 * cur[p] - (1.0 - a) * prev[p] + c->w[p] * lap[p]) / (1.0 + a);
    }
}

/* Forward modelling from rest.  data [nt+1][nrec] (row 0 = R u^0 = 0).
 * traj (nullable) receives u^0..u^nt, [(nt+1)][P].  last (nullable)
 * receives (u^nt, u^{nt-1}) as [2][P]. */
int or_forward(const or_ctx *c, double *data, double *traj, double *last)
{
    long P = c->P;
    double *u0 = calloc(P, sizeof(double)), *u1 = calloc(P, sizeof(double));
    double *u2 = calloc(P, sizeof(double)), *lap = malloc(sizeof(double) * P);
    if (!u0 || !u1 || !u2 || !lap) { free(u0); free(u1); free(u2); free(lap); return OR_ENOMEM; }
    double *prev = u0, *cur = u1, *next = u2;
    if (data) gather(c, 1, cur, data);
    if (traj) memcpy(traj, cur, sizeof(double) * P);
    for (int n = 0; n < c->m.nt; n++) {
        or_forward_step(c, n, cur, prev, next, lap);
        double *t = prev; prev = cur; cur = next; next = t;
        if (data) gather(c, 1, cur, data + (long)(n + 1) * c->nrec);
        if (traj) memcpy(traj + (long)(n + 1) * P, cur, sizeof(double) * P);
    }
    if (last) { memcpy(last, cur, sizeof(double) * P); memcpy(last + P, prev, sizeof(double) * P); }
    free(u0); free(u1); free(u2); free(lap);
    return OR_OK;
}

/* phi = 1/2 sum (d_sim - d_obs)^2, eq. (8), in a fixed serial order. */
double or_misfit(long n, const double *dsim, const double *dobs)
{
    double s = 0.0;
    for (long i = 0; i < n; i++) {
        double r = dsim[i] - dobs[i];
        s += r * r;
    }
    return 0.5 * s;
}

/* One adjoint step k (k = N..1): the transpose of the forward recursion,
 *   lam^{k-1} = [2 lam^k - (1-a) lam^{k+1} + w (B lam^k + R^T r^k)] / (1+a)
 * (B is symmetric: lap is, with the zero halo, and w is diagonal).
 * res_k is residual row k.  Writes lam^{k-1} to out.  lap is scratch [P].   */
void or_adjoint_step(const or_ctx *c, const double *res_k, const double *lam_k, const double *lam_kp1,
                     double *out, double *lap)
{
    or_apply_B(c, lam_k, lap);
    scatter(c, 1, res_k, lap);
#pragma omp parallel for schedule(static) num_threads(c->nthreads)
    for (long p = 0; p < c->P; p++) {
        double a = c->damp[p];
        out[p] = (2.0 * lam_k[p] - (1.0 - a) * lam_kp1[p] + c->w[p] * lap[p]) / (1.0 + a);
    }
}

/* OT4 only: the part of the gradient from the m in B(m),
 *   d/dm [lam . (dt^2/12) lap((1/m) lap u)] = -(dt^2/12)(1/m^2) (lap lam)(lap u),
 * which enters E_n with a minus sign; with w = dt^2/m it is (w^2/12)(lap lam)(lap u)
 * (scaled by -1/dt^2 at the end like the rest). */
static int grad_accum_B(const or_ctx *c, const double *u, const double *lam, double *g)
{
    if (!is_ot4(c)) return OR_OK;
    double *lu = malloc(sizeof(double) * c->P), *ll = malloc(sizeof(double) * c->P);
    if (!lu || !ll) { free(lu); free(ll); return OR_ENOMEM; }
    or_laplacian(c, u, lu);
    or_laplacian(c, lam, ll);
    for (long p = 0; p < c->P; p++) g[p] += c->w[p] * c->w[p] / 12.0 * ll[p] * lu[p];
    free(lu); free(ll);
    return OR_OK;
}

/* gradient contribution of reverse step k:
 *   g += u^k * [(1+a) lam^{k-1} - 2 lam^k + (1-a) lam^{k+1}]
 *        (+ (w^2/12)(lap lam^k)(lap u^k) for OT4)   (scaled by -1/dt^2 at the end) */
static void grad_accum(const or_ctx *c, const double *uk, const double *lkm1, const double *lk,
                       const double *lkp1, double *g)
{
#pragma omp parallel for schedule(static) num_threads(c->nthreads)
    for (long p = 0; p < c->P; p++) {
        double a = c->damp[p];
        g[p] += uk[p] * ((1.0 + a) * lkm1[p] - 2.0 * lk[p] + (1.0 - a) * lkp1[p]);
    }
    grad_accum_B(c, uk, lk, g);
}

static void grad_finish(const or_ctx *c, double *g)
{
    double s = -1.0 / (c->m.dt * c->m.dt);
    for (long p = 0; p < c->P; p++) g[p] *= s;
}

/* Adjoint-state gradient with respect to m from a stored trajectory
 * u^0..u^N (traj, [(N+1)][P]); reverse steps in the order k = N..1:
 *   g_m = -(1/dt^2) sum_k u^k [(1+a) lam^{k-1} - 2 lam^k + (1-a) lam^{k+1}].
 * lam_all (nullable) receives lam^0..lam^{N-1}, [N][P].                      */
int or_gradient_full(const or_ctx *c, const double *traj, const double *residual, double *grad, double *lam_all)
{
    long P = c->P;
    int N = c->m.nt;
    double *l0 = calloc(P, sizeof(double)), *l1 = calloc(P, sizeof(double));
    double *l2 = calloc(P, sizeof(double)), *lap = malloc(sizeof(double) * P);
    if (!l0 || !l1 || !l2 || !lap) { free(l0); free(l1); free(l2); free(lap); return OR_ENOMEM; }
    double *kp1 = l0, *k0 = l1, *km1 = l2;   /* lam^{k+1}, lam^k, lam^{k-1} */
    memset(grad, 0, sizeof(double) * P);
    for (int k = N; k >= 1; k--) {
        or_adjoint_step(c, residual + (long)k * c->nrec, k0, kp1, km1, lap);
        grad_accum(c, traj + (long)k * P, km1, k0, kp1, grad);
        if (lam_all) memcpy(lam_all + (long)(k - 1) * P, km1, sizeof(double) * P);
        double *t = kp1; kp1 = k0; k0 = km1; km1 = t;
    }
    grad_finish(c, grad);
    free(l0); free(l1); free(l2); free(lap);
    return OR_OK;
}

/* The same gradient written as the derivative of the discrete Lagrangian
 * with respect to m (sum over the forward residuals E_n, n = 0..N-1):
 *   g_m = -(1/dt^2) sum_n lam^n [(1+a) u^{n+1} - 2 u^n + (1-a) u^{n-1}],
 * u^{-1} = 0 (plus the OT4 term at the same n).  Used to pin the
 * summation-by-parts identity.                                            */
void or_gradient_nform(const or_ctx *c, const double *traj, const double *lam_all, double *grad)
{
    long P = c->P;
    int N = c->m.nt;
    memset(grad, 0, sizeof(double) * P);
    for (int n = 0; n < N; n++) {
        const double *un1 = traj + (long)(n + 1) * P, *un = traj + (long)n * P;
        const double *unm1 = n > 0 ? traj + (long)(n - 1) * P : NULL;
        const double *ln = lam_all + (long)n * P;
        for (long p = 0; p < P; p++) {
            double a = c->damp[p];
            double um = unm1 ? unm1[p] : 0.0;
            grad[p] += ln[p] * ((1.0 + a) * un1[p] - 2.0 * un[p] + (1.0 - a) * um);
        }
        grad_accum_B(c, un, ln, grad);
    }
    grad_finish(c, grad);
}

/* Pointwise sensitivity of the gradient to the forward states it reads.  By the
 * gradient's definition above the adjoint states do not depend on u, so replacing each
 * u^k by a state within e of it at every point changes g by at most
 *   e * (1/dt^2) sum_k |(1+a) lam^{k-1} - 2 lam^k + (1-a) lam^{k+1}|
 * at each point.  Writes that sum, scaled by 1/dt^2 (without e), to bound.  OT2 only
 * (OR_EINVAL for OT4, whose extra term reads the Laplacian of u^k).                   */
int or_gradient_bound(const or_ctx *c, const double *residual, double *bound)
{
    if (is_ot4(c)) return OR_EINVAL;
    long P = c->P;
    int N = c->m.nt;
    double *l0 = calloc(P, sizeof(double)), *l1 = calloc(P, sizeof(double));
    double *l2 = calloc(P, sizeof(double)), *lap = malloc(sizeof(double) * P);
    if (!l0 || !l1 || !l2 || !lap) { free(l0); free(l1); free(l2); free(lap); return OR_ENOMEM; }
    double *kp1 = l0, *k0 = l1, *km1 = l2;   /* lam^{k+1}, lam^k, lam^{k-1} */
    memset(bound, 0, sizeof(double) * P);
    for (int k = N; k >= 1; k--) {
        or_adjoint_step(c, residual + (long)k * c->nrec, k0, kp1, km1, lap);
        for (long p = 0; p < P; p++) {
            double a = c->damp[p];
            bound[p] += fabs((1.0 + a) * km1[p] - 2.0 * k0[p] + (1.0 - a) * kp1[p]);
        }
        double *t = kp1; kp1 = k0; k0 = km1; km1 = t;
    }
    double s = 1.0 / (c->m.dt * c->m.dt);
    for (long p = 0; p < P; p++) bound[p] *= s;
    free(l0); free(l1); free(l2); free(lap);
    return OR_OK;
}

/* Adjoint source: src_adj[n] = S lam^n for n = 0..N-1 (S = source gather),
 * i.e. the derivative of <d, r> with respect to the wavelet sample q^n.    */
int or_adjoint_src(const or_ctx *c, const double *residual, double *src_adj)
{
    long P = c->P;
    int N = c->m.nt;
    double *l0 = calloc(P, sizeof(double)), *l1 = calloc(P, sizeof(double));
    double *l2 = calloc(P, sizeof(double)), *lap = malloc(sizeof(double) * P);
    double *tmp = malloc(sizeof(double) * (c->nsrc + 1));
    if (!l0 || !l1 || !l2 || !lap || !tmp) { free(l0); free(l1); free(l2); free(lap); free(tmp); return OR_ENOMEM; }
    double *kp1 = l0, *k0 = l1, *km1 = l2;
    for (int k = N; k >= 1; k--) {
        or_adjoint_step(c, residual + (long)k * c->nrec, k0, kp1, km1, lap);
        gather(c, 0, km1, tmp);
        double s = 0.0;
        for (int i = 0; i < c->nsrc; i++) s += tmp[i];
        src_adj[k - 1] = s;
        double *t = kp1; kp1 = k0; k0 = km1; km1 = t;
    }
    free(l0); free(l1); free(l2); free(lap); free(tmp);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* ZFP-kind fixed-accuracy codec (binary32 fields)                      */
/* ------------------------------------------------------------------ */
/*
 * Stream format (little endian), one stream per field:
 *   header, 64 bytes:
 *     u32 magic 0x4B50465A, u32 version 1, u32 ndim, u32 dims[3] (axis 0 fastest;
 *     2-D: dims[2] = 1), f64 tol, u32 nblocks, u32 nchunks, u32 blocks_per_chunk (256),
 *     u32 0, u64 data_words, u64 total_bytes, 8 zero bytes
 *   u64 chunk_word_offset[nchunks]        (from the start of the data words)
 *   u16 block_bits[nblocks], zero-padded to a multiple of 8 bytes
 *   u64 data[data_words]
 * Blocks are 4^d in C order of block coordinates (axis 0 fastest); chunk c holds
 * blocks [256c, 256c+256) concatenated at consecutive bit offsets from a word
 * boundary, bit i of a chunk = bit (i % 64) of word (i / 64).
 * Per block (Lindstrom's fixed-accuracy scheme, own container):
 *   emax = max frexp exponent over the block (clamped to >= -126);
 *   minexp = floor(log2 tol); prec = clamp(emax - minexp + 2(d+1), 0, 32);
 *   all-zero or prec == 0 -> a single 0 bit; else 1 bit, 8 bits emax+127,
 *   block-floating-point ints i = trunc(x 2^(30-emax)), separable forward
 *   lifting transform along axis 0, 1 (, 2), sequency reorder, negabinary,
 *   bit planes 31 .. 32-prec with group testing.
 */
#define ZK_MAGIC 0x4B50465Au
#define ZK_VERSION 1u
#define ZK_BPC 256
#define ZK_HDR 64

/* sequency order: ascending by (sum of indices, sum of squares, then the
 * slowest index first); built by a plain selection sort. */
static void zk_perm(int ndim, int *perm)
{
    int S = ndim == 3 ? 64 : 16;
    int key[64][5];
    int used[64] = {0};
    for (int v = 0; v < S; v++) {
        int i = v & 3, j = (v >> 2) & 3, k = (v >> 4) & 3;
        key[v][0] = i + j + k;
        key[v][1] = i * i + j * j + k * k;
        key[v][2] = k; key[v][3] = j; key[v][4] = i;
    }
    for (int s = 0; s < S; s++) {
        int best = -1;
        for (int v = 0; v < S; v++) {
            if (used[v]) continue;
            if (best < 0) { best = v; continue; }
            int less = 0;
            for (int t = 0; t < 5; t++) {
                if (key[v][t] != key[best][t]) { less = key[v][t] < key[best][t]; break; }
            }
            if (less) best = v;
        }
        used[best] = 1;
        perm[s] = best;
    }
}

/* forward lifting on four integers with stride s (exactly the matrix
 * (1/16)[[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],[-2,6,-6,2]] in exact arithmetic) */
static void zk_fwd_lift(int32_t *p, int s)
{
    int32_t x = p[0], y = p[s], z = p[2 * s], w = p[3 * s];
    x += w; x >>= 1; w -= x;
    z += y; z >>= 1; y -= z;
    x += z; x >>= 1; z -= x;
    w += y; w >>= 1; y -= w;
    w += y >> 1; y -= w >> 1;
    p[0] = x; p[s] = y; p[2 * s] = z; p[3 * s] = w;
}

/* inverse lifting: each real-valued forward step undone in reverse order;
 * wrap-around arithmetic so that any stream decodes deterministically */
static void zk_inv_lift(int32_t *p, int s)
{
    uint32_t x = (uint32_t)p[0], y = (uint32_t)p[s], z = (uint32_t)p[2 * s], w = (uint32_t)p[3 * s];
    y += (uint32_t)((int32_t)w >> 1); w -= (uint32_t)((int32_t)y >> 1);
    y += w; w <<= 1; w -= y;
    z += x; x <<= 1; x -= z;
    y += z; z <<= 1; z -= y;
    w += x; x <<= 1; x -= w;
    p[0] = (int32_t)x; p[s] = (int32_t)y; p[2 * s] = (int32_t)z; p[3 * s] = (int32_t)w;
}

typedef struct { uint64_t *w; long cap_words; long pos; int overflow; } zk_writer;

static void zk_put(zk_writer *wr, int bit)
{
    long wi = wr->pos >> 6;
    if (wi >= wr->cap_words) { wr->overflow = 1; wr->pos++; return; }
    if (bit) wr->w[wi] |= (uint64_t)1 << (wr->pos & 63);
    wr->pos++;
}

typedef struct { const uint64_t *w; long nwords; long pos; int overrun; } zk_reader;

static int zk_get(zk_reader *rd)
{
    long wi = rd->pos >> 6;
    if (wi >= rd->nwords) { rd->overrun = 1; rd->pos++; return 0; }
    int b = (int)((rd->w[wi] >> (rd->pos & 63)) & 1);
    rd->pos++;
    return b;
}

static int zk_minexp(double tol)
{
    int e;
    frexp(tol, &e);
    return e - 1;
}

static int zk_block_exponent(const float *v, int S, int *allzero)
{
    int emax = -126;
    *allzero = 1;
    for (int i = 0; i < S; i++) {
        if (v[i] != 0.0f) {
            int e;
            frexp((double)v[i], &e);
            if (e < -126) e = -126;
            if (e > emax) emax = e;
            *allzero = 0;
        }
    }
    return emax;
}

/* Encode one block of 4^d binary32 values (axis 0 fastest) into the writer.
 * Returns the number of bits written.                                       */
long or_zk_encode_block(const float *vals, int ndim, double tol, zk_writer *wr)
{
    int S = ndim == 3 ? 64 : 16;
    long start = wr->pos;
    int allzero;
    int emax = zk_block_exponent(vals, S, &allzero);
    int prec = emax - zk_minexp(tol) + 2 * (ndim + 1);
    if (prec > 32) prec = 32;
    if (allzero || prec <= 0) { zk_put(wr, 0); return wr->pos - start; }
    zk_put(wr, 1);
    for (int b = 0; b < 8; b++) zk_put(wr, ((emax + 127) >> b) & 1);
    int32_t q[64];
    for (int i = 0; i < S; i++) q[i] = (int32_t)trunc(ldexp((double)vals[i], 30 - emax));
    /* separable transform: axis 0, then axis 1, then axis 2 */
    if (ndim == 3) {
        for (int k = 0; k < 4; k++) for (int j = 0; j < 4; j++) zk_fwd_lift(q + 16 * k + 4 * j, 1);
        for (int k = 0; k < 4; k++) for (int i = 0; i < 4; i++) zk_fwd_lift(q + 16 * k + i, 4);
        for (int j = 0; j < 4; j++) for (int i = 0; i < 4; i++) zk_fwd_lift(q + 4 * j + i, 16);
    } else {
        for (int j = 0; j < 4; j++) zk_fwd_lift(q + 4 * j, 1);
        for (int i = 0; i < 4; i++) zk_fwd_lift(q + i, 4);
    }
    int perm[64];
    zk_perm(ndim, perm);
    uint32_t u[64];
    for (int s = 0; s < S; s++) u[s] = ((uint32_t)q[perm[s]] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu;
    int n = 0;
    for (int k = 31; k >= 32 - prec; k--) {
        /* the plane bits of the coefficients already known to be significant */
        for (int s = 0; s < n; s++) zk_put(wr, (u[s] >> k) & 1);
        /* group tests over the rest */
        while (n < S) {
            int any = 0;
            for (int s = n; s < S; s++) any |= (u[s] >> k) & 1;
            zk_put(wr, any);
            if (!any) break;
            int b;
            do { b = (u[n] >> k) & 1; zk_put(wr, b); n++; } while (!b);
        }
    }
    return wr->pos - start;
}

/* Decode one block; returns 0, or -1 if the reader ran past its words. */
int or_zk_decode_block(zk_reader *rd, int ndim, double tol, float *vals)
{
    int S = ndim == 3 ? 64 : 16;
    if (!zk_get(rd)) { for (int i = 0; i < S; i++) vals[i] = 0.0f; return rd->overrun ? -1 : 0; }
    int ebits = 0;
    for (int b = 0; b < 8; b++) ebits |= zk_get(rd) << b;
    int emax = ebits - 127;
    int prec = emax - zk_minexp(tol) + 2 * (ndim + 1);
    if (prec > 32) prec = 32;
    uint32_t u[64] = {0};
    int n = 0;
    for (int k = 31; k >= 32 - prec; k--) {
        for (int s = 0; s < n; s++) u[s] |= (uint32_t)zk_get(rd) << k;
        while (n < S) {
            if (!zk_get(rd)) break;
            int b;
            do { b = zk_get(rd); if (b) u[n] |= (uint32_t)1 << k; n++; } while (!b && n < S);
        }
        if (rd->overrun) break;
    }
    int perm[64];
    zk_perm(ndim, perm);
    int32_t q[64];
    for (int s = 0; s < S; s++) q[perm[s]] = (int32_t)((u[s] ^ 0xAAAAAAAAu) - 0xAAAAAAAAu);
    if (ndim == 3) {
        for (int j = 0; j < 4; j++) for (int i = 0; i < 4; i++) zk_inv_lift(q + 4 * j + i, 16);
        for (int k = 0; k < 4; k++) for (int i = 0; i < 4; i++) zk_inv_lift(q + 16 * k + i, 4);
        for (int k = 0; k < 4; k++) for (int j = 0; j < 4; j++) zk_inv_lift(q + 16 * k + 4 * j, 1);
    } else {
        for (int i = 0; i < 4; i++) zk_inv_lift(q + i, 4);
        for (int j = 0; j < 4; j++) zk_inv_lift(q + 4 * j, 1);
    }
    /* single rounding of the exact value q 2^(emax-30) to binary32 */
    for (int i = 0; i < S; i++) vals[i] = (float)ldexp((double)q[i], emax - 30);
    return rd->overrun ? -1 : 0;
}

/* convenience wrappers over a caller buffer, for block-level tests */
long or_zk_encode_block_buf(const float *vals, int ndim, double tol, uint64_t *words, long cap_words)
{
    memset(words, 0, sizeof(uint64_t) * cap_words);
    zk_writer wr = {words, cap_words, 0, 0};
    long nb = or_zk_encode_block(vals, ndim, tol, &wr);
    return wr.overflow ? -1 : nb;
}

int or_zk_decode_block_buf(const uint64_t *words, long nwords, long bitpos, int ndim, double tol, float *vals)
{
    zk_reader rd = {words, nwords, bitpos, 0};
    return or_zk_decode_block(&rd, ndim, tol, vals);
}

static void zk_geometry(int ndim, const int *dims, int nb[3], long *nblocks)
{
    for (int d = 0; d < 3; d++) nb[d] = (d < ndim) ? (dims[d] + 3) / 4 : 1;
    *nblocks = (long)nb[0] * nb[1] * nb[2];
}

/* bytes before the data words */
long or_zk_prefix_bytes(int ndim, const int *dims)
{
    int nb[3];
    long nblocks;
    zk_geometry(ndim, dims, nb, &nblocks);
    long nchunks = (nblocks + ZK_BPC - 1) / ZK_BPC;
    long lenbytes = ((nblocks * 2 + 7) / 8) * 8;
    return ZK_HDR + 8 * nchunks + lenbytes;
}

static void zk_gather_block(const float *f, int ndim, const int *dims, int bx, int by, int bz, float *v)
{
    int ext[3] = {dims[0], ndim == 3 ? dims[1] : dims[1], ndim == 3 ? dims[2] : 1};
    for (int k = 0; k < (ndim == 3 ? 4 : 1); k++)
        for (int j = 0; j < 4; j++)
            for (int i = 0; i < 4; i++) {
                int x = 4 * bx + i, y = 4 * by + j, z = 4 * bz + k;
                if (x > ext[0] - 1) x = ext[0] - 1;
                if (y > ext[1] - 1) y = ext[1] - 1;
                if (z > ext[2] - 1) z = ext[2] - 1;
                v[16 * k + 4 * j + i] = f[((long)z * ext[1] + y) * ext[0] + x];
            }
}

static void zk_scatter_block(float *f, int ndim, const int *dims, int bx, int by, int bz, const float *v)
{
    int ext[3] = {dims[0], dims[1], ndim == 3 ? dims[2] : 1};
    for (int k = 0; k < (ndim == 3 ? 4 : 1); k++)
        for (int j = 0; j < 4; j++)
            for (int i = 0; i < 4; i++) {
                int x = 4 * bx + i, y = 4 * by + j, z = 4 * bz + k;
                if (x < ext[0] && y < ext[1] && z < ext[2])
                    f[((long)z * ext[1] + y) * ext[0] + x] = v[16 * k + 4 * j + i];
            }
}

/* Encode a whole field.  dims: axis 0 fastest (2-D: dims[0], dims[1]).
 * Returns OR_OK and the stream size in *nbytes, OR_ECAP if cap is too small,
 * OR_EINVAL for bad arguments or a non-finite value.                        */
int or_zk_encode(const float *f, int ndim, const int *dims, double tol, uint8_t *out, long cap, long *nbytes)
{
    if ((ndim != 2 && ndim != 3) || !(tol > 0) || !isfinite(tol)) return OR_EINVAL;
    for (int d = 0; d < ndim; d++) if (dims[d] < 1) return OR_EINVAL;
    int nb[3];
    long nblocks;
    zk_geometry(ndim, dims, nb, &nblocks);
    long P = (long)dims[0] * dims[1] * (ndim == 3 ? dims[2] : 1);
    for (long p = 0; p < P; p++) if (!isfinite(f[p])) return OR_EINVAL;
    long nchunks = (nblocks + ZK_BPC - 1) / ZK_BPC;
    long prefix = or_zk_prefix_bytes(ndim, dims);
    if (cap < prefix) return OR_ECAP;
    memset(out, 0, prefix);
    uint64_t *chunk_off = (uint64_t *)(out + ZK_HDR);
    uint16_t *lens = (uint16_t *)(out + ZK_HDR + 8 * nchunks);
    long cap_words = (cap - prefix) / 8;
    uint64_t *data = (uint64_t *)(out + prefix);
    memset(data, 0, sizeof(uint64_t) * cap_words);
    int S = ndim == 3 ? 64 : 16;
    float v[64];
    long word = 0;
    int overflow = 0;
    for (long c = 0; c < nchunks; c++) {
        chunk_off[c] = (uint64_t)word;
        zk_writer wr = {data + word, cap_words - word, 0, 0};
        for (long b = c * ZK_BPC; b < nblocks && b < (c + 1) * ZK_BPC; b++) {
            int bx = (int)(b % nb[0]), by = (int)((b / nb[0]) % nb[1]), bz = (int)(b / ((long)nb[0] * nb[1]));
            zk_gather_block(f, ndim, dims, bx, by, bz, v);
            (void)S;
            long nbits = or_zk_encode_block(v, ndim, tol, &wr);
            lens[b] = (uint16_t)nbits;
        }
        if (wr.overflow) overflow = 1;
        word += (wr.pos + 63) / 64;
    }
    if (overflow) return OR_ECAP;
    uint32_t *h32 = (uint32_t *)out;
    h32[0] = ZK_MAGIC; h32[1] = ZK_VERSION; h32[2] = (uint32_t)ndim;
    h32[3] = (uint32_t)dims[0]; h32[4] = (uint32_t)dims[1]; h32[5] = ndim == 3 ? (uint32_t)dims[2] : 1u;
    memcpy(out + 24, &tol, 8);
    h32[8] = (uint32_t)nblocks; h32[9] = (uint32_t)nchunks; h32[10] = ZK_BPC; h32[11] = 0;
    uint64_t dw = (uint64_t)word, tb = (uint64_t)(prefix + 8 * word);
    memcpy(out + 48, &dw, 8);
    memcpy(out + 56, &tb, 8);
    *nbytes = (long)tb;
    return OR_OK;
}

/* Decode a stream produced by or_zk_encode (or the GPU encoder). */
int or_zk_decode(const uint8_t *in, long nbytes, float *f)
{
    if (nbytes < ZK_HDR) return OR_EINVAL;
    const uint32_t *h32 = (const uint32_t *)in;
    if (h32[0] != ZK_MAGIC || h32[1] != ZK_VERSION) return OR_EINVAL;
    int ndim = (int)h32[2];
    int dims[3] = {(int)h32[3], (int)h32[4], (int)h32[5]};
    double tol;
    memcpy(&tol, in + 24, 8);
    int nb[3];
    long nblocks;
    zk_geometry(ndim, dims, nb, &nblocks);
    long nchunks = (nblocks + ZK_BPC - 1) / ZK_BPC;
    if ((long)h32[8] != nblocks || (long)h32[9] != nchunks) return OR_EINVAL;
    long prefix = or_zk_prefix_bytes(ndim, dims);
    uint64_t dw;
    memcpy(&dw, in + 48, 8);
    if (prefix + 8 * (long)dw > nbytes) return OR_EINVAL;
    const uint64_t *chunk_off = (const uint64_t *)(in + ZK_HDR);
    const uint16_t *lens = (const uint16_t *)(in + ZK_HDR + 8 * nchunks);
    const uint64_t *data = (const uint64_t *)(in + prefix);
    float v[64];
    for (long c = 0; c < nchunks; c++) {
        long bit = (long)chunk_off[c] * 64;
        for (long b = c * ZK_BPC; b < nblocks && b < (c + 1) * ZK_BPC; b++) {
            int bx = (int)(b % nb[0]), by = (int)((b / nb[0]) % nb[1]), bz = (int)(b / ((long)nb[0] * nb[1]));
            zk_reader rd = {data, (long)dw, bit, 0};
            if (or_zk_decode_block(&rd, ndim, tol, v)) return OR_EINVAL;
            if (rd.pos - bit != lens[b]) return OR_EINVAL;
            zk_scatter_block(f, ndim, dims, bx, by, bz, v);
            bit += lens[b];
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Checkpointed reversal driven by an explicit action list              */
/* ------------------------------------------------------------------ */
/* Actions are int triples (op, a, b):
 *   1 ADVANCE from x_a to x_b;  2 STORE x_a into slot b;  3 RESTORE x_a from slot b;
 *   4 FREE slot b (holding x_a);  5 REVERSE step a (needs x_a = (u^a, u^{a-1})).
 * Slot 0 holds x_0, the state at rest.  Checkpoints either hold both time
 * levels, (u^k, u^{k-1}), or the level and its increment, (u^k, u^k - u^{k-1})
 * (mode 1).  With tol > 0 each field of a checkpoint is rounded to binary32
 * and passed through the codec; tol = 0 keeps exact binary64 copies.
 * stats (nullable, 6 longs): advances, stores, restores, reverses, bytes stored
 * (sum), peak bytes held.                                                    */
int or_gradient_actions(const or_ctx *c, const double *residual, const int32_t *act, long nact, int nslots,
                        double tol, int mode, double *grad, long *stats)
{
    long P = c->P;
    int N = c->m.nt;
    int nd = c->m.ndim;
    int dims[3] = {c->N[0], c->N[1], c->N[2]};
    if (nd == 2) { dims[2] = 1; }
    double *cur = calloc(P, sizeof(double)), *prev = calloc(P, sizeof(double));
    double *next = calloc(P, sizeof(double)), *lap = malloc(sizeof(double) * P);
    double *l0 = calloc(P, sizeof(double)), *l1 = calloc(P, sizeof(double)), *l2 = calloc(P, sizeof(double));
    double **slot_d = calloc(nslots, sizeof(double *));
    uint8_t **slot_z = calloc(nslots, sizeof(uint8_t *));
    long *slot_n = calloc(nslots, sizeof(long));
    int *slot_k = calloc(nslots, sizeof(int));
    float *tmpf = malloc(sizeof(float) * P);
    int rc = OR_OK;
    long st[6] = {0, 0, 0, 0, 0, 0};
    long held = 0;
    if (!cur || !prev || !next || !lap || !l0 || !l1 || !l2 || !slot_d || !slot_z || !slot_n || !slot_k || !tmpf) {
        rc = OR_ENOMEM; goto done;
    }
    for (int s = 0; s < nslots; s++) slot_k[s] = -1;
    memset(grad, 0, sizeof(double) * P);
    int wm = 0;                 /* index k of the state in working memory */
    int next_rev = N;           /* reverse steps run N, N-1, ..., 1 */
    double *kp1 = l0, *k0 = l1, *km1 = l2;
    long zcap = or_zk_prefix_bytes(nd, dims) + 8 * (P * 5 + 64);
    for (long i = 0; i < nact && rc == OR_OK; i++) {
        int op = act[3 * i], a = act[3 * i + 1], b = act[3 * i + 2];
        switch (op) {
        case 1:
            if (wm != a || b < a || b > N) { rc = OR_ESTATE; break; }
            for (int n = a; n < b; n++) {
                or_forward_step(c, n, cur, prev, next, lap);
                double *t = prev; prev = cur; cur = next; next = t;
            }
            st[0] += b - a;
            wm = b;
            break;
        case 2: {
            if (wm != a || b <= 0 || b >= nslots || slot_k[b] >= 0) { rc = OR_ESTATE; break; }
            if (tol > 0) {
                long tot = 0;
                uint8_t *buf = malloc(2 * zcap);
                if (!buf) { rc = OR_ENOMEM; break; }
                for (int fi = 0; fi < 2; fi++) {
                    for (long p = 0; p < P; p++)
                        tmpf[p] = (float)(fi == 0 ? cur[p] : (mode == 1 ? cur[p] - prev[p] : prev[p]));
                    long nb = 0;
                    int e = or_zk_encode(tmpf, nd, dims, tol, buf + tot, zcap, &nb);
                    if (e) { rc = e; break; }
                    tot += nb;
                }
                slot_z[b] = buf; slot_n[b] = tot;
            } else {
                double *buf = malloc(sizeof(double) * 2 * P);
                if (!buf) { rc = OR_ENOMEM; break; }
                memcpy(buf, cur, sizeof(double) * P);
                for (long p = 0; p < P; p++) buf[P + p] = mode == 1 ? cur[p] - prev[p] : prev[p];
                slot_d[b] = buf; slot_n[b] = 16 * P;
            }
            slot_k[b] = a;
            st[1]++;
            st[4] += slot_n[b];
            held += slot_n[b];
            if (held > st[5]) st[5] = held;
            break;
        }
        case 3:
            if (b < 0 || b >= nslots) { rc = OR_ESTATE; break; }
            if (b == 0) {
                if (a != 0) { rc = OR_ESTATE; break; }
                memset(cur, 0, sizeof(double) * P);
                memset(prev, 0, sizeof(double) * P);
            } else {
                if (slot_k[b] != a) { rc = OR_ESTATE; break; }
                if (tol > 0) {
                    long off = 0;
                    for (int fi = 0; fi < 2; fi++) {
                        long tb;
                        memcpy(&tb, slot_z[b] + off + 56, 8);
                        int e = or_zk_decode(slot_z[b] + off, tb, tmpf);
                        if (e) { rc = e; break; }
                        for (long p = 0; p < P; p++) (fi == 0 ? cur : prev)[p] = (double)tmpf[p];
                        off += tb;
                    }
                } else {
                    memcpy(cur, slot_d[b], sizeof(double) * P);
                    memcpy(prev, slot_d[b] + P, sizeof(double) * P);
                }
                if (mode == 1)
                    for (long p = 0; p < P; p++) prev[p] = cur[p] - prev[p];
            }
            wm = a;
            st[2]++;
            break;
        case 4:
            if (b <= 0 || b >= nslots || slot_k[b] != a) { rc = OR_ESTATE; break; }
            held -= slot_n[b];
            free(slot_d[b]); free(slot_z[b]);
            slot_d[b] = NULL; slot_z[b] = NULL; slot_k[b] = -1; slot_n[b] = 0;
            break;
        case 5:
            if (wm != a || a != next_rev || a < 1) { rc = OR_ESTATE; break; }
            or_adjoint_step(c, residual + (long)a * c->nrec, k0, kp1, km1, lap);
            grad_accum(c, cur, km1, k0, kp1, grad);
            { double *t = kp1; kp1 = k0; k0 = km1; km1 = t; }
            next_rev--;
            st[3]++;
            break;
        default:
            rc = OR_EINVAL;
        }
    }
    if (rc == OR_OK && next_rev != 0) rc = OR_ESTATE;
    if (rc == OR_OK) grad_finish(c, grad);
    if (stats) memcpy(stats, st, sizeof(st));
done:
    if (slot_d) for (int s = 0; s < nslots; s++) free(slot_d[s]);
    if (slot_z) for (int s = 0; s < nslots; s++) free(slot_z[s]);
    free(cur); free(prev); free(next); free(lap); free(l0); free(l1); free(l2);
    free(slot_d); free(slot_z); free(slot_n); free(slot_k); free(tmpf);
    return rc;
}

/* Exposed pieces of the codec for pin tests. */
void or_zk_fwd_lift4(int32_t *p) { zk_fwd_lift(p, 1); }
void or_zk_inv_lift4(int32_t *p) { zk_inv_lift(p, 1); }
void or_zk_perm(int ndim, int *perm) { zk_perm(ndim, perm); }
uint32_t or_zk_negabinary(int32_t x) { return ((uint32_t)x + 0xAAAAAAAAu) ^ 0xAAAAAAAAu; }
