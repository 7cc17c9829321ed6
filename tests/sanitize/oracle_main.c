/* Exercises the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer: model
 * set-up, forward and adjoint runs, the full-storage and checkpointed gradients (plain
 * and compressed), OT4, and the codec on ragged 2-D and 3-D fields.  Any sanitizer report
 * aborts with a non-zero status; the run prints OK at the end. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim; int n[3]; double h[3]; int nbl; int order; int nt; double dt; double vmax; int time_order;
} or_model;
typedef struct or_ctx or_ctx;
double or_cfl_dt_to(int ndim, const double *h, int order, double vmax, int time_order);
or_ctx *or_create(const or_model *m, const double *vel, int nsrc, const double *src_xyz, const double *wavelet,
                  int nrec, const double *rec_xyz, int nthreads, int *status);
void or_destroy(or_ctx *c);
long or_npoints(const or_ctx *c);
int or_forward(const or_ctx *c, double *data, double *traj, double *last);
int or_gradient_full(const or_ctx *c, const double *traj, const double *residual, double *grad, double *lam_all);
int or_gradient_actions(const or_ctx *c, const double *residual, const int32_t *act, long nact, int nslots,
                        double tol, int mode, double *grad, long *stats);
int or_adjoint_src(const or_ctx *c, const double *residual, double *src_adj);
long or_zk_prefix_bytes(int ndim, const int *dims);
int or_zk_encode(const float *f, int ndim, const int *dims, double tol, uint8_t *out, long cap, long *nbytes);
int or_zk_decode(const uint8_t *in, long nbytes, float *f);

static void fail(const char *what) { fprintf(stderr, "FAILED: %s\n", what); exit(1); }

/* the recursive Revolve actions with the smallest optimal split, for M slots */
static long binom(int c, int r) { long b = 1; for (int i = 1; i <= r; ++i) b = b * (c + i) / i; return b; }
static long tsteps(long l, int c)
{
    if (l <= 1) return 0;
    if (c == 1) return l * (l - 1) / 2;
    int r = 0;
    while (binom(c, r) < l) ++r;
    return r * l - binom(c + 1, r - 1);
}
static long nact_g;
static int32_t *act_g;
static int depth_g, wm_g;
static void put(int op, int a, int b) { act_g[3 * nact_g] = op; act_g[3 * nact_g + 1] = a; act_g[3 * nact_g + 2] = b; ++nact_g; }
static void need(int s, int slot) { if (wm_g != s) { put(3, s, slot); wm_g = s; } }
static void rev(int s, int l, int c, int slot)
{
    if (l == 1) { if (s > 0) { need(s, slot); put(5, s, 0); } return; }
    if (c == 1) {
        for (int i = l - 1; i >= 0; --i) {
            if (s + i == 0) break;
            need(s, slot);
            if (i > 0) { put(1, s, s + i); wm_g = s + i; }
            put(5, s + i, 0);
        }
        return;
    }
    int k = 1;
    if (c < l - 1) {
        long best = -1;
        for (int kk = 1; kk < l; ++kk) {
            long v = kk + tsteps(kk, c) + tsteps(l - kk, c - 1);
            if (best < 0 || v < best) { best = v; k = kk; }
        }
    }
    need(s, slot);
    put(1, s, s + k); wm_g = s + k;
    int ns = ++depth_g;
    put(2, s + k, ns);
    rev(s + k, l - k, c - 1, ns);
    put(4, s + k, ns);
    --depth_g;
    rev(s, k, c, slot);
}

static void run_case(int ndim, int nx, int nz, int order, int nt, int time_order)
{
    or_model m;
    memset(&m, 0, sizeof(m));
    m.ndim = ndim; m.n[0] = nx; m.n[1] = ndim == 3 ? nx - 3 : nz; m.n[2] = ndim == 3 ? nz : 1;
    m.h[0] = m.h[1] = m.h[2] = 10.0; m.nbl = 5; m.order = order; m.nt = nt; m.vmax = 3000.0;
    m.time_order = time_order;
    m.dt = 0.4 * or_cfl_dt_to(ndim, m.h, order, m.vmax, time_order);
    long P = 1;
    for (int a = 0; a < ndim; ++a) P *= m.n[a] + 2 * m.nbl;
    double *vel = malloc(sizeof(double) * P), *velt = malloc(sizeof(double) * P);
    for (long p = 0; p < P; ++p) { vel[p] = 2000.0 + 500.0 * sin(0.01 * p); velt[p] = vel[p] + (p % 7 == 0 ? 50.0 : 0.0); }
    double src[3] = {0.5 * 10.0 * (nx - 1), ndim == 3 ? 30.0 : 20.0, 20.0};
    const int nrec = nx;
    double *rec = malloc(sizeof(double) * nrec * ndim);
    for (int r = 0; r < nrec; ++r) { rec[r * ndim] = 10.0 * r; rec[r * ndim + 1] = 20.0; if (ndim == 3) rec[r * ndim + 2] = 20.0; }
    double *wav = malloc(sizeof(double) * nt);
    for (int n = 0; n < nt; ++n) { double t = n * m.dt - 0.06, a = 3.14159 * 15 * t; wav[n] = (1 - 2 * a * a) * exp(-a * a); }
    int st;
    or_ctx *c = or_create(&m, vel, 1, src, wav, nrec, rec, 2, &st), *ct = or_create(&m, velt, 1, src, wav, nrec, rec, 2, &st);
    if (!c || !ct) fail("or_create");
    const long nd = (long)(nt + 1) * nrec;
    double *data = calloc(nd, sizeof(double)), *dobs = calloc(nd, sizeof(double));
    double *traj = calloc((size_t)(nt + 1) * P, sizeof(double)), *last = calloc(2 * P, sizeof(double));
    if (or_forward(c, data, traj, last) || or_forward(ct, dobs, NULL, NULL)) fail("or_forward");
    for (long i = 0; i < nd; ++i) data[i] -= dobs[i];
    double *g = calloc(P, sizeof(double)), *g2 = calloc(P, sizeof(double)), *sa = calloc(nt, sizeof(double));
    if (or_gradient_full(c, traj, data, g, NULL)) fail("or_gradient_full");
    if (or_adjoint_src(c, data, sa)) fail("or_adjoint_src");
    for (int M = 1; M <= 5; M += 2) {
        act_g = malloc(sizeof(int32_t) * 3 * 64 * (nt + 2) * 8);
        nact_g = 0; depth_g = 0; wm_g = 0;
        rev(0, nt + 1, M, 0);
        long stats[6];
        for (int comp = 0; comp < 2; ++comp)
            if (or_gradient_actions(c, data, act_g, nact_g, M, comp ? 1e-4 : 0.0, comp, g2, stats)) fail("actions");
        free(act_g);
    }
    or_destroy(c); or_destroy(ct);
    free(vel); free(velt); free(rec); free(wav); free(data); free(dobs); free(traj); free(last); free(g); free(g2); free(sa);
}

static void codec_case(int ndim, int nx, int ny, int nz, double tol)
{
    int dims[3] = {nx, ny, ndim == 3 ? nz : 1};
    long n = (long)nx * ny * dims[2];
    float *f = malloc(sizeof(float) * n), *d = malloc(sizeof(float) * n);
    for (long i = 0; i < n; ++i) f[i] = (float)(sin(0.37 * i) * exp(-1e-4 * i) + (i % 13 == 0 ? 1e-30 : 0.0));
    long cap = or_zk_prefix_bytes(ndim, dims) + 8 * n + 4096, nb = 0;
    uint8_t *s = calloc(cap, 1);
    if (or_zk_encode(f, ndim, dims, tol, s, cap, &nb)) fail("or_zk_encode");
    if (or_zk_decode(s, nb, d)) fail("or_zk_decode");
    for (long i = 0; i < n; ++i)
        if (fabs((double)d[i] - (double)f[i]) > tol && fabs(f[i]) > 1e-7) fail("codec error bound");
    free(f); free(d); free(s);
}

int main(void)
{
    run_case(2, 23, 19, 4, 40, 2);
    run_case(2, 17, 21, 8, 30, 4);
    run_case(3, 11, 9, 4, 16, 2);
    run_case(3, 9, 10, 16, 10, 4);
    codec_case(2, 37, 23, 1, 1e-3);
    codec_case(3, 13, 7, 9, 1e-5);
    codec_case(3, 4, 4, 4, 1e-1);
    printf("OK\n");
    return 0;
}
