/*
 * wv.h -- checkpointed, compressed adjoint acoustic gradients on MI355X (gfx950).
 *
 * C ABI of the library libwv.so.  Plain pointers and sizes only.
 *
 * Method: Kukreja, Hueckelheim, Louboutin, Hovland, Gorman, "Combining
 * checkpointing and data compression to accelerate adjoint-based optimization
 * problems".  The problem solved per shot is the one stated in Sec. "Problem and
 * test case": the acoustic wave equation, eq. (7), m u_tt - lap u = q with
 * m = 1/c^2, the misfit of eq. (8), phi = 1/2 ||d_sim - d_obs||^2, and its
 * adjoint-state gradient.  The reversal is checkpointed with classic Revolve
 * (Sec. "Checkpointing performance model", eqs. (2)-(3)) and, when a tolerance
 * is given, every stored checkpoint passes through a ZFP-kind fixed-accuracy
 * (absolute error) block-transform codec (Sec. "Lossy Compression",
 * Sec. "Performance model including compression", eq. (6)).
 *
 * Discretisation (the paper gives only the continuous problem):
 *   - grid: n[a] interior points per axis plus nbl absorbing cells on each side;
 *     axis 0 (x) is contiguous, the last axis is depth; arrays are C order
 *     [z][y][x] (3-D) or [z][x] (2-D); P = prod(n[a] + 2 nbl); every array the
 *     caller passes is dense (the library pads the rows of its own field arrays,
 *     see wv_field_elements);
 *   - centred space_order-th order second differences (space_order = 2K,
 *     K = 1..8), zero halo outside the padded grid;
 *   - damping a(x) = dt/2 sum_a smax_a (delta_a/nbl)^2,
 *     smax_a = 3 vmax ln(1000) / (2 nbl h[a]), delta_a = cells into the layer;
 *   - OT2 leapfrog: u^{n+1} = [2u^n - (1-a)u^{n-1} + dt^2 c^2 (lap u^n + s^n)]/(1+a),
 *     u^0 = u^{-1} = 0, n = 0..nt-1; data d^n = R u^n, n = 0..nt;
 *     s^n = S^T q^n (multilinear spreading of the wavelet sample q^n);
 *   - gradient with respect to m = 1/c^2 (the paper's model parameter):
 *       g = -(1/dt^2) sum_{k=1..nt} u^k [(1+a)lam^{k-1} - 2lam^k + (1-a)lam^{k+1}]
 *     with the discrete adjoint lam (exact transpose of the recursion above).
 *
 * OT4 (time_order = 4): the paper's fourth-order-in-time kernel (Sec. "Problem and
 * test case" names it without formulas), read as the modified-equation scheme: the
 * spatial term lap u^n of the step becomes
 *   B u^n = lap u^n + (dt^2/12) lap((1/m) lap u^n),
 * i.e. u^{n+1} = [2u^n - (1-a)u^{n-1} + w lap u^n + (w/12) lap(w lap u^n) + w s^n]/(1+a),
 * w = c^2 dt^2; the adjoint is the same recursion (B is symmetric), and the gradient
 * gains the term from the m inside B:
 *   g += -(1/dt^2) sum_k (w^2/12) (lap lam^k)(lap u^k).
 * Stability: sqrt(3) times the OT2 limit (wv_cfl_dt_to).
 *
 * Precision: wavefields are binary32; the gradient accumulates in binary64;
 * misfit and other reductions are binary64.
 *
 * Conventions for every call:
 *   - device pointers are caller-owned; the library never allocates device
 *     memory: every call takes a caller workspace `ws` of at least the size the
 *     matching *_workspace_bytes query returns (256-byte aligned);
 *   - inputs are read-only; outputs are fully overwritten;
 *   - all device work is enqueued on `stream` (a hipStream_t, NULL = default);
 *     calls synchronise the stream only where a status must be read back
 *     (noted per call); one call per stream at a time;
 *   - return value: WV_OK or a negative WV_E* code (wv_strerror).
 */
#ifndef WV_H
#define WV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WV_OK 0
#define WV_EINVAL (-1)     /* bad argument, dims, geometry, non-finite or out-of-range velocity */
#define WV_ECFL (-2)       /* dt above the stability limit wv_cfl_dt */
#define WV_EBUDGET (-3)    /* memory too small: an engine request whose workspace exceeds the whole pool */
#define WV_EARENA (-4)     /* compressed checkpoints overflowed mem_budget even after the retries (the gradient
                              calls re-plan with half the ratio, up to three times, the last time uncompressed-sized) */
#define WV_ENOMEM (-5)     /* workspace too small */
#define WV_EHIP (-6)       /* a HIP runtime call failed */
#define WV_EUNSTABLE (-7)  /* non-finite wavefield detected */
#define WV_ENOTIMPL (-8)
#define WV_ECAP (-9)       /* codec output buffer too small */
#define WV_ETIMEOUT (-10)  /* wv_engine_wait: the request has not finished yet */

typedef struct {
    int ndim;            /* 2 or 3 */
    int n[3];            /* interior points per axis, axis 0 fastest, last = depth */
    double h[3];         /* grid spacing per axis, metres */
    int nbl;             /* absorbing cells on each side (>= 0) */
    int space_order;     /* 2, 4, ..., 16 */
    int nt;              /* number of time steps N (>= 1) */
    double dt;           /* time step, seconds; must satisfy dt <= wv_cfl_dt(...) */
    double vmax;         /* m/s: upper bound of vel; sets the damping strength and CFL check */
    const float *vel;    /* device [P] padded velocity, m/s, 0 < vel <= vmax */
    int time_order;      /* 2 (or 0): the OT2 leapfrog; 4: the OT4 kernel, see below */
} wv_model;

typedef struct {
    int nsrc;                /* >= 1 point sources sharing one wavelet */
    const double *src_xyz;   /* host [nsrc][ndim], metres from the first interior point, (x[,y],z) */
    const float *wavelet;    /* device [nt] wavelet samples q^n */
    int nrec;                /* >= 1 receivers */
    const double *rec_xyz;   /* host [nrec][ndim], same convention */
} wv_geom;

#define WV_PROFILE 17    /* samples of a compressibility profile */

typedef struct {
    int timing;          /* input: bit 0 = time every schedule action with HIP events;
                            bit 1 = also time every stencil launch on its own */
    long advances;       /* forward steps executed (first sweep + recomputation) */
    long stores;         /* checkpoints written (u^{k-1} is written only for checkpoints the schedule
                            later advances from; a reverse step needs only u^k) */
    long restores;       /* restore actions (a restore reads the checkpoint in place: no copy) */
    long fields;         /* binary32 fields written to checkpoint memory (1 or 2 per store) */
    long decodes;        /* fields decoded from compressed checkpoints (u^k at a restore unless it is still
                            decoded; u^{k-1} only when the schedule advances from the restore) */
    long reverses;       /* adjoint steps */
    long slots;          /* M: checkpoint slots of the schedule (x_0 included) */
    double bytes_stored; /* sum of bytes written to checkpoint memory */
    double peak_bytes;   /* peak checkpoint memory in use */
    double ratio;        /* achieved compression ratio (binary32 bytes of the fields written / bytes stored),
                            1 if tol = 0 */
    double ratio_planned;/* ratio the slot count M was planned with */
    double misfit;       /* phi (wv_misfit_gradient only) */
    double ms_total;     /* device time of the call, ms (HIP events) */
    double ms_forward;   /* with timing: device ms in forward steps (stencil + source injection) */
    double ms_adjoint;   /* with timing: device ms in adjoint steps (stencil + gradient + residual injection) */
    double ms_store;     /* with timing: device ms writing checkpoints (copies or encodes) */
    double ms_restore;   /* with timing: device ms restoring checkpoints (decodes; uncompressed restores are free) */
    double ms_fwd_kernel;/* with timing bit 1: device ms inside the forward stencil launches (one per advance) */
    double ms_adj_kernel;/* with timing bit 1: device ms inside the adjoint+gradient stencil launches (one per reverse) */
    long retries;        /* compressed runs repeated because checkpoints outgrew mem_budget (see WV_EARENA) */
    double profile[WV_PROFILE];  /* compressed runs: stream bytes of one field of u^k at k = 0 (the empty
                            field) and k = ceil(j nt / (WV_PROFILE-1)), j = 1..WV_PROFILE-1, taken from
                            the states this call stored (nearest stored k); 0 where unknown.  For wv_plan. */
} wv_stats;

/* ------------------------------------------------------------------ queries */

/* Stability limit of the OT2 scheme with this stencil (von Neumann):
 *   dt_max = 2 / (vmax sqrt(sum_a S / h[a]^2)),  S = |a_0| + 2 sum_k |a_k|.
 * Host only; returns <= 0 on bad arguments. */
double wv_cfl_dt(int ndim, const double *h, int space_order, double vmax);

/* The same limit for a time order: 2 as wv_cfl_dt; 4 (OT4): sqrt(3) times it, since
 * the OT4 step advances each mode with lam - lam^2/12 in place of lam = c^2 dt^2 times
 * its eigenvalue of -lap, which stays in [0, 4] while lam <= 12.  <= 0 on bad arguments. */
double wv_cfl_dt_to(int ndim, const double *h, int space_order, double vmax, int time_order);

/* Operation selectors for wv_workspace_bytes. */
#define WV_OP_FORWARD 0
#define WV_OP_GRADIENT 1
#define WV_OP_COMPRESSIBILITY 2   /* wv_compressibility (mem_budget ignored) */

/* Workspace bytes needed by wv_forward (op = WV_OP_FORWARD, mem_budget ignored)
 * or by wv_gradient / wv_misfit_gradient / wv_adjoint_src (op = WV_OP_GRADIENT;
 * the checkpoint arena of mem_budget bytes is part of the workspace).  Returns 0
 * on invalid arguments.  Host only. */
size_t wv_workspace_bytes(const wv_model *model, const wv_geom *geom, int op, size_t mem_budget);

/* Elements of one solver field array.  The library keeps its own wavefields, w and
 * uncompressed checkpoints with every row of a 3-D grid padded to a multiple of 32
 * elements (128 bytes), so that rows start on cache lines; the caller's arrays stay
 * dense.  An uncompressed checkpoint slot takes 8 times this many bytes; compressed
 * slots and all ratios refer to the dense 4 P bytes of a field.  A field array must
 * stay below 2^31 elements (point indices are 32-bit): every call returns WV_EINVAL for
 * a larger grid.  Returns 0 on an invalid model.  Host only. */
long long wv_field_elements(const wv_model *model);

/* ------------------------------------------------------------------ solver */

/* Forward modelling, eq. (7): data[n][r] = (R u^n)_r for n = 0..nt (row 0 is 0).
 *   data       device [nt+1][nrec] float, overwritten
 *   state_out  device [2][P] float or NULL: receives (u^nt, u^{nt-1})
 * Synchronises the stream once after set-up to validate the velocity. */
int wv_forward(const wv_model *model, const wv_geom *geom, float *data, float *state_out,
               void *ws, size_t ws_bytes, void *stream);

/* Adjoint-state gradient with respect to m for a given data residual r = d_sim - d_obs,
 * reversed with Revolve checkpointing inside mem_budget bytes of checkpoint memory, on
 * the schedule wv_schedule gives (write_min = 1 when tol == 0, 0 when tol > 0).
 *   residual    device [nt+1][nrec] float (row 0 unused)
 *   mem_budget  bytes available for checkpoints (SI bytes); the slot count is
 *               M = min(nt, 1 + floor(mem_budget / slot)), the 1 being x_0 (the zero
 *               state, which takes no memory; a budget below one checkpoint gives M = 1,
 *               recomputation from x_0 alone); slot = S uncompressed, S / F + 512
 *               compressed (two 256-byte aligned streams), S = 8 P bytes per
 *               uncompressed checkpoint (u^k and u^{k-1}; compressed, the pair is
 *               stored as u^k and the increment u^k - u^{k-1}),
 *               F = 1 if tol == 0, else ratio_hint if > 0.  Without a hint the call
 *               first stores every state (M = nt): if they all fit, that attempt is
 *               the run.  Otherwise it stops before the reversal with the stream size
 *               of every state it stored (once the arena is full, only the profile's
 *               16 sample states are still encoded): the compressibility profile
 *               (late states compress worst, as the paper notes), and M is the
 *               largest slot count whose peak arena use, simulated over the exact
 *               schedule with those sizes, fits (as wv_plan).  That first attempt is
 *               not counted in stats->retries;
 *   tol         0: checkpoints are exact copies; > 0: absolute error bound of the codec
 *   grad_m      device [P] double, overwritten (layer cells included); the sum over the
 *               adjoint steps is formed in binary64, in 3-D OT2 runs one update per pair of
 *               steps k = 2j, 2j-1 (the term of step 2j rounded to binary32 first)
 *   stats       host, may be NULL
 * If the compressed checkpoints outgrow mem_budget, the call re-plans with half the
 * ratio and runs again (at most three times; the last plan uses the uncompressed
 * size, which always fits) and reports the repeats in stats->retries.  WV_EARENA is
 * returned only if that still fails.  Synchronises the stream at the end. */
int wv_gradient(const wv_model *model, const wv_geom *geom, const float *residual, size_t mem_budget,
                double tol, double ratio_hint, double *grad_m, wv_stats *stats,
                void *ws, size_t ws_bytes, void *stream);

/* One checkpointed sweep for misfit and gradient: the first forward pass of the
 * schedule produces d_sim, then r = d_sim - d_obs (binary64 difference),
 * phi = 1/2 sum r^2 (eq. (8), binary64), then the reversal as in wv_gradient.
 *   d_obs   device [nt+1][nrec] float
 *   misfit  host double, receives phi
 *   d_sim   device [nt+1][nrec] float or NULL */
int wv_misfit_gradient(const wv_model *model, const wv_geom *geom, const float *d_obs, size_t mem_budget,
                       double tol, double ratio_hint, double *misfit, double *grad_m, float *d_sim,
                       wv_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* Adjoint source (dot-product test hook): src_adj[n] = sum_s (S lam^n)_s for
 * n = 0..nt-1, the derivative of <d, r> with respect to the wavelet sample q^n.
 *   residual device [nt+1][nrec] float; src_adj device [nt] float. */
int wv_adjoint_src(const wv_model *model, const wv_geom *geom, const float *residual, float *src_adj,
                   void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ velocity helpers (autograd) */

/* vel_padded = interior velocity extended into the absorbing layer by the nearest
 * interior value.  vel_interior device [prod n] float, vel_padded device [P] float. */
int wv_pad_velocity(int ndim, const int *n, int nbl, const float *vel_interior, float *vel_padded, void *stream);

/* Gradient with respect to the interior velocity from the gradient with respect to
 * m on the padded grid: chain rule dm/dc = -2/c^3, then the adjoint of the edge
 * padding (layer cells summed into the interior cell they copy).
 *   vel_padded device [P] float, grad_m device [P] double, grad_vel device [prod n] double. */
int wv_velocity_gradient(int ndim, const int *n, int nbl, const float *vel_padded, const double *grad_m,
                         double *grad_vel, void *stream);

/* ------------------------------------------------------------------ codec (test hooks) */

/* Stream format (one stream per binary32 field, little endian):
 *   header 64 B: u32 magic 0x4B50465A, u32 version 1, u32 ndim, u32 dims[3] (axis 0 fastest,
 *     2-D dims[2] = 1), f64 tol, u32 nblocks, u32 nchunks, u32 256, u32 0, u64 data_words,
 *     u64 total_bytes, 8 zero bytes;
 *   u64 chunk_word_offset[nchunks]; u16 block_bits[nblocks] zero-padded to 8 B; u64 data[].
 * Blocks of 4^d values in C order of block coordinates; chunks of 256 blocks start at a
 * word boundary; inside a chunk blocks follow at consecutive bit offsets, LSB first.
 * Per block: emax (max frexp exponent, >= -126), prec = clamp(emax - floor(log2 tol) + 2(d+1),
 * 0, 32); a single 0 bit if the block is zero or prec = 0, else 1, emax+127 in 8 bits,
 * then bit planes 31..32-prec of the negabinary sequency-ordered coefficients of the
 * separable lifting transform of trunc(x 2^(30-emax)), with group tests.
 * Guarantees |x - decode(encode(x))| <= tol where binary32 can resolve tol. */

/* Device scratch bytes wv_zfpk_encode needs (per chunk of 256 blocks: its word count,
 * its offset and a 16 KiB staging slot). */
size_t wv_zfpk_workspace_bytes(int ndim, const int *dims);

/* Upper bound of the stream size for these dims (any tolerance). */
size_t wv_zfpk_max_bytes(int ndim, const int *dims);

/* Encode field (device [dims[2]][dims[1]][dims[0]] or [dims[1]][dims[0]] float) at
 * absolute tolerance tol > 0 into out (device, cap bytes, 8-byte aligned).
 * *nbytes (host) receives the stream size.  Synchronises the stream.
 * WV_ECAP if cap is too small, WV_EINVAL for a non-finite value or bad arguments. */
int wv_zfpk_encode(const float *field, int ndim, const int *dims, double tol, void *out, size_t cap,
                   size_t *nbytes, void *ws, size_t ws_bytes, void *stream);

/* wv_zfpk_encode for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same encoder and
 * the same stream, with no workspace argument.  Its scratch (bookkeeping words, and
 * the word count and offset of each chunk of 256 blocks) is a fixed 192 KiB array in
 * device memory that each GPU the library runs on holds until the process ends; the
 * call allocates and frees nothing and clears the bookkeeping with a fill kernel (no
 * memset).  Without staging slots it encodes every chunk twice (count, then emit at
 * its offset).  Limit: fields of at most 4,172,288 blocks (e.g. 3-D fields up to 640^3
 * values); a larger field returns WV_ENOMEM (wv_last_error says why) and launches
 * nothing.  Every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (concurrent streams or threads) race: run them one at a time.
 * Arguments, output, errors and synchronisation as wv_zfpk_encode. */
int wv_zfpk_encode_noalloc(const float *field, int ndim, const int *dims, double tol, void *out, size_t cap,
                           size_t *nbytes, void *stream);

/* Decode a stream made by wv_zfpk_encode into field (device, same dims).
 *   in      device, nbytes readable bytes holding the stream (8-byte aligned)
 *   nbytes  readable bytes at `in` (at least the stream's total size)
 * Before anything is launched the 64-byte header is copied to the host and checked
 * against the caller's ndim and dims and against nbytes (magic, version, block and
 * chunk counts, chunk size, data words, total size); any mismatch, a truncated
 * stream included, returns WV_EINVAL and launches nothing.  Inside the stream every
 * word the decoder reads is bounds-checked against nbytes, so corrupt chunk offsets
 * or block lengths decode to wrong values but never read outside [in, in + nbytes).
 * Synchronises the stream once (the header copy). */
int wv_zfpk_decode(const void *in, size_t nbytes, int ndim, const int *dims, float *field, void *stream);

/* ------------------------------------------------------------------ batched 2-D shots */

/* Misfit and gradient of nshots 2-D shots at once, advanced by one persistent kernel.
 * Shots are independent (the paper computes one gradient per shot and sums them, Sec.
 * "Example adjoint problem: Seismic inversion"), and a small 2-D shot cannot fill the GPU
 * one step per launch.  The shots of a batch share the grid (n, h, nbl), space order,
 * nt, dt, vmax and receiver count (time_order 2); velocity, wavelet, source and receiver
 * positions and observed data are their own.  They run the checkpoint schedule of
 * wv_misfit_gradient with the same slot count M (each shot has mem_budget bytes of
 * checkpoint memory; compressed, M is the smallest any shot's compressibility probe
 * plans, unless ratio_hint > 0 plans it), and one kernel launch executes the whole
 * reversal: the host turns the schedule into a program of phases (stencil steps, source
 * and residual injections, checkpoint encodes and decodes, the misfit), and every phase
 * runs for all shots, with a device-wide barrier between phases (a plain launch of at
 * most as many workgroups as the device holds at once).  Each shot's arithmetic is the
 * solo call's, in the same order, so its misfit, gradient and d_sim are bit-identical to
 * wv_misfit_gradient's for that shot alone, whatever else is in the batch.  If a barrier
 * cannot complete within a fraction of a second (other streams' kernels keep some of
 * the launch's workgroups off the device), the launch ends early; a wide one is launched
 * again with half the workgroups (twice at most), and then every shot runs alone,
 * through wv_misfit_gradient in its part of ws: the same results, with stats.retries
 * counting the launches that ended early.  (The environment variable WV_BATCH_SPIN_LIMIT, read at each
 * call, sets that bound in polls; 0 makes every launch end at its first barrier, for
 * tests of this path.)
 *   models, geoms       host [nshots]
 *   d_obs               host [nshots] of device [nt+1][nrec] float
 *   misfits             host [nshots], receives phi of each shot
 *   grad_m              host [nshots] of device [P] double, overwritten
 *   d_sim               host [nshots] of device [nt+1][nrec] float, or NULL (entries nullable)
 *   stats               host [nshots] or NULL (retries: repeats of the whole batch, and
 *                       1 for a launch that ended early)
 *   ws                  wv_batch_workspace_bytes(...) bytes, 256-byte aligned
 * Errors as wv_misfit_gradient, plus WV_EINVAL for shots that do not share the above.
 * Synchronises the stream. */
size_t wv_batch_workspace_bytes(int nshots, const wv_model *models, const wv_geom *geoms, size_t mem_budget);
int wv_batch_misfit_gradient(int nshots, const wv_model *models, const wv_geom *geoms, const float *const *d_obs,
                             size_t mem_budget, double tol, double ratio_hint, double *misfits,
                             double *const *grad_m, float *const *d_sim, wv_stats *stats, void *ws, size_t ws_bytes,
                             void *stream);

/* ------------------------------------------------------------------ serving engine */

/* Continuous batching of shot-gradient requests (shots are independent; the paper
 * computes one gradient per shot and sums them, Sec. "Example adjoint problem").
 * The engine owns max_active worker threads, each with its own HIP stream (default
 * priority) on the device current at creation.  Admission is first fit in arrival
 * order: a free worker takes the oldest queued request whose workspace
 * (wv_workspace_bytes with WV_OP_GRADIENT and its mem_budget, i.e. its working fields
 * plus its checkpoint arena) fits a contiguous free slice of the pool; a request passed
 * over 8 times by later ones is not passed again (nothing behind it is admitted until
 * it is).  Its kernels then run beside those of the other admitted requests.  With
 * batching on (wv_engine_set_batching), 2-D requests are served by one more worker
 * that runs the oldest queued 2-D request together with every later one that can share
 * its call (same grid, order, nt, dt, vmax, receiver count, tolerance, budget and ratio
 * hint), up to max_batch of them, as one wv_batch_misfit_gradient (a lone request as one
 * wv_misfit_gradient); requests arriving while a batch runs join the next.  A request's result does not depend on what else is
 * in flight: batched or not, it is bit-identical to wv_misfit_gradient alone. */
typedef struct wv_engine wv_engine;

typedef struct {
    int status;          /* WV_OK or the wv_misfit_gradient error */
    double misfit;
    double t_submit_ms;  /* engine clock (ms since creation) */
    double t_start_ms;   /* admission */
    double t_end_ms;     /* completion */
    wv_stats stats;
} wv_result;

/* pool: device memory, 256-byte aligned, caller-owned, must outlive the engine.
 * max_active: 1..64 requests in flight. */
int wv_engine_create(void *pool, size_t pool_bytes, int max_active, wv_engine **engine);

/* Turn the batch lane on (max_batch 2..256: 2-D requests run in batches of up to that
 * many) or leave it off (0 or 1).  Only before the first request.  WV_EINVAL otherwise. */
int wv_engine_set_batching(wv_engine *engine, int max_batch);

/* Queue a misfit + gradient request (as wv_misfit_gradient).  model->vel, wavelet,
 * d_obs, grad_m and d_sim (nullable) must stay valid until wv_engine_wait returns
 * for it; src/rec host arrays are copied.  Returns the request id (>= 0), WV_EBUDGET
 * if its workspace exceeds the whole pool, or WV_EINVAL. */
int wv_engine_submit(wv_engine *engine, const wv_model *model, const wv_geom *geom, const float *d_obs,
                     size_t mem_budget, double tol, double ratio_hint, double *grad_m, float *d_sim);

/* Wait for request id (timeout_ms < 0: no limit) and release it.  WV_ETIMEOUT if it
 * did not finish in time (it stays queued or running). */
int wv_engine_wait(wv_engine *engine, int id, double timeout_ms, wv_result *result);

/* Requests waiting for admission and requests running. */
int wv_engine_pending(wv_engine *engine, int *queued, int *active);

/* Finish every queued and running request, then release the engine. */
int wv_engine_destroy(wv_engine *engine);

/* ------------------------------------------------------------------ schedule (host) */

/* Action list of the Revolve reversal of nt steps with M slots (x_0 held in slot 0),
 * the same schedule the gradient calls execute.  Actions are int32 triples (op, a, b):
 *   1 ADVANCE x_a -> x_b, 2 STORE x_a in slot b, 3 RESTORE x_a from slot b,
 *   4 FREE slot b (holding x_a), 5 REVERSE step a.
 * Every split takes a first advance from Griewank's binomial interval of optimal ones,
 * so the forward steps are the minimum t(nt+1, M) of recurrence (3) either way:
 *   write_min = 0: the smallest optimal first advance.  Compressed gradient calls run
 *     this one: their checkpoint streams grow over the run, and these splits hold the
 *     earliest states, so more slots fit a budget.
 *   write_min != 0: the first advance that minimises the checkpoint writes of the whole
 *     reversal (W in the storage overhead W S / B; the smallest such advance among
 *     equal counts), and no store of a state that is reversed at once from the working
 *     state.  Uncompressed gradient calls run this one: their slots are of one size.
 *     Its host table takes 8 (C+1)(nt+2) bytes, C = min(M, largest c with
 *     C(c+2, 2) < nt+1), kept per thread for later calls of the same nt; where that
 *     exceeds 2^26 entries (512 MB) the smallest optimal advance is used instead.
 * actions: host [cap][3]; *n_actions receives the count; WV_ECAP if cap is too small
 * (the count is still returned). */
int wv_schedule(int nt, int M, int write_min, int32_t *actions, size_t cap, size_t *n_actions);

/* Forward steps of that schedule: t(nt+1, M) = r (nt+1) - C(M+1+r-1, r-1),
 * r = min{r : C(M+r, r) >= nt+1}. */
long wv_schedule_forward_steps(int nt, int M);

/* Compressibility over time: the paper studies how the compression ratio of the
 * wavefield changes with the time step (Sec. "Results and discussion": early states,
 * with little energy spread, compress far better; the last state is the worst case).
 * Runs the forward problem and, after every `stride` steps, encodes u^n with the
 * codec at tol; bytes[i] receives the stream size of u^{(i+1) stride} (header and
 * block lengths included; the uncompressed field is 4 P bytes).  *count receives
 * nt / stride; WV_ECAP if that exceeds cap.  ws: wv_workspace_bytes(...,
 * WV_OP_COMPRESSIBILITY, 0) bytes.  Synchronises the stream after every sample. */
int wv_compressibility(const wv_model *model, const wv_geom *geom, double tol, int stride, size_t *bytes,
                       int cap, int *count, void *ws, size_t ws_bytes, void *stream);

/* Checkpoint slots for a compressibility profile (WV_PROFILE stream sizes as in
 * wv_stats.profile, e.g. from an earlier call with the same shot and tolerance): the
 * largest M whose peak arena use fits 97 % of mem_budget, simulated over the exact
 * schedule (slots freed last-in first-out, the second level stored where the schedule
 * advances from a checkpoint, each stream rounded up to 256 bytes, sizes interpolated
 * linearly between the samples).  *ratio_hint receives the planning ratio with which a
 * gradient call plans exactly these M slots (0 when M = 1).  Host only. */
int wv_plan(int nt, long long points, size_t mem_budget, const double *profile, int nprofile, int *slots,
            double *ratio_hint);

/* ------------------------------------------------------------ performance model
 * The run-time model of Sec. "Checkpointing performance model" (eqs. (1)-(5)) and
 * Sec. "Performance model including compression" (eq. (6)), for this library's
 * executor.  The executor restores in place (no read copy; a compressed restore
 * decodes), and writes u^{k-1} only for checkpoints the schedule advances from.  Each
 * cost is one unit's device time, e.g. from the stats of an earlier call with timing:
 * c_f = ms_forward / advances, c_r = ms_adjoint / reverses, t_c or t_copy =
 * ms_store / fields, t_d = ms_restore / decodes, ratio = stats ratio.  The counts come
 * from the exact schedule and a host-only pass of the executor's bookkeeping, so they
 * equal what a gradient call with the same slot count does.
 *   T = c_f * advances + c_r * nt + (t_c | t_copy) * fields + t_d * decodes
 * and the full-storage time of eq. (1), (c_f + c_r) * nt. */
typedef struct {
    double c_f;      /* ms per forward step (stencil, source, receivers) */
    double c_r;      /* ms per adjoint step (stencil, gradient, residual) */
    double t_copy;   /* ms to copy one binary32 field into checkpoint memory */
    double t_c;      /* ms to encode one field */
    double t_d;      /* ms to decode one field */
    double ratio;    /* compression ratio of checkpoint streams (required if compressed) */
    double slot_bytes; /* bytes of one uncompressed checkpoint slot (8 wv_field_elements);
                          0 = 8 points */
} wv_costs;

typedef struct {
    int slots;                 /* M as a gradient call plans it for this budget and ratio */
    long advances, stores, fields, decodes;
    double ms_forward, ms_adjoint, ms_store, ms_restore, ms_total;
    double ms_full_storage;    /* eq. (1): no checkpointing at all */
} wv_prediction;

/* Predicted gradient time for nt steps on a grid of `points` padded points with
 * mem_budget bytes of checkpoint memory, uncompressed (compressed = 0) or compressed.
 * Host only.  A budget below one checkpoint gives M = 1 (recomputation from x_0). */
int wv_predict(int nt, long long points, size_t mem_budget, int compressed, const wv_costs *costs,
               wv_prediction *out);

typedef struct {
    int compressed;          /* 1 if compressed checkpoints are predicted faster, else 0 */
    int slots;               /* M of the chosen strategy */
    double ratio_hint;       /* compressed choice: the planning ratio to pass to the gradient call */
    double ms_plain;         /* predicted time of plain Revolve */
    double ms_compressed;    /* predicted time with compressed checkpoints */
} wv_choice;

/* The decision the run-time model exists for (Sec. "Performance model including
 * compression"): whether compressing the checkpoints of this gradient pays at this
 * budget.  Both strategies are priced as wv_predict does, plain with `plain` (its
 * slot_bytes sizes the slots) and compressed with `compressed`.  With a compressibility
 * profile (WV_PROFILE sizes, as wv_plan takes; NULL if none) the compressed slot count
 * is wv_plan's, else the one compressed->ratio gives.  Plain wins ties: it is also
 * exact.  Host only. */
int wv_choose(int nt, long long points, size_t mem_budget, const wv_costs *plain, const wv_costs *compressed,
              const double *profile, int nprofile, wv_choice *out);

/* Measurement hook: the HBM ceiling of this device for a streaming kernel that reads
 * `reads` (1..4) arrays and writes one, each stream_bytes long, four 16-byte loads per
 * lane in flight: the first array is read through the caches and the others and the
 * written one with nontemporal accesses, the stencils' mix (their marched field cached,
 * their pointwise operands and output nontemporal), over ws (at least (reads + 1)
 * stream_bytes, 256-byte aligned; overwritten).  *gbs receives the best of reps timed
 * launches, in GB/s (bytes read plus written).  Synchronises the stream. */
int wv_stream_ceiling(int reads, size_t stream_bytes, void *ws, size_t ws_bytes, int reps, double *gbs, void *stream);

/* wv_misfit_gradient with the choice of wv_choose made per call: the run-time model,
 * fed with the per-unit costs of earlier calls (plain and compressed, as wv_choose takes
 * them) and, when given, the compressibility profile of an earlier compressed call of
 * this shot and tolerance, predicts plain Revolve and compressed checkpoints at this
 * budget; the call then runs the faster, compressed at tol with the planning ratio of
 * the choice (so M is the choice's slot count), or plain (tol ignored).  *choice
 * (nullable) receives the decision and both predictions.  Errors as wv_choose and
 * wv_misfit_gradient; tol must be > 0 (the tolerance stays the caller's: it is an
 * accuracy choice, not a speed one). */
int wv_misfit_gradient_auto(const wv_model *model, const wv_geom *geom, const float *d_obs, size_t mem_budget,
                            double tol, const wv_costs *plain, const wv_costs *compressed, const double *profile,
                            int nprofile, double *misfit, double *grad_m, float *d_sim, wv_stats *stats,
                            wv_choice *choice, void *ws, size_t ws_bytes, void *stream);

const char *wv_strerror(int code);

/* Detail of the last WV_EHIP returned on the calling thread: the failing runtime
 * call, its source line and the HIP error string (empty if none). */
const char *wv_last_error(void);

/* Library version string. */
const char *wv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WV_H */
