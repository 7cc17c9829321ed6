// Internal declarations of libwv (GPU path).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/wv.h"

namespace wv {

constexpr int kMaxK = 8;            // space order up to 16
constexpr int kBlocksPerChunk = 256; // codec: blocks per chunk (one workgroup)

// Geometry and coefficients of one padded grid, as the stencil kernels see it.
// Axes are named for the array layout: x contiguous, z slowest.  In 2-D, y is
// absent (ny = 1) and the model's second axis is z.
// The solver's field arrays (wavefields, w, checkpoint slots) are pitched: point
// (x, y, z) sits at x + px (y + ny z), with px = nx rounded up to 32 in 3-D, so that
// every row starts on a 128-byte line (columns nx..px-1 hold zeros and are never
// read as grid points).  In 2-D px = nx.  Arrays the caller owns (velocity,
// gradient, final state) are dense: x + nx (y + ny z).
struct Grid {
    int nx, ny, nz;          // padded extents
    int px;                  // row pitch of the solver's field arrays (elements)
    int ix0[3], ix1[3];      // interior index range [ix0, ix1] per array axis (x, y, z)
    float cx[kMaxK + 1];     // a_k / h^2 per axis, k = 1..K;
    float cy[kMaxK + 1];     // cy[0] = h_x^2/h_y^2 and cz[0] = h_x^2/h_z^2 (the 3-D kernel
    float cz[kMaxK + 1];     // applies cx[k] on every axis and scales y, z by these)
    float cf2[3];            // 2 sum_{k>=2} of the axis's weights (x from cx, y from cy, z from cz)
    float dampx, dampy, dampz; // 0.5 dt smax_axis / nbl^2; a = sum damp_axis * delta_axis^2
    int K;
    int ndim;
    int time_order;          // 2 (OT2) or 4 (OT4)
    long long P;             // elements of one field array: px * ny * nz
};

// Sparse point operators (sources / receivers), built on the host.
//   gather:  out[r] = sum_c wt[r*nc + c] * f[idx[r*nc + c]]
//   scatter: unique points pts[i], entries [start[i], start[i+1]) of (col, wt)
struct Sparse {
    int n;            // number of sources or receivers
    int nc;           // corners per point (4 or 8)
    const int *g_idx; const float *g_wt;          // gather tables [n*nc]
    int npts;         // unique grid points touched
    const int *s_pts; const int *s_start;        // [npts], [npts+1]
    const int *s_col; const float *s_wt;         // [nnz]
};

// ---------------------------------------------------------------- stencil launches (wv_stencil.hip)
// Optional pair of events recorded by the kernel dispatch itself (start and end of the
// stencil kernel, nothing else), for per-launch timing.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
// Forward step: u_out = u_in + ((1-a)(u_in - u_prev) + w lap u_in)/(1+a).
// u_out may equal u_prev (in place); it must differ from u_in.  2-D only: with src, the
// same launch then injects sample q_n (a device pointer) at the table's points, as
// launch_inject_src would; with rec and row_prev, it also gathers the receivers of u_in
// (the previous step's level) into row_prev, as launch_gather would.
hipError_t launch_fwd_step(const Grid &g, const float *u_in, const float *u_prev, float *u_out, const float *w,
                           hipStream_t s, LaunchEvents ev = {}, const Sparse *src = nullptr,
                           const float *q_n = nullptr, const Sparse *rec = nullptr, float *row_prev = nullptr);
// How an adjoint step's gradient term t = uk * (w lap lam_in) reaches G.  The carried
// forms are for 3-D grids: a step with kGCarryOut leaves t, rounded to binary32, in a
// field-sized array, and the next adjoint step (kGCarryIn) adds it with its own term,
// so that a pair of steps reads and writes G once.
constexpr int kGNone = 0, kGAdd = 1, kGCarryOut = 2, kGCarryIn = 3;
// Adjoint step (lam_in = lam^k, lam_next = lam^{k+1}, lam_out = lam^{k-1}, may equal
// lam_next): the same update, and (if G) G += gscale * uk * (w lap lam_in), or the
// carried form gmode selects with the array carry (pitched like a field).
// 2-D only: with rec, the same launch then injects the residual row r_row at the
// receivers (and their gradient term), as launch_inject_res would.
hipError_t launch_adj_step(const Grid &g, const float *lam_in, const float *lam_next, float *lam_out,
                           const float *w, const float *uk, double *G, double gscale, hipStream_t s,
                           LaunchEvents ev = {}, float *carry = nullptr, int gmode = kGAdd,
                           const Sparse *rec = nullptr, const float *r_row = nullptr);
// OT4, first pass: v_out = w lap f.
hipError_t launch_lapw(const Grid &g, const float *f, float *v_out, const float *w, hipStream_t s,
                       LaunchEvents ev = {});
// OT4, second pass: u_out = u_in + ((1-a)(u_in - u_prev) + v + (w/12) lap v)/(1+a), v = w lap u_in
// from the first pass; with G, G += gscale * (uk * (v + (w/12) lap v) + v * vu / 12), vu = w lap uk.
// u_out may equal u_prev.
hipError_t launch_ot4_update(const Grid &g, const float *v, const float *u_in, const float *u_prev, float *u_out,
                             const float *w, const float *uk, const float *vu, double *G, double gscale,
                             hipStream_t s, LaunchEvents ev = {});
// Source injection of sample q[n] (forward) at the unique source points of u_out.
hipError_t launch_inject_src(const Grid &g, const Sparse &sp, const float *q, int n, const float *w,
                             float *u_out, hipStream_t s);
// Residual injection of row r_row (adjoint) at the unique receiver points; gradient term.
hipError_t launch_inject_res(const Grid &g, const Sparse &sp, const float *r_row, const float *w, float *lam_out,
                             const float *uk, double *G, double gscale, hipStream_t s);
// Receiver gather out[r] = (R f)_r.
hipError_t launch_gather(const Sparse &sp, const float *f, float *out, hipStream_t s);
// Sum over sources of the gathered field: out[0] = sum_s (S f)_s.
hipError_t launch_gather_sum(const Sparse &sp, const float *f, float *out, hipStream_t s);
// w = dt^2 vel^2 (vel dense, w pitched, pad columns 0) and validation; err bit 1:
// non-finite or out of (0, vmax].
hipError_t launch_setup_w(const Grid &g, const float *vel, float *w, double dt, double vmax, unsigned *err,
                          hipStream_t s);
hipError_t launch_fill_f32(float *p, long long n, float v, hipStream_t s);
hipError_t launch_fill_f64(double *p, long long n, double v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, long long n, uint64_t v, hipStream_t s);
// r = (float)((double)dsim - (double)dobs) for rows 1..nt (row 0 = 0); partial sums of r^2 (binary64).
hipError_t launch_residual_misfit(const float *dsim, const float *dobs, float *res, long long nrow_elems,
                                  long long nrec, double *partials, int nparts, double *misfit, hipStream_t s);
hipError_t launch_pad_velocity(int ndim, const int *n, int nbl, const float *vin, float *vout, hipStream_t s);
hipError_t launch_velocity_gradient(int ndim, const int *n, int nbl, const float *vpad, const double *gm,
                                    double *gv, hipStream_t s);
hipError_t launch_check_finite(const float *f, long long n, unsigned *err, hipStream_t s);

// ---------------------------------------------------------------- codec (wv_codec.hip)
struct CodecDims {
    int ndim;
    int dims[3];       // axis 0 fastest; 2-D: dims[2] = 1
    int pitch;         // elements from one row (axis 0) of the field array to the next (>= dims[0])
    int nb[3];         // blocks per axis
    long long nblocks;
    long long nchunks;
    long long prefix_bytes;  // header + chunk table + block lengths
};
// pitch 0: dense rows (pitch = dims[0])
CodecDims codec_dims(int ndim, const int *dims, int pitch = 0);
size_t codec_max_bytes(const CodecDims &cd);
// Encode field (or field - sub, in binary32, when sub is not null) into out + *base
// (device offset), capacity cap bytes from `out`.
// Writes *next = *base + stream bytes rounded up to 256.  work: encode_work_bytes(cd,
// staged) bytes, 256-byte aligned, any contents (chunk word counts, offsets and, when
// staged, a kLdsWords-word slot per chunk; without staging every chunk is encoded twice).
// size_out (nullable) receives the stream's size in bytes.
// err: bit 2 = capacity overflow, bit 1 = non-finite input.
// stats[0] += stream bytes, stats[1] = max(stats[1], *next).
size_t encode_work_bytes(const CodecDims &cd, bool staged);
hipError_t launch_encode(const CodecDims &cd, const float *field, const float *sub, double tol, uint8_t *out,
                         uint64_t cap, const uint64_t *base, uint64_t *next, uint8_t *work, bool staged,
                         unsigned *err, unsigned long long *stats, hipStream_t s, uint64_t *size_out = nullptr);
// Decode the stream at in + *base (base == nullptr: offset 0) into field, or, when sub
// is not null, store sub - decoded; cap bytes are readable from `in` (a stream that
// does not fit decodes to zeros).
hipError_t launch_decode(const CodecDims &cd, const uint8_t *in, const uint64_t *base, uint64_t cap, float *field,
                         const float *sub, hipStream_t s);

// ---------------------------------------------------------------- batched 2-D solver (wv_batch.hip)
// Several 2-D shots of one grid, order, step count and schedule advanced together by
// one persistent kernel that runs a program of phases, all shots per phase, with a
// device-wide barrier between phases.  Each shot keeps the buffers of a solo call
// (field arrays dense in 2-D).
struct BatchShot {
    float *U[2], *UB, *DB, *Lm[2], *Z, *W;
    const float *wavelet;     // [nt]
    const float *dobs;        // [nt+1][nrec]
    float *dsim, *res;        // [nt+1][nrec]
    double *G;                // gradient (caller's, dense [P])
    double *partials;         // residual partial sums [kParts]
    double *misfit;           // phi (device)
    uint8_t *arena;           // checkpoint memory of this shot
    uint64_t arena_bytes;
    uint64_t *offs;           // stream offsets (as the solo executor's)
    uint64_t *sizes;          // stream bytes of u^k per stored k
    uint32_t *chunk_words;    // [2][nchunks]: words per chunk of the two fields of a store
    unsigned *err;            // bit 1: velocity, 2: non-finite input to the codec, 4: arena overflow,
                              // 8: non-finite wavefield, 16: barrier timeout
    unsigned long long *stats;  // [0] stream bytes stored, [1] peak arena offset
    Sparse src, rec;
};

// Buffers of a program step, by id: the shot's own arrays, or level l of checkpoint
// slot b (uncompressed) as kBufSlot + 2 b + l.
enum BatchBuf { kBufZ = 0, kBufU0, kBufU1, kBufUB, kBufDB, kBufL0, kBufL1, kBufNone = 15, kBufSlot = 16 };
// Program steps.  Every shot executes each one; a device-wide barrier follows each.
//   kOpFwd:      forward steps n .. d-1 from u^n in a and u^{n-1} in b, each a stencil phase and
//                a phase that injects the source sample and (for steps s >= e) gathers data row
//                s+1; the output of each step is the work buffer (kBufU0 / kBufU1) that does not
//                hold its input, as in the solo executor
//   kOpAdj:      adjoint step k = n, a = lam^k, b = lam^{k+1} (the output, in place), c = u^k: a
//                stencil phase with the gradient term, then the residual injection of row k
//   kOpEncCount: bit counts of the chunks of a store: a = u^k, b = u^{k-1} (kBufNone: one field)
//   kOpEncEmit:  the store's streams at offs[d] (and offs[d+1] for the second field), next offset at
//                offs[d+2] (one field) or offs[d+1], offs[d+2]; n = k (stream size recorded), -1 none
//   kOpDec:      decode the stream at offs[d] into a (b != kBufNone: a = b - decoded)
//   kOpCopy:     copy field a into b
//   kOpResid:    residual r = d_sim - d_obs, partial sums of r^2, finiteness of field a
//   kOpMisfit:   phi = 1/2 sum of the partials
enum BatchOpKind { kOpNop = 0, kOpFwd, kOpAdj, kOpEncCount, kOpEncEmit, kOpDec, kOpCopy, kOpResid, kOpMisfit };
struct BatchOp {
    int32_t kind, n, a, b, c, d, e;
};

struct BatchArgs {
    Grid g;
    CodecDims cd;
    const BatchShot *shots;
    int nshots;
    const BatchOp *ops;
    int nops;
    double gscale;
    double tol;
    int minexp;
    int nrec;                 // receivers per shot (every shot of a batch has as many)
    int src_pts, rec_pts;     // largest scatter-table size over the shots (sources, receivers)
    int nt;
    int zlen;                 // rows per stencil work item
    long long slot_elems;     // elements of one uncompressed checkpoint slot (two fields)
    unsigned *bar;            // device-wide barrier words: group counters, top, generation, abort (zero at launch)
    int nwg;                  // workgroups of the launch (at most what the device holds at once)
    unsigned spin_limit;      // polls before a barrier gives up and the launch aborts
};
// Workgroups the persistent kernel can keep resident for space order 2K (0 on error).
int batch2d_resident_workgroups(int K);
// Launch of the persistent kernel with A.nwg workgroups.
hipError_t launch_batch2d(const BatchArgs &A, int K, hipStream_t s);

}  // namespace wv
