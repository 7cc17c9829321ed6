// Batched 2-D solver: one persistent kernel advances several 2-D shots together.
//
// Shots are independent (the paper computes one gradient per shot and sums them,
// Sec. "Example adjoint problem: Seismic inversion"), and small 2-D shots cannot fill
// the GPU one launch at a time: a 512^2 step is a few microseconds of work behind a
// launch of about the same cost.  So shots of one grid, space order, step count and
// checkpoint schedule run as one batch: the host turns the schedule into a program of
// phases (stencil steps, source and residual injections, checkpoint encodes and
// decodes, the misfit), and a persistent kernel, launched once for the whole reversal,
// executes every phase for every shot of the batch, with a device-wide barrier between
// phases.  Each shot's arithmetic is the solo solver's (the same point update,
// injection, gather, codec block and reduction code, in the same order), so a shot
// gives the same bits alone, in a solo call and in any batch.
#include "wv_codec_dev.h"
#include "wv_stencil_dev.h"

namespace wv {

namespace {

constexpr int kBatchParts = 1024;   // residual partial sums per shot (as the solo misfit)
constexpr int kCopyItem = 65536;    // elements per copy or finiteness work item

__device__ __forceinline__ float *batch_buf(const BatchShot &S, int id, long long slot_elems, long long P)
{
    switch (id) {
    case kBufZ: return S.Z;
    case kBufU0: return S.U[0];
    case kBufU1: return S.U[1];
    case kBufUB: return S.UB;
    case kBufDB: return S.DB;
    case kBufL0: return S.Lm[0];
    case kBufL1: return S.Lm[1];
    case kBufNone: return nullptr;
    default: {
        const int b = (id - kBufSlot) >> 1, l = (id - kBufSlot) & 1;
        return reinterpret_cast<float *>(S.arena) + (long long)(b - 1) * slot_elems + (long long)l * P;
    }
    }
}

// Device-wide barrier of the persistent launch.  Two levels: workgroup b arrives at the
// counter of its group b % 8 (the XCD it runs on under round-robin dispatch), the last
// arrival of a group at the top counter, and the last of those resets it and advances the
// generation; everyone else waits for the generation to move.  Counters, top, generation
// and the abort word sit 1 KB apart so that arrivals of different groups and the polling
// do not meet on one line.  Memory order: a release fence before each arrival, acquire +
// release fences around the group's and the top's last arrival, relaxed polling (an
// acquire poll would invalidate the L2 on every spin) and one acquire fence after the
// wait, so every write of the phase is visible to every workgroup of the next.
// The barrier needs every workgroup resident.  The spin is bounded (spin_limit polls, 2^18
// by default: a fraction of a second, where a phase takes microseconds): past the bound, or when another
// workgroup has given up, it sets err bit 16 and the abort word and returns false, and the
// kernel ends at once; the host then runs the batch's shots one by one.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned nwg, unsigned spin_limit, unsigned *err,
                                             unsigned *s_flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned ng = nwg < 8u ? nwg : 8u;
        const unsigned grp = blockIdx.x & 7u;
        const unsigned in_grp = (nwg - grp + 7u) / 8u;
        unsigned *sub = bar + 256u * grp, *top = bar + 2048, *gen = bar + 3072, *abort = bar + 3584;
        const unsigned g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bool waiting = true, ok = true;
        if (__hip_atomic_fetch_add(sub, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == in_grp - 1u) {
            __hip_atomic_store(sub, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            if (__hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ng - 1u) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                waiting = false;
            }
        }
        if (waiting) {
            unsigned spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                if (++spins > spin_limit || __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    atomicOr(err, 16u);
                    __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_flag = ok ? 1u : 0u;
    }
    __syncthreads();
    return *s_flag != 0u;
}

// inclusive workgroup scan of v (s_scan: scratch for the wave totals); the trailing
// barrier lets the caller reuse s_scan at once
__device__ __forceinline__ unsigned block_scan(unsigned *s_scan, unsigned v, unsigned &total)
{
    const unsigned r = wg_scan256(v, s_scan, total);
    __syncthreads();
    return r;
}

// sum of w[0..n) by one workgroup (wave 0 does the adding), broadcast through *out
__device__ __forceinline__ unsigned long long block_sum_words(const uint32_t *w, long long n,
                                                              unsigned long long *out)
{
    if (threadIdx.x < 64) {
        unsigned long long s = 0;
        for (long long i = threadIdx.x; i < n; i += 64) s += w[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (threadIdx.x == 0) *out = s;
    }
    __syncthreads();
    const unsigned long long r = *out;
    __syncthreads();
    return r;
}

template <bool VEC>
__device__ __forceinline__ void load_block2(const float *f, const float *sub, const CodecDims &cd, long long b,
                                            float *v)
{
    const int bx = (int)(b % cd.nb[0]);
    const int by = (int)((b / cd.nb[0]) % cd.nb[1]);
    load_block<2, VEC>(f, sub, cd.dims, cd.pitch, bx, by, 0, v);
}

// Phase bodies.  A phase runs work items item = shot * per + j over all workgroups; every
// lane of a workgroup takes part in each of its items (items hold workgroup barriers).
struct BatchCtx {
    const BatchArgs &A;
    const Grid &g;
    const CodecDims &cd;
    long long P;
    int tiles_x, st_items;
    bool vec;
    long long nch;
};

template <typename Body>
__device__ __forceinline__ void for_items(const BatchArgs &A, int per, Body body)
{
    const int items = per * A.nshots;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int si = it / per;
        body(A.shots[si], it - si * per);
    }
}

// One forward (GRAD false) or adjoint (GRAD true) step of every shot, injections fused.
// Items [0, st_items) of a shot march one z-chunk of one 256-column tile, then add the
// injections whose grid point lies in that chunk and tile: the source's sample n into
// `out` (forward), or the residual's row n into `out` with its gradient term (adjoint).
// Every point has one owner, and its value is the stencil's and then the injection's, as
// in the solo solver.  Item st_items of a shot gathers the receivers of `gin` into data
// row `grow` (if grow >= 0): the deferred gather of the previous step's output, which
// nothing writes during this step.
template <int K, bool GRAD>
__device__ __forceinline__ void phase_step(const BatchCtx &C, int fin, int prev, int out, int uk, int n, int gin,
                                           int grow, float *s_row)
{
    const BatchArgs &A = C.A;
    const int tid = threadIdx.x, nx = C.g.nx;
    for_items(A, C.st_items + 1, [&](const BatchShot &S, int j) {
        if (j == C.st_items) {
            if (grow >= 0) {
                const float *f = batch_buf(S, gin, A.slot_elems, C.P);
                for (int r = tid; r < A.nrec; r += 256) S.dsim[(long long)grow * A.nrec + r] = gather_point(S.rec, r, f);
            }
            return;
        }
        const int tix = j % C.tiles_x, zc = j / C.tiles_x;
        const int z0 = zc * A.zlen, z1 = min(z0 + A.zlen, C.g.nz);
        float *f = batch_buf(S, out, A.slot_elems, C.P);
        const float *u = GRAD ? batch_buf(S, uk, A.slot_elems, C.P) : nullptr;
        march2d<K, GRAD, kOT2>(C.g, batch_buf(S, fin, A.slot_elems, C.P), batch_buf(S, prev, A.slot_elems, C.P), f,
                               S.W, u, nullptr, nullptr, GRAD ? S.G : nullptr, GRAD ? A.gscale : 0.0, tix, z0, z1,
                               s_row);
        __syncthreads();
        const Sparse &sp = GRAD ? S.rec : S.src;
        const int x0 = tix * 256, x1 = min(x0 + 256, nx);
        for (int i = tid; i < sp.npts; i += 256) {
            const int p = sp.s_pts[i];
            const int z = p / nx, x = p - z * nx;
            if (z < z0 || z >= z1 || x < x0 || x >= x1) continue;
            if constexpr (GRAD)
                inject_point<true>(C.g, sp, i, p, x, 0, z, S.res + (long long)n * A.nrec, S.W, f, u, S.G, p,
                                   A.gscale);
            else
                inject_point<false>(C.g, sp, i, p, x, 0, z, S.wavelet + n, S.W, f, nullptr, nullptr, p, 0.0);
        }
    });
}

// One workgroup per shot: the receivers of `gin` into data row `grow`.
__device__ __forceinline__ void phase_gather(const BatchCtx &C, int gin, int grow)
{
    const BatchArgs &A = C.A;
    for_items(A, 1, [&](const BatchShot &S, int) {
        const float *f = batch_buf(S, gin, A.slot_elems, C.P);
        for (int r = threadIdx.x; r < A.nrec; r += 256) S.dsim[(long long)grow * A.nrec + r] = gather_point(S.rec, r, f);
    });
}

__device__ __forceinline__ void phase_encode(const BatchCtx &C, const BatchOp &op, bool emit, unsigned *s_scan,
                             unsigned long long *s_words, unsigned long long *s_one)
{
    const BatchArgs &A = C.A;
    const CodecDims &cd = C.cd;
    const long long nch = C.nch;
    const int tid = threadIdx.x;
    for_items(A, (int)(op.b != kBufNone ? 2 * nch : nch), [&](const BatchShot &S, int j) {
        const int f = (int)(j / nch);
        const long long c = j - (long long)f * nch;
        const float *field = batch_buf(S, op.a, A.slot_elems, C.P);
        const float *sub = f == 1 ? batch_buf(S, op.b, A.slot_elems, C.P) : nullptr;
        const long long b = c * kBlocksPerChunk + tid;
        const bool valid = b < cd.nblocks;
        float v[16];
        if (valid) {
            if (C.vec) load_block2<true>(field, sub, cd, b, v);
            else load_block2<false>(field, sub, cd, b, v);
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = 0.0f;
        }
        BlockEnc<2> blk;
        uint32_t m_lo[32], m_hi[32];
        blk.prepare(v, valid, A.minexp, m_lo, m_hi);
        const unsigned nbits = blk.count(m_lo, m_hi);
        unsigned total_bits;
        const unsigned incl = block_scan(s_scan, nbits, total_bits);
        const uint32_t chunk_words = (total_bits + 63u) / 64u;
        __syncthreads();
        if (!emit) {
            if (!blk.finite) atomicOr(S.err, 2u);
            if (tid == 0) S.chunk_words[(long long)f * nch + c] = chunk_words;
            return;
        }
        // the stream of field f starts at its base; the second field's base follows the
        // first stream, rounded up to 256 bytes
        const unsigned long long words0 = block_sum_words(S.chunk_words, nch, s_one);
        uint64_t base = S.offs[op.d];
        if (f == 1) base += (cd.prefix_bytes + 8ull * words0 + 255ull) & ~255ull;
        const unsigned long long excl = block_sum_words(S.chunk_words + (long long)f * nch, c, s_one);
        const unsigned long long fwords = f == 0 ? words0 : block_sum_words(S.chunk_words + nch, nch, s_one);
        const uint64_t cap = S.arena_bytes;
        const bool prefix_fits = base + (uint64_t)cd.prefix_bytes <= cap;
        const bool fits = prefix_fits && base + (uint64_t)cd.prefix_bytes + (excl + chunk_words) * 8ull <= cap;
        uint8_t *hdr = S.arena + base;
        uint64_t *chunk_off = (uint64_t *)(hdr + 64);
        uint16_t *lens = (uint16_t *)(hdr + 64 + 8 * nch);
        if (valid && prefix_fits) lens[b] = (uint16_t)nbits;
        if (tid == 0 && prefix_fits) chunk_off[c] = excl;
        if (tid == 0 && !fits) atomicOr(S.err, 4u);
        unsigned long long *data = (unsigned long long *)(hdr + cd.prefix_bytes) + excl;
        const unsigned excl_bits = incl - nbits;
        if (fits && chunk_words <= (uint32_t)kLdsWords) {
            for (uint32_t q = tid; q < chunk_words; q += 256) s_words[q] = 0ull;
            __syncthreads();
            if (valid) {
                auto sink = [&](long long w, unsigned long long bits) { atomicOr(&s_words[w], bits); };
                blk.emit((long long)excl_bits, sink, m_lo, m_hi);
            }
            __syncthreads();
            for (uint32_t q = tid; q < chunk_words; q += 256) data[q] = s_words[q];
        } else if (fits) {
            for (uint32_t q = tid; q < chunk_words; q += 256) data[q] = 0ull;
            __syncthreads();
            if (valid) {
                auto sink = [&](long long w, unsigned long long bits) { atomicOr(&data[w], bits); };
                blk.emit((long long)excl_bits, sink, m_lo, m_hi);
            }
        }
        __syncthreads();
        if (c == nch - 1 && tid == 0) {
            const unsigned long long total = (unsigned long long)cd.prefix_bytes + 8ull * fwords;
            if (prefix_fits) {
                uint32_t *h32 = (uint32_t *)hdr;
                h32[0] = kMagic;
                h32[1] = kVersion;
                h32[2] = 2u;
                h32[3] = (uint32_t)cd.dims[0];
                h32[4] = (uint32_t)cd.dims[1];
                h32[5] = (uint32_t)cd.dims[2];
                *(double *)(hdr + 24) = A.tol;
                h32[8] = (uint32_t)cd.nblocks;
                h32[9] = (uint32_t)nch;
                h32[10] = kBlocksPerChunk;
                h32[11] = 0;
                *(unsigned long long *)(hdr + 48) = fwords;
                *(unsigned long long *)(hdr + 56) = total;
                const long long lb = 64 + 8 * nch + 2 * cd.nblocks;
                for (long long q = lb; q < cd.prefix_bytes; ++q) hdr[q] = 0;
            }
            const unsigned long long nxt = base + ((total + 255ull) & ~255ull);
            // next offset: after a single field at d+2; of two, the first ends at d+1
            S.offs[op.d + ((op.b != kBufNone && f == 0) ? 1 : 2)] = nxt;
            if (f == 0 && op.n >= 0) S.sizes[op.n] = total;
            atomicAdd(&S.stats[0], total);
            atomicMax(&S.stats[1], nxt);
        }
    });
}

__device__ __forceinline__ void phase_decode(const BatchCtx &C, const BatchOp &op, unsigned *s_scan, unsigned long long *s_words)
{
    const BatchArgs &A = C.A;
    const CodecDims &cd = C.cd;
    const long long nch = C.nch;
    const int tid = threadIdx.x;
    for_items(A, (int)nch, [&](const BatchShot &S, int j) {
        float *field = batch_buf(S, op.a, A.slot_elems, C.P);
        const float *sub = op.b != kBufNone ? batch_buf(S, op.b, A.slot_elems, C.P) : nullptr;
        const long long c = j;
        const long long b = c * kBlocksPerChunk + tid;
        const bool valid = b < cd.nblocks;
        const uint64_t boff = S.offs[op.d];
        const uint64_t cap = S.arena_bytes;
        if (boff + (uint64_t)cd.prefix_bytes > cap) {
            // a stream outside the arena (an overflowed store) decodes to zeros, as in the
            // solo decoder
            if (valid) {
                float zero[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) zero[q] = 0.0f;
                if (C.vec) store_block<2, true>(field, sub, cd.dims, cd.pitch, cd.nb, b, zero);
                else store_block<2, false>(field, sub, cd.dims, cd.pitch, cd.nb, b, zero);
            }
            return;
        }
        const uint8_t *hdr = S.arena + boff;
        const uint64_t *chunk_off = (const uint64_t *)(hdr + 64);
        const uint16_t *lens = (const uint16_t *)(hdr + 64 + 8 * nch);
        const unsigned long long *data = (const unsigned long long *)(hdr + cd.prefix_bytes);
        long long nwords = (long long)*(const unsigned long long *)(hdr + 48);
        const long long maxw = (long long)((cap - boff - (uint64_t)cd.prefix_bytes) / 8);
        nwords = nwords < maxw ? nwords : maxw;
        const double tol = *(const double *)(hdr + 24);
        int te;
        frexp(tol, &te);
        const int minexp = te - 1;
        const unsigned nbits = valid ? lens[b] : 0u;
        unsigned total_bits;
        const unsigned incl = block_scan(s_scan, nbits, total_bits);
        long long cbase = (long long)chunk_off[c];
        cbase = cbase < 0 ? 0 : (cbase > nwords ? nwords : cbase);
        const long long cw = ((long long)total_bits + 63) / 64 + 1;
        const bool staged = cw <= kDecLdsWords;
        if (staged) {
            for (long long q = tid; q < cw; q += 256) {
                const long long jw = cbase + q;
                s_words[q] = (jw >= 0 && jw < nwords) ? data[jw] : 0ull;
            }
        }
        __syncthreads();
        if (valid) {
            const long long rel = (long long)(incl - nbits);
            BitReader rd = staged ? BitReader{s_words, cw, 0, 0ull, 0ull, 0} : BitReader{data, nwords, 0, 0ull, 0ull, 0};
            rd.init(staged ? rel : cbase * 64 + rel);
            float out[16];
            decode_block<2>(rd, minexp, out);
            if (C.vec) store_block<2, true>(field, sub, cd.dims, cd.pitch, cd.nb, b, out);
            else store_block<2, false>(field, sub, cd.dims, cd.pitch, cd.nb, b, out);
        }
        __syncthreads();
    });
}

// residual r = d_sim - d_obs and its partial sums of r^2 (the solo misfit's blocks and
// order), plus the finiteness check of the last forward state (field a)
__device__ __forceinline__ void phase_residual(const BatchCtx &C, int ufield, double *s_red)
{
    const BatchArgs &A = C.A;
    const int tid = threadIdx.x;
    const int nfin = (int)((C.P + kCopyItem - 1) / kCopyItem);
    for_items(A, kBatchParts + nfin, [&](const BatchShot &S, int j) {
        if (j < kBatchParts) {
            const long long n = (long long)(A.nt + 1) * A.nrec;
            double acc = 0.0;
            for (long long e = (long long)j * 256 + tid; e < n; e += (long long)kBatchParts * 256) {
                if (e < A.nrec) {
                    S.res[e] = 0.0f;
                    continue;
                }
                const double r = (double)S.dsim[e] - (double)S.dobs[e];
                S.res[e] = (float)r;
                acc += r * r;
            }
            s_red[tid] = acc;
            __syncthreads();
            for (int sft = 128; sft > 0; sft >>= 1) {
                if (tid < sft) s_red[tid] += s_red[tid + sft];
                __syncthreads();
            }
            if (tid == 0) S.partials[j] = s_red[0];
            __syncthreads();
        } else {
            const float *u = batch_buf(S, ufield, A.slot_elems, C.P);
            const long long e0 = (long long)(j - kBatchParts) * kCopyItem, e1 = min(e0 + kCopyItem, C.P);
            bool bad = false;
            for (long long e = e0 + tid; e < e1; e += 256) bad |= !isfinite(u[e]);
            if (bad) atomicOr(S.err, 8u);
        }
    });
}

// phi = 1/2 sum of the partials (the solo final sum's order)
__device__ __forceinline__ void phase_misfit(const BatchCtx &C, double *s_red)
{
    const int tid = threadIdx.x;
    for_items(C.A, 1, [&](const BatchShot &S, int) {
        double acc = 0.0;
        for (int q = tid; q < kBatchParts; q += 256) acc += S.partials[q];
        s_red[tid] = acc;
        __syncthreads();
        for (int sft = 128; sft > 0; sft >>= 1) {
            if (tid < sft) s_red[tid] += s_red[tid + sft];
            __syncthreads();
        }
        if (tid == 0) S.misfit[0] = 0.5 * s_red[0];
        __syncthreads();
    });
}

__device__ __forceinline__ void phase_copy(const BatchCtx &C, int src, int dst)
{
    const BatchArgs &A = C.A;
    for_items(A, (int)((C.P + kCopyItem - 1) / kCopyItem), [&](const BatchShot &S, int j) {
        const float *a = batch_buf(S, src, A.slot_elems, C.P);
        float *b = batch_buf(S, dst, A.slot_elems, C.P);
        const long long e0 = (long long)j * kCopyItem, e1 = min(e0 + kCopyItem, C.P);
        for (long long e = e0 + threadIdx.x; e < e1; e += 256) b[e] = a[e];
    });
}

template <int K>
__global__ __launch_bounds__(256) void batch2d_kernel(BatchArgs A)
{
    __shared__ unsigned s_scan[4];
    __shared__ unsigned long long s_words[kDecLdsWords];
    __shared__ unsigned long long s_one;
    __shared__ float s_row[256 + 2 * K];
    __shared__ double s_red[256];
    const int tiles_x = (A.g.nx + 255) / 256;
    const BatchCtx C{A, A.g, A.cd, A.g.P, tiles_x, tiles_x * ((A.g.nz + A.zlen - 1) / A.zlen),
                     A.cd.dims[0] % 4 == 0 && A.cd.pitch % 4 == 0, A.cd.nchunks};
    __shared__ unsigned s_flag;
    unsigned *err0 = A.shots[0].err;
    auto barrier = [&]() { return grid_barrier(A.bar, (unsigned)A.nwg, A.spin_limit, err0, &s_flag); };

    for (int oi = 0; oi < A.nops; ++oi) {
        const BatchOp op = A.ops[oi];
        switch (op.kind) {
        case kOpFwd: {
            // step n writes u^{n+1}; its gather (n >= op.e) runs in the next step's phase,
            // or in a phase of its own after the last step
            int fin = op.a, prev = op.b, grow = -1, gin = kBufNone;
            for (int n = op.n; n < op.d; ++n) {
                const int out = fin == kBufU0 ? kBufU1 : kBufU0;
                phase_step<K, false>(C, fin, prev, out, kBufNone, n, gin, grow, s_row);
                if (!barrier()) return;
                grow = n >= op.e ? n + 1 : -1;
                gin = out;
                prev = fin;
                fin = out;
            }
            if (grow >= 0) {
                phase_gather(C, gin, grow);
                if (!barrier()) return;
            }
            break;
        }
        case kOpAdj:
            phase_step<K, true>(C, op.a, op.b, op.b, op.c, op.n, kBufNone, -1, s_row);
            if (!barrier()) return;
            break;
        case kOpEncCount:
            phase_encode(C, op, false, s_scan, s_words, &s_one);
            if (!barrier()) return;
            break;
        case kOpEncEmit:
            phase_encode(C, op, true, s_scan, s_words, &s_one);
            if (!barrier()) return;
            break;
        case kOpDec:
            phase_decode(C, op, s_scan, s_words);
            if (!barrier()) return;
            break;
        case kOpCopy:
            phase_copy(C, op.a, op.b);
            if (!barrier()) return;
            break;
        case kOpResid:
            phase_residual(C, op.a, s_red);
            if (!barrier()) return;
            break;
        case kOpMisfit:
            phase_misfit(C, s_red);
            if (!barrier()) return;
            break;
        default:
            break;
        }
    }
}

template <int K>
int resident_of()
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch2d_kernel<K>, 256, 0) != hipSuccess) return 0;
    return cus * per_cu;
}

// A plain launch: the grid is at most what the device holds at once, and a barrier that
// does not complete (workgroups kept out by other streams' kernels) aborts the launch.
template <int K>
hipError_t launch_of(const BatchArgs &A, hipStream_t s)
{
    hipLaunchKernelGGL(batch2d_kernel<K>, dim3(A.nwg), dim3(256), 0, s, A);
    return hipGetLastError();
}

}  // namespace

int batch2d_resident_workgroups(int K)
{
    switch (K) {
    case 1: return resident_of<1>();
    case 2: return resident_of<2>();
    case 3: return resident_of<3>();
    case 4: return resident_of<4>();
    case 5: return resident_of<5>();
    case 6: return resident_of<6>();
    case 7: return resident_of<7>();
    case 8: return resident_of<8>();
    default: return 0;
    }
}

hipError_t launch_batch2d(const BatchArgs &A, int K, hipStream_t s)
{
    switch (K) {
    case 1: return launch_of<1>(A, s);
    case 2: return launch_of<2>(A, s);
    case 3: return launch_of<3>(A, s);
    case 4: return launch_of<4>(A, s);
    case 5: return launch_of<5>(A, s);
    case 6: return launch_of<6>(A, s);
    case 7: return launch_of<7>(A, s);
    case 8: return launch_of<8>(A, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace wv
