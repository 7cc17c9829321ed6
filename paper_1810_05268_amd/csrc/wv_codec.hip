// ZFP-kind fixed-accuracy codec for binary32 checkpoints (gfx950).
//
// The paper stores every checkpoint through ZFP in its fixed-tolerance mode, i.e.
// with an absolute error bound (Sec. "Lossy Compression").  This codec follows the
// published ZFP block scheme (Lindstrom 2014): 4^d blocks, a common block exponent,
// block-floating-point integers, a separable decorrelating lifting transform, a
// sequency reordering, negabinary coefficients and embedded bit-plane coding with
// group tests, truncated at the plane that guarantees the tolerance.  The stream
// container is this library's own (documented in wv.h), designed for the GPU:
//   * one lane encodes one block, so a 256-lane workgroup encodes a chunk of 256
//     blocks; a block's bit length has a closed form per bit plane, so each lane
//     first counts its bits and the workgroup scans them;
//   * three launches place the chunks: every chunk counts its words and assembles
//     its bits at chunk-local positions in a staging slot; one workgroup scans the
//     word counts into offsets; every chunk copies its slot to its offset (a chunk
//     longer than a slot, or every chunk without staging, is encoded again there).
//     No workgroup waits for another: a single pass with a look-back over the
//     preceding chunks spent most of its time in those waits, each a trip to memory;
//   * chunks start at 64-bit word boundaries and record their word offsets, so the
//     decoder needs only a per-chunk scan of the 16-bit block lengths and every
//     block decodes independently.
#include "wv_codec_dev.h"

namespace wv {

namespace {

struct EncArgs {
    const float *field;
    const float *sub;        // nullable: encode field - sub
    int dims[3];
    int pitch;               // elements between rows of field and sub
    int nb[3];
    long long nblocks, nchunks, prefix_bytes;
    int ndim;
    int minexp;
    double tol;
    uint8_t *out;
    uint64_t cap;
    const uint64_t *base;
    uint64_t *next;
    uint32_t *words;         // per chunk: its stream words
    uint64_t *offs;          // per chunk: its first word in the data area
    unsigned long long *staging;   // nullable: slot_words words per chunk
    int slot_words;
    uint64_t *size_out;      // nullable: receives the stream's size in bytes
    unsigned *err;
    unsigned long long *stats;
};

// The blocks of chunk c: values, exponent, transform, planes and bit counts, and the
// workgroup scan of the counts; returns whether the lane has a block.  The planes are
// the caller's local arrays (inside a struct they would be placed in scratch).  Every
// lane of the workgroup calls it.
template <int ND, bool VEC>
__device__ __forceinline__ bool chunk_prepare(const EncArgs &A, long long c, BlockEnc<ND> &blk,
                                              uint32_t (&m_lo)[32], uint32_t (&m_hi)[32], unsigned &nbits,
                                              unsigned &excl_bits, unsigned &total_bits, unsigned *s_scan)
{
    constexpr int S = ND == 3 ? 64 : 16;
    const long long b = c * kBlocksPerChunk + threadIdx.x;
    const bool valid = b < A.nblocks;
    float v[S];
    if (valid) {
        const int bx = (int)(b % A.nb[0]);
        const int by = (int)((b / A.nb[0]) % A.nb[1]);
        const int bz = (int)(b / ((long long)A.nb[0] * A.nb[1]));
        load_block<ND, VEC>(A.field, A.sub, A.dims, A.pitch, bx, by, bz, v);
    } else {
#pragma unroll
        for (int i = 0; i < S; ++i) v[i] = 0.0f;
    }
    blk.prepare(v, valid, A.minexp, m_lo, m_hi);
    nbits = blk.count(m_lo, m_hi);
    excl_bits = wg_scan256(nbits, s_scan, total_bits) - nbits;
    return valid;
}

// Exclusive scan of the chunk word counts into offs (and the stream's chunk offsets),
// then the header, the stream size and the next free offset; one workgroup.  Each lane
// sums a run of up to 16 counts held in registers.
__device__ __forceinline__ void scan_chunks(const EncArgs &A, unsigned long long *s_scan)
{
    const int tid = threadIdx.x;
    const long long n = A.nchunks;
    const long long per = (n + 1023) / 1024 * 4;   // a multiple of 4: whole uint4 loads
    const long long i0 = min((long long)tid * per, n), i1 = min(i0 + per, n);
    const uint32_t *__restrict__ words = A.words;
    constexpr int kReg = 16;
    uint32_t wr[kReg];
    const bool in_reg = per <= kReg && i1 - i0 == per;
    unsigned long long part = 0;
    if (in_reg) {
        const uint4 *w4 = reinterpret_cast<const uint4 *>(words + i0);   // 16-byte aligned
#pragma unroll
        for (int q = 0; q < kReg / 4; ++q) {
            const uint4 t = q < per / 4 ? w4[q] : make_uint4(0u, 0u, 0u, 0u);
            wr[4 * q] = t.x;
            wr[4 * q + 1] = t.y;
            wr[4 * q + 2] = t.z;
            wr[4 * q + 3] = t.w;
        }
#pragma unroll
        for (int k = 0; k < kReg; ++k) part += wr[k];
    } else {
        for (long long i = i0; i < i1; ++i) part += words[i];
    }
    unsigned long long data_words;
    unsigned long long run = wg_scan256(part, s_scan, data_words) - part;
    const uint64_t base = *A.base;
    const bool prefix_fits = base + (uint64_t)A.prefix_bytes <= A.cap;
    uint8_t *hdr = A.out + base;
    uint64_t *chunk_off = (uint64_t *)(hdr + kHdr);
    if (in_reg) {
#pragma unroll
        for (int k = 0; k < kReg; ++k)
            if (k < per) {
                A.offs[i0 + k] = run;
                if (prefix_fits) chunk_off[i0 + k] = run;
                run += wr[k];
            }
    } else {
        for (long long i = i0; i < i1; ++i) {
            A.offs[i] = run;
            if (prefix_fits) chunk_off[i] = run;
            run += words[i];
        }
    }
    if (tid != 0) return;
    const unsigned long long total = (unsigned long long)A.prefix_bytes + 8ull * data_words;
    if (!prefix_fits || base + total > A.cap) atomicOr(A.err, 4u);
    if (prefix_fits) {
        uint32_t *h32 = (uint32_t *)hdr;
        h32[0] = kMagic;
        h32[1] = kVersion;
        h32[2] = (uint32_t)A.ndim;
        h32[3] = (uint32_t)A.dims[0];
        h32[4] = (uint32_t)A.dims[1];
        h32[5] = (uint32_t)A.dims[2];
        *(double *)(hdr + 24) = A.tol;
        h32[8] = (uint32_t)A.nblocks;
        h32[9] = (uint32_t)A.nchunks;
        h32[10] = kBlocksPerChunk;
        h32[11] = 0;
        *(unsigned long long *)(hdr + 48) = data_words;
        *(unsigned long long *)(hdr + 56) = total;
        // zero the padding after the block lengths
        const long long lb = kHdr + 8 * A.nchunks + 2 * A.nblocks;
        for (long long i = lb; i < A.prefix_bytes; ++i) hdr[i] = 0;
    }
    const unsigned long long nxt = base + ((total + 255ull) & ~255ull);
    *A.next = nxt;
    if (A.size_out) *A.size_out = total;
    atomicAdd(&A.stats[0], total);
    atomicMax(&A.stats[1], nxt);
}

// Pass 1, one workgroup per chunk: the block lengths (into the stream's prefix), the
// chunk's word count, and, when it fits a staging slot, the chunk's bits, assembled in
// LDS at chunk-local positions.  Chunks are independent: no workgroup waits for another.
template <int ND, bool VEC>
__global__ __launch_bounds__(256, 4) void encode_count_kernel(EncArgs A)
{
    __shared__ unsigned s_scan[4];
    __shared__ unsigned long long s_bits[kLdsWords];
    const int tid = threadIdx.x;
    const long long c = blockIdx.x;
    const uint64_t base = *A.base;
    const bool prefix_fits = base + (uint64_t)A.prefix_bytes <= A.cap;
    BlockEnc<ND> blk;
    uint32_t m_lo[32], m_hi[32];
    unsigned nbits, excl_bits, total_bits;
    const bool valid = chunk_prepare<ND, VEC>(A, c, blk, m_lo, m_hi, nbits, excl_bits, total_bits, s_scan);
    if (!blk.finite) atomicOr(A.err, 2u);
    const long long b = c * kBlocksPerChunk + tid;
    if (valid && prefix_fits) {
        uint16_t *lens = (uint16_t *)(A.out + base + kHdr + 8 * A.nchunks);
        lens[b] = (uint16_t)nbits;
    }
    const uint32_t cw = (total_bits + 63u) / 64u;
    if (tid == 0) A.words[c] = cw;
    if (A.staging && cw <= (uint32_t)A.slot_words) {   // else encoded again by pass 3
        for (uint32_t i = tid; i < cw; i += 256) s_bits[i] = 0ull;
        __syncthreads();
        if (valid) {
            auto sink = [&](long long w, unsigned long long bits) { atomicOr(&s_bits[w], bits); };
            blk.emit((long long)excl_bits, sink, m_lo, m_hi);
        }
        __syncthreads();
        unsigned long long *slot = A.staging + c * (long long)A.slot_words;
        for (uint32_t i = tid; i < cw; i += 256) slot[i] = s_bits[i];
    }
}

// Pass 2, one workgroup: the offsets scan (a kernel of its own: finishing pass 1 with a
// last-workgroup scan needs an agent-scope release in every workgroup, each an L2
// write-back, which cost more than this launch).
__global__ __launch_bounds__(256) void encode_scan_kernel(EncArgs A)
{
    __shared__ unsigned long long s_scan64[4];
    scan_chunks(A, s_scan64);
}

// Pass 3, one workgroup per chunk: a staged chunk is copied to its offset; a chunk too
// long for its slot (or every chunk, without staging) is encoded again and emitted there.
template <int ND, bool VEC>
__global__ __launch_bounds__(256) void encode_place_kernel(EncArgs A)
{
    __shared__ unsigned s_scan[4];
    const int tid = threadIdx.x;
    const long long c = blockIdx.x;
    const uint64_t base = *A.base;
    const uint32_t cw = A.words[c];
    const unsigned long long off = A.offs[c];
    if (base + (uint64_t)A.prefix_bytes + (off + cw) * 8ull > A.cap) return;   // flagged by pass 2
    unsigned long long *data = (unsigned long long *)(A.out + base + A.prefix_bytes) + off;
    if (A.staging && cw <= (uint32_t)A.slot_words) {
        const unsigned long long *slot = A.staging + c * (long long)A.slot_words;
        for (uint32_t i = tid; i < cw; i += 256) data[i] = slot[i];
        return;
    }
    BlockEnc<ND> blk;
    uint32_t m_lo[32], m_hi[32];
    unsigned nbits, excl_bits, total_bits;
    const bool valid = chunk_prepare<ND, VEC>(A, c, blk, m_lo, m_hi, nbits, excl_bits, total_bits, s_scan);
    for (uint32_t i = tid; i < cw; i += 256) data[i] = 0ull;
    __syncthreads();
    if (valid) {
        auto sink = [&](long long w, unsigned long long bits) { atomicOr(&data[w], bits); };
        blk.emit((long long)excl_bits, sink, m_lo, m_hi);
    }
}

struct DecArgs {
    const float *sub;        // nullable: store sub - decoded
    const uint8_t *in;
    const uint64_t *base;
    uint64_t cap;        // bytes readable from `in`
    float *field;
    int dims[3];
    int pitch;           // elements between rows of the field
    int nb[3];
    long long nblocks, nchunks, prefix_bytes;
};

template <int ND, bool VEC>
__global__ __launch_bounds__(256) void decode_kernel(DecArgs A)
{
    constexpr int S = ND == 3 ? 64 : 16;
    __shared__ unsigned s_scan[4];
    __shared__ unsigned long long s_words[kDecLdsWords];
    const int tid = threadIdx.x;
    const long long c = blockIdx.x;
    const long long b = c * kBlocksPerChunk + tid;
    const bool valid = b < A.nblocks;
    const uint64_t boff = A.base ? *A.base : 0ull;
    if (boff + (uint64_t)A.prefix_bytes > A.cap) {
        // stream outside the readable range (an overflowed store): decode zeros
        if (valid) {
            const int bx = (int)(b % A.nb[0]);
            const int by = (int)((b / A.nb[0]) % A.nb[1]);
            const int bz = (int)(b / ((long long)A.nb[0] * A.nb[1]));
            const int nzz = ND == 3 ? A.dims[2] : 1;
            for (int k = 0; k < (ND == 3 ? 4 : 1); ++k)
                for (int j = 0; j < 4; ++j)
                    for (int i = 0; i < 4; ++i) {
                        const int x = 4 * bx + i, y = 4 * by + j, z = 4 * bz + k;
                        if (x < A.dims[0] && y < A.dims[1] && z < nzz) {
                            const long long p = ((long long)z * A.dims[1] + y) * A.pitch + x;
                            A.field[p] = A.sub ? A.sub[p] : 0.0f;
                        }
                    }
        }
        return;
    }
    const uint8_t *hdr = A.in + boff;
    const uint64_t *chunk_off = (const uint64_t *)(hdr + kHdr);
    const uint16_t *lens = (const uint16_t *)(hdr + kHdr + 8 * A.nchunks);
    const unsigned long long *data = (const unsigned long long *)(hdr + A.prefix_bytes);
    long long nwords = (long long)*(const unsigned long long *)(hdr + 48);
    const long long maxw = (long long)((A.cap - boff - (uint64_t)A.prefix_bytes) / 8);
    nwords = nwords < maxw ? nwords : maxw;
    const double tol = *(const double *)(hdr + 24);
    int te;
    frexp(tol, &te);
    const int minexp = te - 1;

    const unsigned nbits = valid ? lens[b] : 0u;
    unsigned total_bits;
    const unsigned incl = wg_scan256(nbits, s_scan, total_bits);
    // The chunk's words are contiguous: stage them in LDS with one coalesced pass, so
    // that each lane's sequential bit reads are LDS reads instead of a chain of
    // dependent global loads.  Chunks too long for the buffer read global memory.
    // a chunk offset outside the data words (only a corrupt stream has one) is clamped,
    // so that every word read below stays inside the readable range
    long long cbase = (long long)chunk_off[c];
    cbase = cbase < 0 ? 0 : (cbase > nwords ? nwords : cbase);
    const long long cw = ((long long)total_bits + 63) / 64 + 1;   // + the reader's look-ahead word
    const bool staged = cw <= kDecLdsWords;
    if (staged) {
        for (long long i = tid; i < cw; i += 256) {
            const long long j = cbase + i;
            s_words[i] = (j >= 0 && j < nwords) ? data[j] : 0ull;
        }
    }
    __syncthreads();
    if (!valid) return;
    const long long rel = (long long)(incl - nbits);
    BitReader rd = staged ? BitReader{s_words, cw, 0, 0ull, 0ull, 0} : BitReader{data, nwords, 0, 0ull, 0ull, 0};
    rd.init(staged ? rel : cbase * 64 + rel);
    float out[S];
    decode_block<ND>(rd, minexp, out);
    store_block<ND, VEC>(A.field, A.sub, A.dims, A.pitch, A.nb, b, out);
}

}  // namespace

CodecDims codec_dims(int ndim, const int *dims, int pitch)
{
    CodecDims cd{};
    cd.ndim = ndim;
    cd.pitch = pitch > 0 ? pitch : dims[0];
    for (int a = 0; a < 3; ++a) {
        cd.dims[a] = (a < ndim) ? dims[a] : 1;
        cd.nb[a] = (a < ndim) ? (dims[a] + 3) / 4 : 1;
    }
    cd.nblocks = (long long)cd.nb[0] * cd.nb[1] * cd.nb[2];
    cd.nchunks = (cd.nblocks + kBlocksPerChunk - 1) / kBlocksPerChunk;
    cd.prefix_bytes = kHdr + 8 * cd.nchunks + ((2 * cd.nblocks + 7) / 8) * 8;
    return cd;
}

size_t codec_max_bytes(const CodecDims &cd)
{
    // worst case per block: 1 + 8 + 32 planes of (S verbatim + S group + 1) bits
    const long long S = cd.ndim == 3 ? 64 : 16;
    const long long per_block_bits = 9 + 32 * (2 * S + 1);
    const long long words = cd.nchunks + (cd.nblocks * per_block_bits + 63) / 64;
    return (size_t)(cd.prefix_bytes + 8 * words);
}

size_t encode_work_bytes(const CodecDims &cd, bool staged)
{
    const size_t n = (size_t)cd.nchunks;
    size_t b = (n * 4 + 255) / 256 * 256 + (n * 8 + 255) / 256 * 256;
    if (staged) b += n * (size_t)kLdsWords * 8;
    return b;
}

hipError_t launch_encode(const CodecDims &cd, const float *field, const float *sub, double tol, uint8_t *out,
                         uint64_t cap, const uint64_t *base, uint64_t *next, uint8_t *work, bool staged,
                         unsigned *err, unsigned long long *stats, hipStream_t s, uint64_t *size_out)
{
    EncArgs A{};
    A.field = field;
    A.sub = sub;
    for (int a = 0; a < 3; ++a) {
        A.dims[a] = cd.dims[a];
        A.nb[a] = cd.nb[a];
    }
    A.pitch = cd.pitch;
    A.nblocks = cd.nblocks;
    A.nchunks = cd.nchunks;
    A.prefix_bytes = cd.prefix_bytes;
    A.ndim = cd.ndim;
    int te;
    frexp(tol, &te);
    A.minexp = te - 1;
    A.tol = tol;
    A.out = out;
    A.cap = cap;
    A.base = base;
    A.next = next;
    const size_t n = (size_t)cd.nchunks;
    A.words = reinterpret_cast<uint32_t *>(work);
    A.offs = reinterpret_cast<uint64_t *>(work + (n * 4 + 255) / 256 * 256);
    A.staging = staged ? reinterpret_cast<unsigned long long *>(work + (n * 4 + 255) / 256 * 256 +
                                                                 (n * 8 + 255) / 256 * 256)
                       : nullptr;
    A.slot_words = staged ? kLdsWords : 0;
    A.size_out = size_out;
    A.err = err;
    A.stats = stats;
    const bool vec = cd.dims[0] % 4 == 0 && cd.pitch % 4 == 0;
    const dim3 grid((unsigned)cd.nchunks);
    if (cd.ndim == 3) {
        if (vec) hipLaunchKernelGGL((encode_count_kernel<3, true>), grid, dim3(256), 0, s, A);
        else hipLaunchKernelGGL((encode_count_kernel<3, false>), grid, dim3(256), 0, s, A);
    } else {
        if (vec) hipLaunchKernelGGL((encode_count_kernel<2, true>), grid, dim3(256), 0, s, A);
        else hipLaunchKernelGGL((encode_count_kernel<2, false>), grid, dim3(256), 0, s, A);
    }
    hipLaunchKernelGGL(encode_scan_kernel, dim3(1), dim3(256), 0, s, A);
    if (cd.ndim == 3) {
        if (vec) hipLaunchKernelGGL((encode_place_kernel<3, true>), grid, dim3(256), 0, s, A);
        else hipLaunchKernelGGL((encode_place_kernel<3, false>), grid, dim3(256), 0, s, A);
    } else {
        if (vec) hipLaunchKernelGGL((encode_place_kernel<2, true>), grid, dim3(256), 0, s, A);
        else hipLaunchKernelGGL((encode_place_kernel<2, false>), grid, dim3(256), 0, s, A);
    }
    return hipGetLastError();
}

hipError_t launch_decode(const CodecDims &cd, const uint8_t *in, const uint64_t *base, uint64_t cap, float *field,
                         const float *sub, hipStream_t s)
{
    DecArgs A{};
    A.sub = sub;
    A.in = in;
    A.base = base;
    A.cap = cap;
    A.field = field;
    for (int a = 0; a < 3; ++a) {
        A.dims[a] = cd.dims[a];
        A.nb[a] = cd.nb[a];
    }
    A.pitch = cd.pitch;
    A.nblocks = cd.nblocks;
    A.nchunks = cd.nchunks;
    A.prefix_bytes = cd.prefix_bytes;
    const bool vec = cd.dims[0] % 4 == 0 && cd.pitch % 4 == 0;
    const dim3 grid((unsigned)cd.nchunks);
    if (cd.ndim == 3) {
        if (vec) hipLaunchKernelGGL((decode_kernel<3, true>), grid, dim3(256), 0, s, A);
        else hipLaunchKernelGGL((decode_kernel<3, false>), grid, dim3(256), 0, s, A);
    } else {
        if (vec) hipLaunchKernelGGL((decode_kernel<2, true>), grid, dim3(256), 0, s, A);
        else hipLaunchKernelGGL((decode_kernel<2, false>), grid, dim3(256), 0, s, A);
    }
    return hipGetLastError();
}

}  // namespace wv
