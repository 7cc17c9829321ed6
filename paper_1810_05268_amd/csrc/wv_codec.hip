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
//     first counts its bits, the workgroup scans them, and the chunk's word offset
//     in the stream comes from a decoupled look-back over the preceding chunks
//     (one wave reads 256 predecessor status words per round);
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
    uint64_t *flags;
    uint32_t epoch;
    unsigned *ticket;        // chunk order = start order (0 at launch, reset by the last taker)
    uint64_t *size_out;      // nullable: receives the stream's size in bytes
    unsigned *err;
    unsigned long long *stats;
};

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;

__device__ __forceinline__ uint64_t make_flag(uint64_t status, uint32_t epoch, uint32_t value)
{
    return status | ((uint64_t)(epoch & 0x3FFFFFFFu) << 32) | value;
}


template <int ND, bool VEC>
__global__ __launch_bounds__(256) void encode_kernel(EncArgs A)
{
    constexpr int S = ND == 3 ? 64 : 16;
    __shared__ unsigned s_scan[256];
    __shared__ unsigned long long s_excl;
    __shared__ unsigned long long s_bits[kLdsWords];
    const int tid = threadIdx.x;
    // Chunk index = the order in which workgroups start (an atomic ticket), so every
    // chunk a look-back waits for belongs to a workgroup that is already running or
    // finished, whatever else the device runs concurrently; the wait always ends.  The
    // workgroup taking the last ticket resets the word for the next launch.
    __shared__ unsigned s_chunk;
    if (tid == 0) {
        const unsigned t = atomicAdd(A.ticket, 1u);
        if (t == (unsigned)(A.nchunks - 1)) atomicExch(A.ticket, 0u);
        s_chunk = t;
    }
    __syncthreads();
    const long long c = s_chunk;
    const long long b = c * kBlocksPerChunk + tid;
    const bool valid = b < A.nblocks;
    const uint64_t base = *A.base;
    const bool prefix_fits = base + (uint64_t)A.prefix_bytes <= A.cap;

    int bx = 0, by = 0, bz = 0;
    if (valid) {
        bx = (int)(b % A.nb[0]);
        by = (int)((b / A.nb[0]) % A.nb[1]);
        bz = (int)(b / ((long long)A.nb[0] * A.nb[1]));
    }
    float v[S];
    if (valid) load_block<ND, VEC>(A.field, A.sub, A.dims, A.pitch, bx, by, bz, v);
    else {
#pragma unroll
        for (int i = 0; i < S; ++i) v[i] = 0.0f;
    }
    BlockEnc<ND> blk;
    uint32_t m_lo[32], m_hi[32];
    blk.prepare(v, valid, A.minexp, m_lo, m_hi);
    if (!blk.finite) atomicOr(A.err, 2u);
    const unsigned nbits = blk.count(m_lo, m_hi);
    uint8_t *hdr = A.out + base;
    uint64_t *chunk_off = (uint64_t *)(hdr + kHdr);
    uint16_t *lens = (uint16_t *)(hdr + kHdr + 8 * A.nchunks);
    if (valid && prefix_fits) lens[b] = (uint16_t)nbits;

    // workgroup inclusive scan of the bit counts
    s_scan[tid] = nbits;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned add = tid >= off ? s_scan[tid - off] : 0u;
        __syncthreads();
        s_scan[tid] += add;
        __syncthreads();
    }
    const unsigned excl_bits = s_scan[tid] - nbits;
    const unsigned total_bits = s_scan[255];
    const uint32_t chunk_words = (total_bits + 63u) / 64u;
    // successors may sum this chunk's size as soon as it is known
    if (tid == 0 && c > 0)
        __hip_atomic_store(&A.flags[c], make_flag(kFlagAgg, A.epoch, chunk_words), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);

    // A chunk that fits the LDS buffer is assembled there first: its bit positions are
    // chunk-local, so the emission needs no global offset and runs while the
    // predecessors finish (the look-back below then rarely waits).
    const bool in_lds = chunk_words <= (uint32_t)kLdsWords;
    if (in_lds) {
        for (uint32_t i = tid; i < chunk_words; i += 256) s_bits[i] = 0ull;
        __syncthreads();
        if (valid) {
            auto sink = [&](long long w, unsigned long long bits) { atomicOr(&s_bits[w], bits); };
            blk.emit((long long)excl_bits, sink, m_lo, m_hi);
        }
    }
    __syncthreads();

    // decoupled look-back: one wave reads 256 predecessor status words per round
    // (4 per lane, nearest first) and stops at the nearest inclusive prefix
    if (tid < 64) {
        const uint32_t ep = A.epoch & 0x3FFFFFFFu;
        unsigned long long excl = 0;
        if (c > 0) {
            long long top = c - 1;
            unsigned spins = 0;
            while (true) {
                uint64_t f[4];
                int firstp = 4;            // nearest prefix among this lane's four
                bool allok = true;         // every word up to (and incl.) that prefix is valid
                unsigned long long sum = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const long long j = top - 4 * tid - i;
                    f[i] = j >= 0 ? __hip_atomic_load(&A.flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : make_flag(kFlagPrefix, A.epoch, 0u);   // before the first chunk: 0
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint64_t st = f[i] & (3ull << 62);
                    const bool ok = st != 0 && (uint32_t)((f[i] >> 32) & 0x3FFFFFFFu) == ep;
                    if (firstp == 4) {
                        allok = allok && ok;
                        sum += ok ? (uint32_t)f[i] : 0u;
                        if (ok && st == kFlagPrefix) firstp = i;
                    }
                }
                const unsigned long long pm = __ballot(firstp < 4);
                const int fl = pm ? __ffsll((long long)pm) - 1 : 64;     // nearest lane with a prefix
                const unsigned long long bad = __ballot(!allok && tid <= fl);
                if (bad) {
                    if (++spins > (1u << 22)) {
                        if (tid == 0) atomicOr(A.err, 16u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                long long val = tid <= fl ? (long long)sum : 0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) val += __shfl_xor(val, o);
                excl += (unsigned long long)val;
                if (fl < 64) break;
                top -= 256;
            }
        }
        if (tid == 0) {
            __hip_atomic_store(&A.flags[c], make_flag(kFlagPrefix, A.epoch, (uint32_t)(excl + chunk_words)),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_excl = excl;
        }
    }
    __syncthreads();
    const unsigned long long excl = s_excl;
    const bool fits = prefix_fits &&
                      base + (uint64_t)A.prefix_bytes + (excl + chunk_words) * 8ull <= A.cap;
    if (tid == 0 && prefix_fits) chunk_off[c] = excl;
    if (tid == 0 && !fits) atomicOr(A.err, 4u);
    unsigned long long *data = (unsigned long long *)(hdr + A.prefix_bytes) + excl;

    if (fits && in_lds) {
        for (uint32_t i = tid; i < chunk_words; i += 256) data[i] = s_bits[i];
    } else if (fits) {
        for (uint32_t i = tid; i < chunk_words; i += 256) data[i] = 0ull;
        __syncthreads();
        if (valid) {
            auto sink = [&](long long w, unsigned long long bits) { atomicOr(&data[w], bits); };
            blk.emit((long long)excl_bits, sink, m_lo, m_hi);
        }
    }
    if (c == A.nchunks - 1 && tid == 0) {
        const unsigned long long data_words = excl + chunk_words;
        const unsigned long long total = (unsigned long long)A.prefix_bytes + 8ull * data_words;
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
    __shared__ unsigned s_scan[256];
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
    s_scan[tid] = nbits;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned add = tid >= off ? s_scan[tid - off] : 0u;
        __syncthreads();
        s_scan[tid] += add;
        __syncthreads();
    }
    // The chunk's words are contiguous: stage them in LDS with one coalesced pass, so
    // that each lane's sequential bit reads are LDS reads instead of a chain of
    // dependent global loads.  Chunks too long for the buffer read global memory.
    // a chunk offset outside the data words (only a corrupt stream has one) is clamped,
    // so that every word read below stays inside the readable range
    long long cbase = (long long)chunk_off[c];
    cbase = cbase < 0 ? 0 : (cbase > nwords ? nwords : cbase);
    const long long cw = ((long long)s_scan[255] + 63) / 64 + 1;   // + the reader's look-ahead word
    const bool staged = cw <= kDecLdsWords;
    if (staged) {
        for (long long i = tid; i < cw; i += 256) {
            const long long j = cbase + i;
            s_words[i] = (j >= 0 && j < nwords) ? data[j] : 0ull;
        }
    }
    __syncthreads();
    if (!valid) return;
    const long long rel = (long long)(s_scan[tid] - nbits);
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

hipError_t launch_encode(const CodecDims &cd, const float *field, const float *sub, double tol, uint8_t *out,
                         uint64_t cap, const uint64_t *base, uint64_t *next, uint64_t *flags, uint32_t epoch,
                         unsigned *ticket, unsigned *err, unsigned long long *stats, hipStream_t s,
                         uint64_t *size_out)
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
    A.flags = flags;
    A.epoch = epoch;
    A.ticket = ticket;
    A.size_out = size_out;
    A.err = err;
    A.stats = stats;
    const bool vec = cd.dims[0] % 4 == 0 && cd.pitch % 4 == 0;
    const dim3 grid((unsigned)cd.nchunks);
    if (cd.ndim == 3) {
        if (vec) hipLaunchKernelGGL((encode_kernel<3, true>), grid, dim3(256), 0, s, A);
        else hipLaunchKernelGGL((encode_kernel<3, false>), grid, dim3(256), 0, s, A);
    } else {
        if (vec) hipLaunchKernelGGL((encode_kernel<2, true>), grid, dim3(256), 0, s, A);
        else hipLaunchKernelGGL((encode_kernel<2, false>), grid, dim3(256), 0, s, A);
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
