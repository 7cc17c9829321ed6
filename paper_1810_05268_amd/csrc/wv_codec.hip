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
#include "wv_internal.h"

namespace wv {

namespace {

constexpr uint32_t kMagic = 0x4B50465Au;
constexpr uint32_t kVersion = 1u;
constexpr int kHdr = 64;

struct Perm { int v[64]; };

// Coefficient order: ascending total degree i+j+k, then i^2+j^2+k^2, then the
// slowest index first (k, j, i).  Built at compile time by insertion sort.
constexpr Perm make_perm(int nd)
{
    Perm p{};
    const int S = nd == 3 ? 64 : 16;
    int key[64][5]{};
    for (int v = 0; v < S; ++v) {
        const int i = v & 3, j = (v >> 2) & 3, k = (v >> 4) & 3;
        key[v][0] = i + j + k;
        key[v][1] = i * i + j * j + k * k;
        key[v][2] = k;
        key[v][3] = j;
        key[v][4] = i;
        p.v[v] = v;
    }
    for (int a = 1; a < S; ++a) {
        const int cur = p.v[a];
        int b = a - 1;
        while (b >= 0) {
            const int o = p.v[b];
            bool less = false;
            for (int t = 0; t < 5; ++t)
                if (key[cur][t] != key[o][t]) {
                    less = key[cur][t] < key[o][t];
                    break;
                }
            if (!less) break;
            p.v[b + 1] = o;
            --b;
        }
        p.v[b + 1] = cur;
    }
    return p;
}

constexpr Perm kPerm3 = make_perm(3);
constexpr Perm kPerm2 = make_perm(2);

// Forward lifting of four integers (stride s inside the block array):
// the exact-arithmetic map is (1/16)[[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],[-2,6,-6,2]].
__device__ __forceinline__ void fwd_lift(int32_t *p, const int S0, const int S)
{
    int32_t x = p[S0], y = p[S0 + S], z = p[S0 + 2 * S], w = p[S0 + 3 * S];
    x += w; x >>= 1; w -= x;
    z += y; z >>= 1; y -= z;
    x += z; x >>= 1; z -= x;
    w += y; w >>= 1; y -= w;
    w += y >> 1; y -= w >> 1;
    p[S0] = x; p[S0 + S] = y; p[S0 + 2 * S] = z; p[S0 + 3 * S] = w;
}

// Inverse: each real-valued forward step undone in reverse order (wrap-around
// arithmetic keeps any stream well defined).
__device__ __forceinline__ void inv_lift(int32_t *p, const int S0, const int S)
{
    uint32_t x = (uint32_t)p[S0], y = (uint32_t)p[S0 + S], z = (uint32_t)p[S0 + 2 * S], w = (uint32_t)p[S0 + 3 * S];
    y += (uint32_t)((int32_t)w >> 1); w -= (uint32_t)((int32_t)y >> 1);
    y += w; w <<= 1; w -= y;
    z += x; x <<= 1; x -= z;
    y += z; z <<= 1; z -= y;
    w += x; x <<= 1; x -= w;
    p[S0] = (int32_t)x; p[S0 + S] = (int32_t)y; p[S0 + 2 * S] = (int32_t)z; p[S0 + 3 * S] = (int32_t)w;
}

template <int ND>
__device__ __forceinline__ void fwd_transform(int32_t *q)
{
    if constexpr (ND == 3) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            fwd_lift(q, 16 * k + 0, 1); fwd_lift(q, 16 * k + 4, 1);
            fwd_lift(q, 16 * k + 8, 1); fwd_lift(q, 16 * k + 12, 1);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            fwd_lift(q, 16 * k + 0, 4); fwd_lift(q, 16 * k + 1, 4);
            fwd_lift(q, 16 * k + 2, 4); fwd_lift(q, 16 * k + 3, 4);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            fwd_lift(q, 4 * j + 0, 16); fwd_lift(q, 4 * j + 1, 16);
            fwd_lift(q, 4 * j + 2, 16); fwd_lift(q, 4 * j + 3, 16);
        }
    } else {
        fwd_lift(q, 0, 1); fwd_lift(q, 4, 1); fwd_lift(q, 8, 1); fwd_lift(q, 12, 1);
        fwd_lift(q, 0, 4); fwd_lift(q, 1, 4); fwd_lift(q, 2, 4); fwd_lift(q, 3, 4);
    }
}

template <int ND>
__device__ __forceinline__ void inv_transform(int32_t *q)
{
    if constexpr (ND == 3) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            inv_lift(q, 4 * j + 0, 16); inv_lift(q, 4 * j + 1, 16);
            inv_lift(q, 4 * j + 2, 16); inv_lift(q, 4 * j + 3, 16);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            inv_lift(q, 16 * k + 0, 4); inv_lift(q, 16 * k + 1, 4);
            inv_lift(q, 16 * k + 2, 4); inv_lift(q, 16 * k + 3, 4);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            inv_lift(q, 16 * k + 0, 1); inv_lift(q, 16 * k + 4, 1);
            inv_lift(q, 16 * k + 8, 1); inv_lift(q, 16 * k + 12, 1);
        }
    } else {
        inv_lift(q, 0, 4); inv_lift(q, 1, 4); inv_lift(q, 2, 4); inv_lift(q, 3, 4);
        inv_lift(q, 0, 1); inv_lift(q, 4, 1); inv_lift(q, 8, 1); inv_lift(q, 12, 1);
    }
}

__device__ __forceinline__ uint64_t low_mask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// In-place transpose of a 32 x 32 bit matrix: bit k of a[s] moves to bit s of a[k]
// (five stages of masked block swaps; an involution).
constexpr uint32_t kSwapMask[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};

__device__ __forceinline__ void transpose32(uint32_t *a)
{
#pragma unroll
    for (int st = 0; st < 5; ++st) {
        const int j = 16 >> st;
        const uint32_t m = kSwapMask[st];
#pragma unroll
        for (int s = 0; s < 32; ++s) {
            if (!(s & j)) {
                const uint32_t t = ((a[s] >> j) ^ a[s + j]) & m;
                a[s] ^= t << j;
                a[s + j] ^= t;
            }
        }
    }
}

// Bit emitter: bits accumulate in `acc` for the word that holds `pos`; each
// completed word, and the last partial one, goes to sink(word_index, bits), which
// ORs it into a zeroed word range (neighbouring lanes share edge words).
struct Emitter {
    long long pos;
    unsigned long long acc;
    template <typename Sink>
    __device__ __forceinline__ void put(unsigned long long v, int nb, Sink &sink)
    {
        const int off = (int)(pos & 63);
        acc |= v << off;
        if (off + nb >= 64) {
            sink(pos >> 6, acc);
            acc = off ? (v >> (64 - off)) : 0ull;
        }
        pos += nb;
    }
    template <typename Sink>
    __device__ __forceinline__ void flush(Sink &sink)
    {
        if (pos & 63) sink(pos >> 6, acc);
    }
};

struct BitReader {
    const unsigned long long *data;
    long long nw;
    long long widx;
    unsigned long long w0, w1;
    int off;
    __device__ __forceinline__ unsigned long long load(long long i) const
    {
        return (i >= 0 && i < nw) ? data[i] : 0ull;
    }
    __device__ __forceinline__ void init(long long pos)
    {
        widx = pos >> 6;
        off = (int)(pos & 63);
        w0 = load(widx);
        w1 = load(widx + 1);
    }
    __device__ __forceinline__ unsigned long long peek() const { return off ? (w0 >> off) | (w1 << (64 - off)) : w0; }
    __device__ __forceinline__ void skip(int nb)
    {
        off += nb;
        if (off >= 64) {
            off -= 64;
            ++widx;
            w0 = w1;
            w1 = load(widx + 1);
        }
    }
};

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

// Block values, axis 0 fastest; partial blocks repeat the last valid index.  With
// VEC (dims[0] % 4 == 0) every block is complete along x and each row is one
// float4 load with no branch, so all 16 row loads of a lane are in flight together.
template <int ND, bool VEC>
__device__ __forceinline__ void load_raw(const float *f, const int *dims, int pitch, int bx, int by, int bz,
                                         float *v)
{
    constexpr int KZ = ND == 3 ? 4 : 1;
    const int ny = dims[1];
    const int nzz = ND == 3 ? dims[2] : 1;
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
        const int z = min(4 * bz + k, nzz - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int y = min(4 * by + j, ny - 1);
            const float *row = f + ((long long)z * ny + y) * pitch;
            if constexpr (VEC) {
                const float4 t = *reinterpret_cast<const float4 *>(row + 4 * bx);
                v[16 * k + 4 * j + 0] = t.x;
                v[16 * k + 4 * j + 1] = t.y;
                v[16 * k + 4 * j + 2] = t.z;
                v[16 * k + 4 * j + 3] = t.w;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) v[16 * k + 4 * j + i] = row[min(4 * bx + i, dims[0] - 1)];
            }
        }
    }
}

// The block of f, or of f - sub (one binary32 subtraction per value) when sub is set.
template <int ND, bool VEC>
__device__ __forceinline__ void load_block(const float *f, const float *sub, const int *dims, int pitch, int bx,
                                           int by, int bz, float *v)
{
    constexpr int S = ND == 3 ? 64 : 16;
    load_raw<ND, VEC>(f, dims, pitch, bx, by, bz, v);
    if (sub) {
        float t[S];
        load_raw<ND, VEC>(sub, dims, pitch, bx, by, bz, t);
#pragma unroll
        for (int i = 0; i < S; ++i) v[i] -= t[i];
    }
}

constexpr int kLdsWords = 1024;      // chunk bitstreams up to 8 KB are assembled in LDS
constexpr int kDecLdsWords = 2048;   // and chunks up to 16 KB are staged in LDS for decoding

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
    int emax = -126;
    bool nonzero = false, finite = true;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const uint32_t u = __float_as_uint(v[i]);
        const int E = (int)((u >> 23) & 0xFFu);
        if (E == 255) finite = false;
        if (u & 0x7FFFFFFFu) {
            nonzero = true;
            const int e = E == 0 ? -126 : E - 126;
            emax = e > emax ? e : emax;
        }
    }
    if (!finite) atomicOr(A.err, 2u);
    int prec = emax - A.minexp + 2 * (ND + 1);
    prec = prec > 32 ? 32 : prec;
    const bool coded = valid && finite && nonzero && prec > 0;
    const int kmin = 32 - prec;

    // bit planes: m_lo[k] / m_hi[k] hold bit k of coefficients 0..31 / 32..63
    uint32_t m_lo[32], m_hi[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) m_lo[k] = m_hi[k] = 0u;
    // waves whose blocks are all empty or below the tolerance (most of an early
    // wavefield) skip the transform and the plane transposes
    if (__ballot(coded) != 0ull) {
        int32_t q[S];
#pragma unroll
        for (int i = 0; i < S; ++i) q[i] = coded ? (int32_t)ldexpf(v[i], 30 - emax) : 0;   // exact scaling, truncation
        fwd_transform<ND>(q);
#pragma unroll
        for (int s = 0; s < 32; ++s) {
            const int src = ND == 3 ? kPerm3.v[s] : kPerm2.v[s & 15];
            m_lo[s] = (s < S) ? (((uint32_t)q[src] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu) : 0u;
            if constexpr (ND == 3) m_hi[s] = (((uint32_t)q[kPerm3.v[32 + s]] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu);
            else m_hi[s] = 0u;
        }
        transpose32(m_lo);
        if constexpr (ND == 3) transpose32(m_hi);
    }
    // Planes run from 31 down to the lowest kmin of the wave in a plain (rolled)
    // loop: the plane index is wave-uniform, so m_lo[k] / m_hi[k] stay in registers
    // (indexed moves), and each lane skips the planes below its own kmin.
    int kmin_w = coded ? kmin : 32;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kmin_w = min(kmin_w, __shfl_xor(kmin_w, o));
    kmin_w = __builtin_amdgcn_readfirstlane(kmin_w);

    // closed-form bit count of the block
    unsigned nbits = valid ? 1u : 0u;
    if (coded) nbits += 8;
    {
        int n = 0;
#pragma unroll 1
        for (int k = 31; k >= kmin_w; --k) {
            if (coded && k >= kmin) {
                nbits += n;
                if (n < S) {
                    const unsigned long long r = ((unsigned long long)m_hi[k] << 32 | m_lo[k]) >> n;
                    if (r == 0ull) nbits += 1;
                    else {
                        const int pt = 63 - __clzll((long long)r);
                        nbits += pt + 1 + __popcll(r);
                        n += pt + 1;
                        if (n < S) nbits += 1;
                    }
                }
            }
        }
    }
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

    auto emit = [&](auto &sink) {
        Emitter em{(long long)excl_bits, 0ull};
        em.put(coded ? 1ull : 0ull, 1, sink);
        if (coded) em.put((unsigned long long)(emax + 127), 8, sink);
        {
            int n = 0;
#pragma unroll 1
            for (int k = 31; k >= kmin_w; --k) {
                if (coded && k >= kmin) {
                    const unsigned long long mk = (unsigned long long)m_hi[k] << 32 | m_lo[k];
                    if (n > 0) em.put(mk & low_mask(n), n, sink);
                    if (n < S) {
                        unsigned long long r = mk >> n;
                        while (r != 0ull) {
                            const int z = __ffsll((long long)r) - 1;
                            em.put(1ull, 1, sink);
                            em.put(1ull << z, z + 1, sink);
                            n += z + 1;
                            r = (z + 1 < 64) ? (r >> (z + 1)) : 0ull;
                        }
                        if (n < S) em.put(0ull, 1, sink);
                    }
                }
            }
        }
        em.flush(sink);
    };

    // A chunk that fits the LDS buffer is assembled there first: its bit positions are
    // chunk-local, so the emission needs no global offset and runs while the
    // predecessors finish (the look-back below then rarely waits).
    const bool in_lds = chunk_words <= (uint32_t)kLdsWords;
    if (in_lds) {
        for (uint32_t i = tid; i < chunk_words; i += 256) s_bits[i] = 0ull;
        __syncthreads();
        if (valid) {
            auto sink = [&](long long w, unsigned long long bits) { atomicOr(&s_bits[w], bits); };
            emit(sink);
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
            emit(sink);
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
    const bool coded = rd.peek() & 1ull;
    rd.skip(1);
    if (!coded) {
#pragma unroll
        for (int i = 0; i < S; ++i) out[i] = 0.0f;
    } else {
        const int emax = (int)(rd.peek() & 0xFFull) - 127;
        rd.skip(8);
        int prec = emax - minexp + 2 * (ND + 1);
        prec = prec > 32 ? 32 : prec;
        const int kmin = 32 - prec;
        unsigned long long m[32];
        int n = 0;
#pragma unroll
        for (int k = 31; k >= 0; --k) {
            unsigned long long mk = 0ull;
            if (k >= kmin) {
                if (n > 0) {
                    mk = rd.peek() & low_mask(n);
                    rd.skip(n);
                }
                while (n < S) {
                    const bool g = rd.peek() & 1ull;
                    rd.skip(1);
                    if (!g) break;
                    const int rem = S - n;
                    const unsigned long long win = rd.peek() & low_mask(rem);
                    if (win == 0ull) {
                        rd.skip(rem);
                        n = S;
                        break;
                    }
                    const int z = __ffsll((long long)win) - 1;
                    mk |= 1ull << (n + z);
                    rd.skip(z + 1);
                    n += z + 1;
                }
            }
            m[k] = mk;
        }
        uint32_t lo[32], hi[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            lo[k] = (uint32_t)m[k];
            hi[k] = (uint32_t)(m[k] >> 32);
        }
        transpose32(lo);
        if constexpr (ND == 3) transpose32(hi);
        int32_t q[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const uint32_t u = s < 32 ? lo[s] : hi[s - 32];
            const int dst = ND == 3 ? kPerm3.v[s] : kPerm2.v[s];
            q[dst] = (int32_t)((u ^ 0xAAAAAAAAu) - 0xAAAAAAAAu);
        }
        inv_transform<ND>(q);
#pragma unroll
        for (int i = 0; i < S; ++i) out[i] = (float)ldexp((double)q[i], emax - 30);   // one rounding
    }
    const int bx = (int)(b % A.nb[0]);
    const int by = (int)((b / A.nb[0]) % A.nb[1]);
    const int bz = (int)(b / ((long long)A.nb[0] * A.nb[1]));
    constexpr int KZ = ND == 3 ? 4 : 1;
    const int nzz = ND == 3 ? A.dims[2] : 1;
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
        const int z = 4 * bz + k;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int y = 4 * by + j;
            if (y >= A.dims[1] || z >= nzz) continue;
            const long long r0 = ((long long)z * A.dims[1] + y) * A.pitch;
            float *row = A.field + r0;
            if (VEC) {
                float4 o = make_float4(out[16 * k + 4 * j + 0], out[16 * k + 4 * j + 1], out[16 * k + 4 * j + 2],
                                       out[16 * k + 4 * j + 3]);
                if (A.sub) {
                    const float4 b = *reinterpret_cast<const float4 *>(A.sub + r0 + 4 * bx);
                    o = make_float4(b.x - o.x, b.y - o.y, b.z - o.z, b.w - o.w);
                }
                // streamed out: the next kernel reads it once, so it need not stay in the
                // caches (and its write-back is paid here, not during that kernel)
                typedef float f4v __attribute__((ext_vector_type(4)));
                const f4v t = {o.x, o.y, o.z, o.w};
                __builtin_nontemporal_store(t, reinterpret_cast<f4v *>(row + 4 * bx));
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * bx + i < A.dims[0]) {
                        const float o = out[16 * k + 4 * j + i];
                        row[4 * bx + i] = A.sub ? A.sub[r0 + 4 * bx + i] - o : o;
                    }
            }
        }
    }
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
