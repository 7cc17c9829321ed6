// Device building blocks of the ZFP-kind fixed-accuracy codec, shared by the codec's
// own kernels and the batched solver (one definition, so every stream and every decoded
// value is the same whichever kernel produced it).  The method and the stream layout
// are described in wv_codec.hip and wv.h.
#pragma once

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

// Inclusive scan of v over a 256-lane workgroup: shuffles inside each wave, then one
// exchange of the four wave totals through s_w[0..3].  Returns the lane's inclusive sum
// and sets total to the workgroup's sum.  Every lane calls it; it holds one barrier, and
// s_w may be written again only after another barrier of the caller.
template <typename T>
__device__ __forceinline__ T wg_scan256(T v, T *s_w, T &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    const T w0 = s_w[0], w1 = s_w[1], w2 = s_w[2], w3 = s_w[3];
    total = w0 + w1 + w2 + w3;
    return x + (wave > 0 ? w0 : T(0)) + (wave > 1 ? w1 : T(0)) + (wave > 2 ? w2 : T(0));
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


// One block of the fixed-accuracy code, one lane per block: exponent, block-floating-
// point integers, forward transform, sequency order, negabinary, and the bit planes
// m_lo[k] / m_hi[k] (bit k of coefficients 0..31 / 32..63).  The planes are the
// caller's own local arrays (a plain array stays in registers under the planes loops'
// wave-uniform indexing; inside a struct it would be placed in scratch).  prepare() is
// called by all lanes of a wave together (waves whose blocks are all uncoded skip the
// transform and the plane transposes; the planes loops run down to the wave's lowest
// kmin).
template <int ND>
struct BlockEnc {
    static constexpr int S = ND == 3 ? 64 : 16;
    bool valid = false, finite = true, coded = false;
    int emax = -126, kmin = 32, kmin_w = 32;

    __device__ __forceinline__ void prepare(const float *v, bool valid_, int minexp, uint32_t (&m_lo)[32],
                                            uint32_t (&m_hi)[32])
    {
        valid = valid_;
        bool nonzero = false;
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
        int prec = emax - minexp + 2 * (ND + 1);
        prec = prec > 32 ? 32 : prec;
        coded = valid && finite && nonzero && prec > 0;
        kmin = 32 - prec;
#pragma unroll
        for (int k = 0; k < 32; ++k) m_lo[k] = m_hi[k] = 0u;
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
            if constexpr (ND == 3) {
                // Two transposes of half-words: the upper halves of coefficients s and
                // 32+s packed into one word (low and high 16 bits) transpose into planes
                // 16..31, the lower halves into planes 0..15.  A wave none of whose blocks
                // codes a plane below 16 (kmin >= 16) needs only the first.
#pragma unroll
                for (int s = 0; s < 32; ++s) {
                    const uint32_t a = m_lo[s], b = m_hi[s];
                    m_lo[s] = (a >> 16) | (b & 0xFFFF0000u);
                    m_hi[s] = (a & 0xFFFFu) | (b << 16);
                }
                transpose32(m_lo);   // word k < 16: plane k+16 of 0..31; k >= 16: plane k of 32..63
                if (__ballot(coded && kmin < 16) != 0ull) transpose32(m_hi);   // planes 0..15 likewise
                else {
#pragma unroll
                    for (int k = 0; k < 32; ++k) m_hi[k] = 0u;
                }
                uint32_t U[32], L[32];
#pragma unroll
                for (int k = 0; k < 32; ++k) {
                    U[k] = m_lo[k];
                    L[k] = m_hi[k];
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    m_lo[k] = L[k];
                    m_lo[k + 16] = U[k];
                    m_hi[k] = L[k + 16];
                    m_hi[k + 16] = U[k + 16];
                }
            } else {
                transpose32(m_lo);
            }
        }
        // Planes run from 31 down to the lowest kmin of the wave in a plain (rolled)
        // loop: the plane index is wave-uniform, so m_lo[k] / m_hi[k] stay in registers
        // (indexed moves), and each lane skips the planes below its own kmin.
        kmin_w = coded ? kmin : 32;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) kmin_w = min(kmin_w, __shfl_xor(kmin_w, o));
        kmin_w = __builtin_amdgcn_readfirstlane(kmin_w);
    }

    // closed-form bit count of the block (0 for a lane without a block)
    __device__ __forceinline__ unsigned count(const uint32_t (&m_lo)[32], const uint32_t (&m_hi)[32]) const
    {
        unsigned nbits = valid ? 1u : 0u;
        if (coded) nbits += 8;
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
        return nbits;
    }

    // the block's bits at bit position pos of the sink's word space
    template <typename Sink>
    __device__ __forceinline__ void emit(long long pos, Sink &sink, const uint32_t (&m_lo)[32],
                                         const uint32_t (&m_hi)[32]) const
    {
        Emitter em{pos, 0ull};
        em.put(coded ? 1ull : 0ull, 1, sink);
        if (coded) em.put((unsigned long long)(emax + 127), 8, sink);
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
        em.flush(sink);
    }
};

// Decode one block from rd (positioned at its first bit) into out[S] (C order of the
// block, axis 0 fastest).
template <int ND>
__device__ __forceinline__ void decode_block(BitReader &rd, int minexp, float *out)
{
    constexpr int S = ND == 3 ? 64 : 16;
    const bool coded = rd.peek() & 1ull;
    rd.skip(1);
    if (!coded) {
#pragma unroll
        for (int i = 0; i < S; ++i) out[i] = 0.0f;
        return;
    }
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

// Write decoded block b (values out, C order) into field, or sub - decoded when sub is
// set; only the grid's own points are written, streamed out past the caches with VEC.
template <int ND, bool VEC>
__device__ __forceinline__ void store_block(float *field, const float *sub, const int *dims, int pitch,
                                            const int *nb, long long b, const float *out)
{
    const int bx = (int)(b % nb[0]);
    const int by = (int)((b / nb[0]) % nb[1]);
    const int bz = (int)(b / ((long long)nb[0] * nb[1]));
    constexpr int KZ = ND == 3 ? 4 : 1;
    const int nzz = ND == 3 ? dims[2] : 1;
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
        const int z = 4 * bz + k;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int y = 4 * by + j;
            if (y >= dims[1] || z >= nzz) continue;
            const long long r0 = ((long long)z * dims[1] + y) * pitch;
            float *row = field + r0;
            if (VEC) {
                float4 o = make_float4(out[16 * k + 4 * j + 0], out[16 * k + 4 * j + 1], out[16 * k + 4 * j + 2],
                                       out[16 * k + 4 * j + 3]);
                if (sub) {
                    const float4 t = *reinterpret_cast<const float4 *>(sub + r0 + 4 * bx);
                    o = make_float4(t.x - o.x, t.y - o.y, t.z - o.z, t.w - o.w);
                }
                // streamed out: the next kernel reads it once, so it need not stay in the
                // caches (and its write-back is paid here, not during that kernel)
                typedef float f4v __attribute__((ext_vector_type(4)));
                const f4v t = {o.x, o.y, o.z, o.w};
                __builtin_nontemporal_store(t, reinterpret_cast<f4v *>(row + 4 * bx));
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * bx + i < dims[0]) {
                        const float o = out[16 * k + 4 * j + i];
                        row[4 * bx + i] = sub ? sub[r0 + 4 * bx + i] - o : o;
                    }
            }
        }
    }
}

constexpr int kLdsWords = 2048;      // chunk bitstreams up to 16 KB are assembled in LDS
constexpr int kDecLdsWords = 2048;   // and chunks up to 16 KB are staged in LDS for decoding

}  // namespace

}  // namespace wv
