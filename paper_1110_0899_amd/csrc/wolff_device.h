// Device-side building blocks of the gfx950 Wolff kernels: the counter-based
// random stream, lattice geometry and the claim-and-flip of a site.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wolff.h"

namespace wolff {

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// words 0 and 2 by the two round multipliers (one 32x32->64 product each,
// a single v_mad_u64_u32 on CDNA) and mixes the high halves into words 1
// and 3 with the round key; the key advances by the Weyl increments after
// every round.  The key is uniform per replica, so k0/k1 and their bumps
// stay in scalar registers.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// K blocks that share words 1..3 and the key (the bond blocks a site needs),
// with their rounds interleaved so that the K dependent chains overlap.
template <int K>
__device__ __forceinline__ void philox_multi(const uint32_t (&c0)[K], uint32_t c1, uint32_t c2,
                                             uint32_t c3, uint32_t k0, uint32_t k1, U4 (&out)[K])
{
    uint32_t x0[K], x1[K], x2[K], x3[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        x0[i] = c0[i];
        x1[i] = c1;
        x2[i] = c2;
        x3[i] = c3;
    }
#pragma unroll
    for (int r = 0; r < 10; ++r) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const uint64_t p0 = (uint64_t)0xD2511F53u * x0[i];
            const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2[i];
            const uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1[i] ^ k0;
            const uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3[i] ^ k1;
            x1[i] = (uint32_t)p1;
            x3[i] = (uint32_t)p0;
            x0[i] = n0;
            x2[i] = n2;
        }
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) out[i] = U4{x0[i], x1[i], x2[i], x3[i]};
}

// Random stream domains (word 3 of the counter).
constexpr uint32_t DOMAIN_BOND = 0u;
constexpr uint32_t DOMAIN_SEED = 1u;
constexpr uint32_t DOMAIN_INIT = 2u;
constexpr uint32_t DOMAIN_COLOUR = 3u;   // q-state Potts: the cluster's new colour

// Seed site of update t: the 64-bit draw (x1:x0) scaled onto [0, N) by a
// multiply-high, exactly uniform for N a power of two.
__device__ __forceinline__ uint32_t seed_site(uint32_t k0, uint32_t k1, uint32_t t, uint32_t N)
{
    const U4 x = philox(0u, t, 0u, DOMAIN_SEED, k0, k1);
    const uint64_t u = ((uint64_t)x.y << 32) | x.x;
    return (uint32_t)__umul64hi(u, (uint64_t)N);
}

// q-state Potts (q >= 2): the colour that the cluster of update t, seed
// colour s0, takes: uniform over the q - 1 others,
// s0 + 1 + floor(x0 (q - 1) / 2^32) mod q with x = philox((0, t, 0, 3)).
__device__ __forceinline__ uint32_t potts_new_colour(uint32_t k0, uint32_t k1, uint32_t t,
                                                     uint32_t q, uint32_t s0)
{
    const U4 x = philox(0u, t, 0u, DOMAIN_COLOUR, k0, k1);
    const uint32_t c = s0 + 1u + __umulhi(x.x, q - 1u);
    return c >= q ? c - q : c;
}

// ---------------------------------------------------------------- geometry
// Exact division of a 32-bit numerator by a constant d >= 1: a shift when d
// is a power of two, otherwise the multiply-high by M = floor(2^64 / d) + 1
// (exact for every numerator < 2^32 because d < 2^32).
struct Div {
    uint32_t shift;     // log2(d) if d is a power of two, else 0xFFFFFFFF
    uint32_t magic_hi;  // M >> 32
    uint32_t magic_lo;  // M & 0xFFFFFFFF

    __device__ __forceinline__ uint32_t div(uint32_t j) const
    {
        if (shift != 0xFFFFFFFFu) return j >> shift;
        const uint64_t a = (uint64_t)j * magic_hi + (((uint64_t)j * magic_lo) >> 32);
        return (uint32_t)(a >> 32);
    }
};

// Periodic L^d lattice.  Sites are *named* by the logical index
// j = x + L*y (+ L*L*z) everywhere the method needs a name (the frontier
// queues, the random-stream counters, the records); spins are *stored*
// either in that order or, when L is a multiple of 16, in tiles of 128
// sites (16 x 8 in 2D, 16 x 4 x 2 in 3D) that each fill one 128-byte L2
// line, so that a site and most of its neighbours share a line:
//   2D: addr = ((y>>3)*ntx + (x>>4))*128 + (y&7)*16 + (x&15)
//   3D: addr = (((z>>1)*nty + (y>>2))*ntx + (x>>4))*128 + (z&1)*64 + (y&3)*16 + (x&15)
// with ntx = L/16 tiles along x and nty = L/TY tiles along y.
struct Geo {
    uint32_t L;
    uint32_t N;
    uint32_t LL;        // L*L (3D); equals N in 2D
    uint32_t tiled;     // 1: tiled storage
    uint32_t ntx;       // tiles along x (tiled storage)
    uint32_t nty;       // tiles along y (tiled storage)
    uint32_t ntz;       // tiles along z (tiled storage, 3D)
    uint32_t pad;
    Div dL;             // division by L
    Div dntx;           // division by ntx
    Div dnty;           // division by nty

    __device__ __forceinline__ uint32_t div_L(uint32_t j) const { return dL.div(j); }

    template <int DIM>
    __device__ __forceinline__ uint32_t tile_addr(uint32_t x, uint32_t y, uint32_t z) const
    {
        if (DIM == 2)
            return ((((y >> 3) * ntx + (x >> 4)) << 7) | ((y & 7u) << 4) | (x & 15u));
        return (((((z >> 1) * nty + (y >> 2)) * ntx + (x >> 4)) << 7) | ((z & 1u) << 6) |
                ((y & 3u) << 4) | (x & 15u));
    }
};

// Storage address of site j.
template <int DIM>
__device__ __forceinline__ uint32_t site_addr(const Geo& g, uint32_t j)
{
    if (!g.tiled) return j;
    const uint32_t q = g.div_L(j);
    const uint32_t x = j - q * g.L;
    if (DIM == 2) return g.tile_addr<2>(x, q, 0u);
    const uint32_t r = g.div_L(q);
    return g.tile_addr<3>(x, q - r * g.L, r);
}

// Storage address of site j and its sublattice parity (x + y (+ z)) mod 2.
template <int DIM>
__device__ __forceinline__ uint32_t site_addr_parity(const Geo& g, uint32_t j, uint32_t& par)
{
    const uint32_t q = g.div_L(j);
    const uint32_t x = j - q * g.L;
    if (DIM == 2) {
        par = (x + q) & 1u;
        return g.tiled ? g.tile_addr<2>(x, q, 0u) : j;
    }
    const uint32_t r = g.div_L(q);
    const uint32_t y = q - r * g.L;
    par = (x + y + r) & 1u;
    return g.tiled ? g.tile_addr<3>(x, y, r) : j;
}

// Neighbours of j in slot order (+x, -x, +y, -y[, +z, -z]): logical indices
// nb[] and storage addresses sa[]; also the storage address of j itself and
// its sublattice parity (x + y (+ z)) mod 2.
template <int DIM>
__device__ __forceinline__ void neighbours(const Geo& g, uint32_t j, uint32_t nb[2 * DIM],
                                           uint32_t sa[2 * DIM], uint32_t& self, uint32_t& par)
{
    const uint32_t L = g.L;
    const uint32_t q = g.div_L(j);
    const uint32_t x = j - q * L;
    const uint32_t xp = (x + 1u == L) ? 0u : x + 1u;
    const uint32_t xm = (x == 0u) ? L - 1u : x - 1u;
    nb[0] = j - x + xp;
    nb[1] = j - x + xm;
    if (DIM == 2) {
        const uint32_t N = g.N;
        const uint32_t y = q;
        nb[2] = (j >= N - L) ? j - (N - L) : j + L;
        nb[3] = (j >= L) ? j - L : j + (N - L);
        par = (x + y) & 1u;
        if (g.tiled) {
            const uint32_t yp = (y + 1u == L) ? 0u : y + 1u;
            const uint32_t ym = (y == 0u) ? L - 1u : y - 1u;
            self = g.tile_addr<2>(x, y, 0u);
            sa[0] = g.tile_addr<2>(xp, y, 0u);
            sa[1] = g.tile_addr<2>(xm, y, 0u);
            sa[2] = g.tile_addr<2>(x, yp, 0u);
            sa[3] = g.tile_addr<2>(x, ym, 0u);
        } else {
            self = j;
#pragma unroll
            for (int m = 0; m < 4; ++m) sa[m] = nb[m];
        }
    } else {
        const uint32_t r = g.div_L(q);
        const uint32_t y = q - r * L;
        const uint32_t z = r;
        const uint32_t LL = g.LL, N = g.N;
        nb[2] = (y + 1u == L) ? j + L - LL : j + L;
        nb[3] = (y == 0u) ? j + LL - L : j - L;
        nb[4] = (j >= N - LL) ? j - (N - LL) : j + LL;
        nb[5] = (j >= LL) ? j - LL : j + (N - LL);
        par = (x + y + z) & 1u;
        if (g.tiled) {
            const uint32_t yp = (y + 1u == L) ? 0u : y + 1u;
            const uint32_t ym = (y == 0u) ? L - 1u : y - 1u;
            const uint32_t zp = (z + 1u == L) ? 0u : z + 1u;
            const uint32_t zm = (z == 0u) ? L - 1u : z - 1u;
            self = g.tile_addr<3>(x, y, z);
            sa[0] = g.tile_addr<3>(xp, y, z);
            sa[1] = g.tile_addr<3>(xm, y, z);
            sa[2] = g.tile_addr<3>(x, yp, z);
            sa[3] = g.tile_addr<3>(x, ym, z);
            sa[4] = g.tile_addr<3>(x, y, zp);
            sa[5] = g.tile_addr<3>(x, y, zm);
        } else {
            self = j;
#pragma unroll
            for (int m = 0; m < 6; ++m) sa[m] = nb[m];
        }
    }
}

template <int DIM>
__device__ __forceinline__ void neighbours(const Geo& g, uint32_t j, uint32_t nb[2 * DIM],
                                           uint32_t sa[2 * DIM])
{
    uint32_t self, par;
    neighbours<DIM>(g, j, nb, sa, self, par);
}

// ------------------------------------------------------------ claim + flip
// Spins are int8 (+1 = 0x01, -1 = 0xFF).  Claiming site k for a cluster of
// spin s0 flips its byte to -s0 with one 32-bit atomic on the aligned word:
//   s0 = +1: OR  0xFE into the byte (0x01 -> 0xFF, 0xFF stays 0xFF)
//   s0 = -1: AND 0x01 into the byte (0xFF -> 0x01, 0x01 stays 0x01)
// The operation is idempotent, so exactly one caller sees the old byte equal
// to s0: that caller owns k.  A flipped member reads -s0 and is never
// eligible again, which makes the spin itself the visit mark of the update:
// no separate mark array, nothing to clear between updates.
template <int SCOPE>
__device__ __forceinline__ bool claim(int8_t* S, uint32_t k, int s0)
{
    uint32_t* w = reinterpret_cast<uint32_t*>(S) + (k >> 2);
    const uint32_t sh = (k & 3u) * 8u;
    if (s0 > 0) {
        const uint32_t m = 0xFEu << sh;
        const uint32_t old = __hip_atomic_fetch_or(w, m, __ATOMIC_RELAXED, SCOPE);
        return ((old >> sh) & 0xFFu) == 0x01u;
    } else {
        const uint32_t m = ~(0xFEu << sh);
        const uint32_t old = __hip_atomic_fetch_and(w, m, __ATOMIC_RELAXED, SCOPE);
        return ((old >> sh) & 0xFFu) == 0xFFu;
    }
}

// Potts claim of byte k (colour s0 -> c, c != s0) for several workgroups:
// a compare-and-swap of the aligned word, retried while only other bytes of
// the word change; exactly one caller finds the byte equal to s0.  Each byte
// of a word changes at most once per update, so the loop ends after at most
// four attempts.
template <int SCOPE>
__device__ __forceinline__ bool claim_colour(int8_t* S, uint32_t k, uint32_t s0, uint32_t c)
{
    uint32_t* w = reinterpret_cast<uint32_t*>(S) + (k >> 2);
    const uint32_t sh = (k & 3u) * 8u;
    uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, SCOPE);
    for (int attempt = 0; attempt < 8; ++attempt) {
        if (((old >> sh) & 0xFFu) != s0) return false;
        const uint32_t nw = (old & ~(0xFFu << sh)) | (c << sh);
        uint32_t expected = old;
        if (__hip_atomic_compare_exchange_strong(w, &expected, nw, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, SCOPE))
            return true;
        old = expected;
    }
    return false;   // unreachable (at most four changes of the word per update)
}

// ------------------------------------------------------------ member tags
// The one-workgroup path can instead tag the members of the current cluster,
// which is what lets it update the bond sum from the cluster alone.  A plain
// spin has bit 0 set (+1 = 0x01, -1 = 0xFF); a tagged byte has bit 0 clear:
//   bits 7..3  epoch: the update index mod 32
//   bit 2      1 once the member has been expanded
//   bit 1      the sign, as in a plain spin (set exactly for -1)
// Bit 1 is the sign of every byte, so the popcount reductions and the host
// copies read tagged bytes unchanged.  A tag of another epoch is read as the
// plain spin it carries, so tags need no clearing after an update; the
// lattice is normalised before an epoch could come round again.
constexpr uint32_t TAG_EPOCHS = 32u;
constexpr uint32_t NO_TAG = 0x100u;      // tag key that no byte matches

__device__ __forceinline__ uint32_t tag_key(uint32_t t) { return (t & (TAG_EPOCHS - 1u)) << 3; }

// member of the current cluster (either state) / expanded member
__device__ __forceinline__ bool is_member(uint32_t b, uint32_t key) { return (b & 0xF9u) == key; }
__device__ __forceinline__ bool is_expanded(uint32_t b, uint32_t key) { return (b & 0xFDu) == (key | 4u); }

// Byte of a site claimed for a cluster of spin s0 (its new spin is -s0):
// tagged with `key`, or the plain spin when key == NO_TAG.
__device__ __forceinline__ int8_t claimed_byte(int s0, uint32_t key)
{
    if (key == NO_TAG) return (int8_t)(s0 > 0 ? -1 : 1);
    return (int8_t)(key | (s0 > 0 ? 2u : 0u));
}

__device__ __forceinline__ int8_t expanded_byte(int s0, uint32_t key)
{
    return (int8_t)(key | 4u | (s0 > 0 ? 2u : 0u));
}

// ------------------------------------------------------- global pointers
// A pointer read from memory (a lattice descriptor field) is generic to the
// compiler, and a generic access is a FLAT instruction, which counts against
// both the vector-memory and the LDS wait counters: every LDS wait after it
// would also wait for the global access.  Accesses through these typed
// pointers are global instructions and leave the LDS counter alone.
typedef __attribute__((address_space(1))) int8_t gbyte;
typedef __attribute__((address_space(1))) uint32_t gword;

__device__ __forceinline__ gbyte* as_global(int8_t* p) { return (gbyte*)p; }
__device__ __forceinline__ gword* as_global(uint32_t* p) { return (gword*)p; }

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask)
{
    // number of set bits of `mask` below this lane (v_mbcnt_lo / v_mbcnt_hi)
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------- counting build
// Built with -DWOLFF_STATS=1 the kernels count what they do per lattice
// (the WOLFF_STAT_* counters of the public header): sites expanded, steps,
// neighbour reads, Philox blocks, claims, and the bytes of every global
// memory access they issue (reads, writes, atomics).  Each thread keeps its
// own counts; flush() sums them over each wave and adds them to the
// lattice's counter array with one atomic per wave and counter.  In the
// normal build the counts compile to nothing.
#ifndef WOLFF_STATS
#define WOLFF_STATS 0
#endif

struct StatAcc {
#if WOLFF_STATS
    unsigned long long c[WOLFF_STAT_COUNT] = {};
#endif
    __device__ __forceinline__ void add(int i, unsigned long long x)
    {
#if WOLFF_STATS
        c[i] += x;
#else
        (void)i;
        (void)x;
#endif
    }
    __device__ __forceinline__ void flush(unsigned long long* dst)
    {
#if WOLFF_STATS
        if (dst == nullptr) return;
#pragma unroll
        for (int i = 0; i < WOLFF_STAT_COUNT; ++i) {
            unsigned long long v = c[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if ((threadIdx.x & 63u) == 0u && v != 0ull) atomicAdd(&dst[i], v);
            c[i] = 0ull;
        }
#else
        (void)dst;
#endif
    }
};

}  // namespace wolff
