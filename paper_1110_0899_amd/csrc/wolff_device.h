// Device-side building blocks of the gfx950 Wolff kernels: the counter-based
// random stream, lattice geometry and the claim-and-flip of a site.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Random stream domains (word 3 of the counter).
constexpr uint32_t DOMAIN_BOND = 0u;
constexpr uint32_t DOMAIN_SEED = 1u;
constexpr uint32_t DOMAIN_INIT = 2u;

// Seed site of update t: the 64-bit draw (x1:x0) scaled onto [0, N) by a
// multiply-high, exactly uniform for N a power of two.
__device__ __forceinline__ uint32_t seed_site(uint32_t k0, uint32_t k1, uint32_t t, uint32_t N)
{
    const U4 x = philox(0u, t, 0u, DOMAIN_SEED, k0, k1);
    const uint64_t u = ((uint64_t)x.y << 32) | x.x;
    return (uint32_t)__umul64hi(u, (uint64_t)N);
}

// ---------------------------------------------------------------- geometry
// Periodic L^d lattice, site j = x + L*y (+ L*L*z), N < 2^32.
// Division by L uses a shift when L is a power of two and otherwise the
// multiply-high by M = floor(2^64 / L) + 1, exact for every j < 2^32.
struct Geo {
    uint32_t L;
    uint32_t N;
    uint32_t LL;        // L*L (3D); equals N in 2D
    uint32_t shift;     // log2(L) if L is a power of two, else 0xFFFFFFFF
    uint32_t magic_hi;  // M >> 32
    uint32_t magic_lo;  // M & 0xFFFFFFFF

    __device__ __forceinline__ uint32_t div_L(uint32_t j) const
    {
        if (shift != 0xFFFFFFFFu) return j >> shift;
        const uint64_t a = (uint64_t)j * magic_hi + (((uint64_t)j * magic_lo) >> 32);
        return (uint32_t)(a >> 32);
    }
};

// Neighbours of j in slot order (+x, -x, +y, -y[, +z, -z]).
template <int DIM>
__device__ __forceinline__ void neighbours(const Geo& g, uint32_t j, uint32_t nb[2 * DIM])
{
    const uint32_t L = g.L;
    const uint32_t q = g.div_L(j);
    const uint32_t x = j - q * L;
    nb[0] = (x + 1u == L) ? j + 1u - L : j + 1u;
    nb[1] = (x == 0u) ? j + L - 1u : j - 1u;
    if (DIM == 2) {
        const uint32_t N = g.N;
        nb[2] = (j >= N - L) ? j - (N - L) : j + L;
        nb[3] = (j >= L) ? j - L : j + (N - L);
    } else {
        const uint32_t r = g.div_L(q);
        const uint32_t y = q - r * L;
        const uint32_t LL = g.LL, N = g.N;
        nb[2] = (y + 1u == L) ? j + L - LL : j + L;
        nb[3] = (y == 0u) ? j + LL - L : j - L;
        nb[4] = (j >= N - LL) ? j - (N - LL) : j + LL;
        nb[5] = (j >= LL) ? j - LL : j + (N - LL);
    }
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
        const uint32_t old = __hip_atomic_fetch_or(w, 0xFEu << sh, __ATOMIC_RELAXED, SCOPE);
        return ((old >> sh) & 0xFFu) == 0x01u;
    } else {
        const uint32_t old = __hip_atomic_fetch_and(w, ~(0xFEu << sh), __ATOMIC_RELAXED, SCOPE);
        return ((old >> sh) & 0xFFu) == 0xFFu;
    }
}

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

}  // namespace wolff
