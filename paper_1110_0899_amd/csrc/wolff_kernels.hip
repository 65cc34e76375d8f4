// gfx950 kernels of the Wolff single-cluster update (Komura & Okabe,
// arXiv:1110.0899, Sections 2 and 4): frontier-parallel growth of one
// cluster per update, claim-and-flip, per-update records, and the lattice
// reductions for the energy (Section 5, "+ measurement").
#include "wolff_kernels.h"

namespace wolff {

constexpr int WAVE = 64;
// Error bits of Rep::err.
constexpr uint32_t ERR_MAG = 1u;          // magnetisation recount != tracked value
constexpr uint32_t ERR_TEAM_WAIT = 2u;    // a team wait passed its bound
constexpr uint32_t ERR_BOND = 4u;         // bond-sum recount != tracked value
// Bound on the polls of one team wait (each poll is at least ~100 ns, so the
// bound is seconds, far above any legitimate wait).
constexpr uint32_t TEAM_SPIN_LIMIT = 1u << 26;
constexpr int SCOPE_AGENT = __HIP_MEMORY_SCOPE_AGENT;

// --------------------------------------------------------------- expansion
// Step (iii') of Section 4 for one frontier site j (already in the cluster
// and flipped): look at the 2*DIM neighbours, test the bond to each one that
// still holds s0, and claim the neighbours whose bond is active.
//   +mu neighbour: bond (j, mu)          -> word mu of philox((j, t, s, 0))
//   -mu neighbour: bond (j - e_mu, mu)   -> word mu of philox((j - e_mu, t, s, 0))
// One Philox block serves all +mu bonds of j.  The cluster does not depend
// on which thread claims a site first, so no ordering between threads is
// needed.  Both paths draw every bond word of j while the neighbour loads
// are in flight: more arithmetic than drawing for eligible neighbours only,
// but a shorter step, and the step's latency bounds the growth.

// Random words of the bonds of j: the +mu bonds from one block keyed by j,
// each -mu bond from the block keyed by its base site j - e_mu.
template <int DIM>
__device__ __forceinline__ void bond_words(uint32_t j, const uint32_t nb[2 * DIM], uint32_t k0,
                                           uint32_t k1, uint32_t t, uint32_t s,
                                           uint32_t rp[3], uint32_t rm[3])
{
    const U4 r = philox(j, t, s, DOMAIN_BOND, k0, k1);
    rp[0] = r.x;
    rp[1] = r.y;
    rp[2] = r.z;
#pragma unroll
    for (int mu = 0; mu < DIM; ++mu) {
        const U4 q = philox(nb[2 * mu + 1], t, s, DOMAIN_BOND, k0, k1);
        rm[mu] = (mu == 0) ? q.x : (mu == 1) ? q.y : q.z;
    }
}

// Team path: spins are plain bytes and a claim is the atomic flip (Ising) or
// the colour compare-and-swap (Potts, pq > 0, new colour c).
template <int DIM, int SCOPE>
__device__ __forceinline__ void expand_site(bool active, uint32_t j, const Geo& g, int8_t* S,
                                            int s0, uint32_t thr, uint32_t k0, uint32_t k1,
                                            uint32_t t, uint32_t s, uint32_t nb[2 * DIM],
                                            bool won[2 * DIM], uint32_t& n_act, uint32_t pq = 0u,
                                            uint32_t c = 0u)
{
    if (!active) j = 0u;
    uint32_t sa[2 * DIM];
    neighbours<DIM>(g, j, nb, sa);
    int b[2 * DIM];
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m) b[m] = S[sa[m]];
    uint32_t rp[3], rm[3];
    bond_words<DIM>(j, nb, k0, k1, t, s, rp, rm);
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m) {
        const uint32_t r = (m & 1) ? rm[m / 2] : rp[m / 2];
        const bool act = active && b[m] == s0 && r < thr;
        n_act += act ? 1u : 0u;
        won[m] = act && (pq ? claim_colour<SCOPE>(S, sa[m], (uint32_t)s0, c) : claim<SCOPE>(S, sa[m], s0));
    }
}

// Claim table of the one-workgroup path.  Only one workgroup touches the
// lattice during a launch, so the only races on a site are between threads
// of the same step: they are settled in an LDS hash table keyed by storage
// address (CAS on an empty slot, linear probing), and the winner writes the
// claimed byte with a plain store, visible to the next step after the
// step's barrier.  A step inserts at most 2d keys per thread, fewer than the
// table's 8 slots per thread, so a probe always ends at the key or at an
// empty slot.  The workgroup empties the table after each step.
constexpr uint32_t TAB_EMPTY = 0xFFFFFFFFu;

// Table entries for a workgroup size: 8 per thread.
__host__ __device__ constexpr uint32_t tab_entries(int wg) { return 8u * (uint32_t)wg; }
__host__ __device__ constexpr uint32_t tab_shift(int wg)
{
    return wg == 64 ? 23u : wg == 128 ? 22u : wg == 256 ? 21u : wg == 512 ? 20u : 19u;
}

// won[m]: this thread won site a[m] for the step.  The first probes of all
// slots go out together (one LDS round trip); a slot whose first probe met
// another key keeps probing linearly.  Two slots of one thread holding the
// same site (L = 2) are settled in slot order: the second finds the first.
template <int WG, int DIM>
__device__ __forceinline__ void table_claims(uint32_t* tab, const uint32_t a[2 * DIM],
                                             const bool act[2 * DIM], bool won[2 * DIM])
{
    uint32_t h[2 * DIM], prev[2 * DIM];
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m) {
        h[m] = (a[m] * 0x9E3779B1u) >> tab_shift(WG);
        prev[m] = act[m] ? atomicCAS(&tab[h[m]], TAB_EMPTY, a[m]) : a[m];
    }
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m) {
        bool w = prev[m] == TAB_EMPTY;
        if (act[m] && prev[m] != TAB_EMPTY && prev[m] != a[m]) {
            uint32_t hh = h[m];
            for (uint32_t p = 1; p < tab_entries(WG); ++p) {   // ends early: the table is never full
                hh = (hh + 1u) & (tab_entries(WG) - 1u);
                const uint32_t pv = atomicCAS(&tab[hh], TAB_EMPTY, a[m]);
                if (pv == TAB_EMPTY) {
                    w = true;
                    break;
                }
                if (pv == a[m]) break;
            }
        }
        won[m] = w;
    }
}

// One-workgroup path.  `key` is the tag of the update (NO_TAG: plain bytes).
// Ising: members of the cluster hold -s0, so a neighbour is eligible exactly
// when its sign is s0.  A neighbour of sign -s0 is a member (original spin
// s0) or an anti-aligned non-member, counted in n_anti; members already
// expanded are counted in n_inner (see run_rep).  Potts: members hold the
// new colour, so a neighbour is eligible exactly when its colour is s0.
// A neighbour byte b is eligible when (b & emask) == evalue: the sign bit
// for Ising, the whole colour byte for Potts.  A claimed site gets byte cb.
template <int DIM, int WG>
__device__ __forceinline__ void expand_site_wg(bool active, uint32_t j, const uint32_t nb[2 * DIM],
                                               const uint32_t sa[2 * DIM], gbyte* S,
                                               uint32_t emask, uint32_t evalue, int8_t cb,
                                               uint32_t key, uint32_t thr, uint32_t k0,
                                               uint32_t k1, uint32_t t, uint32_t s,
                                               bool won[2 * DIM], uint32_t* tab,
                                               uint32_t& n_anti, uint32_t& n_inner,
                                               uint32_t& n_act, uint32_t no_inner = 0u)
{
    uint32_t b[2 * DIM];
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m) b[m] = (uint8_t)S[sa[m]];
    uint32_t rp[3], rm[3];
    bond_words<DIM>(j, nb, k0, k1, t, s, rp, rm);
    bool act[2 * DIM];
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m) {
        const bool same = (b[m] & emask) == evalue;
        const uint32_t r = (m & 1) ? rm[m / 2] : rp[m / 2];
        act[m] = active && same && r < thr;
        n_act += act[m] ? 1u : 0u;
        n_anti += (active && !same && !is_member(b[m], key)) ? 1u : 0u;
        n_inner += (active && is_expanded(b[m], key) && !((no_inner >> m) & 1u)) ? 1u : 0u;
    }
    table_claims<WG, DIM>(tab, sa, act, won);
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m)
        if (won[m]) S[sa[m]] = cb;
}

// Wave-level compaction of the claimed sites: one ballot per neighbour slot,
// the lane's offset from mbcnt.  Returns the wave's item count.
template <int DIM>
__device__ __forceinline__ uint32_t wave_compact(const bool won[2 * DIM], uint32_t pos[2 * DIM])
{
    uint32_t base = 0;
#pragma unroll
    for (int m = 0; m < 2 * DIM; ++m) {
        const uint64_t mask = __ballot(won[m]);
        pos[m] = base + lane_prefix(mask);
        base += (uint32_t)__popcll(mask);
    }
    return base;
}

// ------------------------------------------------------------- reductions
// B = sum_i sum_mu S_i S_{i+e_mu} and M = sum_i S_i.
//
// Vector form (L a multiple of 16): a chunk is 16 consecutive sites of one
// row, read as one 16-byte load.  With +1 = 0x01 and -1 = 0xFF, bit 1 of a
// byte is set exactly for -1, and bit 1 of (a ^ b) is set exactly when two
// spins differ, so per chunk
//   differing bonds = popcount(((a ^ shifted neighbour bytes) & 0x02020202))
//   negative spins  = popcount(a & 0x02020202)
// and over the lattice B = d N - 2 (differing bonds), M = N - 2 (negatives).
// The +x neighbours are the chunk shifted by one byte plus the first byte of
// the next chunk of the row (wrapping to the row start); +y / +z are the
// chunks one row / one plane further (periodic).
// Per-word counts of 4 spin bytes.  Ising (+1 = 0x01, -1 = 0xFF, tags keep
// the sign in bit 1): pair_count = bonds whose spins differ, self_count =
// spins equal to -1.  Potts (colour bytes): pair_count = bonds whose colours
// are equal, self_count = sites of colour 0; a zero byte of v is detected
// exactly by the high bit of ~(((v & 0x7F..) + 0x7F..) | v | 0x7F..).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t v)
{
    return __popc(~(((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v | 0x7F7F7F7Fu));
}

template <bool POTTS>
__device__ __forceinline__ uint32_t pair_count(uint32_t a, uint32_t b)
{
    return POTTS ? zero_bytes(a ^ b) : __popc((a ^ b) & 0x02020202u);
}

template <bool POTTS>
__device__ __forceinline__ uint32_t self_count(uint32_t a)
{
    return POTTS ? zero_bytes(a) : __popc(a & 0x02020202u);
}

template <bool POTTS>
__device__ __forceinline__ uint32_t pair_count1(uint32_t a, uint32_t b)
{
    return POTTS ? (uint32_t)(a == b) : ((a ^ b) >> 1) & 1u;
}

template <bool POTTS>
__device__ __forceinline__ uint32_t self_count1(uint32_t a)
{
    return POTTS ? (uint32_t)(a == 0u) : (a >> 1) & 1u;
}

template <int DIM, bool POTTS>
__device__ __forceinline__ void chunk_counts(const int8_t* S, const Geo& g, uint32_t c,
                                             uint32_t& ndiff, uint32_t& nneg)
{
    const uint4* S4 = reinterpret_cast<const uint4*>(S);
    const uint32_t* S1 = reinterpret_cast<const uint32_t*>(S);
    const uint32_t L = g.L, N = g.N, LL = g.LL;
    const uint32_t i = c * 16u;
    const uint32_t q = g.div_L(i);
    const uint32_t x0 = i - q * L;
    const uint4 a = S4[c];
    const uint32_t inext = (x0 + 16u == L) ? i + 16u - L : i + 16u;
    const uint32_t w4 = S1[inext >> 2];
    const uint32_t s0 = (a.x >> 8) | (a.y << 24);
    const uint32_t s1 = (a.y >> 8) | (a.z << 24);
    const uint32_t s2 = (a.z >> 8) | (a.w << 24);
    const uint32_t s3 = (a.w >> 8) | (w4 << 24);
    uint32_t d = pair_count<POTTS>(a.x, s0) + pair_count<POTTS>(a.y, s1) + pair_count<POTTS>(a.z, s2) +
                 pair_count<POTTS>(a.w, s3);
    uint32_t iy;
    if (DIM == 2) {
        iy = (i >= N - L) ? i - (N - L) : i + L;
    } else {
        const uint32_t y = q - g.div_L(q) * L;
        iy = (y + 1u == L) ? i + L - LL : i + L;
    }
    const uint4 b = S4[iy >> 4];
    d += pair_count<POTTS>(a.x, b.x) + pair_count<POTTS>(a.y, b.y) + pair_count<POTTS>(a.z, b.z) +
         pair_count<POTTS>(a.w, b.w);
    if (DIM == 3) {
        const uint32_t iz = (i >= N - LL) ? i - (N - LL) : i + LL;
        const uint4 z = S4[iz >> 4];
        d += pair_count<POTTS>(a.x, z.x) + pair_count<POTTS>(a.y, z.y) + pair_count<POTTS>(a.z, z.z) +
             pair_count<POTTS>(a.w, z.w);
    }
    ndiff = d;
    nneg = self_count<POTTS>(a.x) + self_count<POTTS>(a.y) + self_count<POTTS>(a.z) + self_count<POTTS>(a.w);
}

// Tiled storage: chunk c is row (c & 7) of tile c >> 3, 16 sites along x.
// The +x neighbours are the row shifted by one byte plus the first byte of
// the same row of the next tile along x; +y / +z neighbours are the next row
// of the tile or the matching row of the next tile (periodic).
template <int DIM, bool POTTS>
__device__ __forceinline__ void chunk_counts_tiled(const int8_t* S, const Geo& g, uint32_t c,
                                                   uint32_t& ndiff, uint32_t& nneg)
{
    const uint4* S4 = reinterpret_cast<const uint4*>(S);
    const uint32_t* S1 = reinterpret_cast<const uint32_t*>(S);
    const uint32_t T = c >> 3, row = c & 7u;
    const uint32_t q1 = g.dntx.div(T);
    const uint32_t tx = T - q1 * g.ntx;
    const uint32_t Tx = (tx + 1u == g.ntx) ? T - tx : T + 1u;
    const uint4 a = S4[c];
    const uint32_t w4 = S1[((Tx << 3) | row) << 2];
    const uint32_t s0 = (a.x >> 8) | (a.y << 24);
    const uint32_t s1 = (a.y >> 8) | (a.z << 24);
    const uint32_t s2 = (a.z >> 8) | (a.w << 24);
    const uint32_t s3 = (a.w >> 8) | (w4 << 24);
    uint32_t d = pair_count<POTTS>(a.x, s0) + pair_count<POTTS>(a.y, s1) + pair_count<POTTS>(a.z, s2) +
                 pair_count<POTTS>(a.w, s3);
    uint32_t cy;
    if (DIM == 2) {
        const uint32_t ty = q1;
        if (row < 7u) {
            cy = c + 1u;
        } else {
            const uint32_t Ty = (ty + 1u == g.nty) ? tx : T + g.ntx;
            cy = Ty << 3;
        }
    } else {
        const uint32_t q2 = g.dnty.div(q1);
        const uint32_t ty = q1 - q2 * g.nty;
        const uint32_t tz = q2;
        const uint32_t oy = row & 3u, oz = row >> 2;
        if (oy < 3u) {
            cy = c + 1u;
        } else {
            const uint32_t Ty = (ty + 1u == g.nty) ? T - ty * g.ntx : T + g.ntx;
            cy = (Ty << 3) | (oz << 2);
        }
        uint32_t cz;
        if (oz == 0u) {
            cz = c + 4u;
        } else {
            const uint32_t plane = g.ntx * g.nty;
            const uint32_t Tz = (tz + 1u == g.ntz) ? T - tz * plane : T + plane;
            cz = (Tz << 3) | oy;
        }
        const uint4 z = S4[cz];
        d += pair_count<POTTS>(a.x, z.x) + pair_count<POTTS>(a.y, z.y) + pair_count<POTTS>(a.z, z.z) +
             pair_count<POTTS>(a.w, z.w);
    }
    const uint4 b = S4[cy];
    d += pair_count<POTTS>(a.x, b.x) + pair_count<POTTS>(a.y, b.y) + pair_count<POTTS>(a.z, b.z) +
         pair_count<POTTS>(a.w, b.w);
    ndiff = d;
    nneg = self_count<POTTS>(a.x) + self_count<POTTS>(a.y) + self_count<POTTS>(a.z) + self_count<POTTS>(a.w);
}

// Scalar form for any L: per site, with coordinates advanced incrementally
// along the thread's stride (no division in the loop).  Accumulates the same
// two counts as the vector form.
template <int DIM, bool POTTS>
__device__ __forceinline__ void scalar_counts(const int8_t* S, const Geo& g, uint32_t first,
                                              uint32_t stride, uint32_t& ndiff, uint32_t& nneg)
{
    const uint32_t L = g.L, N = g.N, LL = g.LL;
    const uint32_t q0 = g.div_L(first);
    uint32_t x = first - q0 * L;
    uint32_t y = q0 - g.div_L(q0) * L;
    const uint32_t dq = g.div_L(stride);
    const uint32_t dx = stride - dq * L;
    const uint32_t dq_mod = dq - g.div_L(dq) * L;
    uint32_t d = 0u, neg = 0u;
    // Ising: only bit 1 (the sign) of a byte is read: bytes may carry member tags
    for (uint32_t i = first; i < N; i += stride) {
        const uint32_t si = (uint8_t)S[i];
        const uint32_t xp = (x + 1u == L) ? i + 1u - L : i + 1u;
        d += pair_count1<POTTS>((uint8_t)S[xp], si);
        if (DIM == 2) {
            const uint32_t yp = (i >= N - L) ? i - (N - L) : i + L;
            d += pair_count1<POTTS>((uint8_t)S[yp], si);
        } else {
            const uint32_t yp = (y + 1u == L) ? i + L - LL : i + L;
            const uint32_t zp = (i >= N - LL) ? i - (N - LL) : i + LL;
            d += pair_count1<POTTS>((uint8_t)S[yp], si) + pair_count1<POTTS>((uint8_t)S[zp], si);
        }
        neg += self_count1<POTTS>(si);
        x += dx;
        uint32_t carry = 0u;
        if (x >= L) {
            x -= L;
            carry = 1u;
        }
        if (DIM == 3) {
            y += dq_mod + carry;
            if (y >= L) y -= L;
        }
    }
    ndiff = d;
    nneg = neg;
}

// This thread's counts over its share of the lattice: items first, first +
// stride, ... (chunks when L % 16 == 0, sites otherwise).  UNROLL chunks are
// in flight per thread: 4 in the grid-wide kernel, 1 inside the growth
// kernel, where the registers of four chunks would halve the resident waves.
template <int DIM, int UNROLL, bool POTTS = false>
__device__ __forceinline__ void lattice_counts(const int8_t* S, const Geo& g, uint32_t first,
                                               uint32_t stride, uint64_t& ndiff, uint64_t& nneg)
{
    uint64_t d = 0u, neg = 0u;
    if (g.tiled) {
        const uint32_t nchunks = g.N >> 4;
        uint32_t c = first;
        if (UNROLL == 4) {
            for (; c + 3u * stride < nchunks; c += 4u * stride) {
                uint32_t d0, n0, d1, n1, d2, n2, d3, n3;
                chunk_counts_tiled<DIM, POTTS>(S, g, c, d0, n0);
                chunk_counts_tiled<DIM, POTTS>(S, g, c + stride, d1, n1);
                chunk_counts_tiled<DIM, POTTS>(S, g, c + 2u * stride, d2, n2);
                chunk_counts_tiled<DIM, POTTS>(S, g, c + 3u * stride, d3, n3);
                d += d0 + d1 + d2 + d3;
                neg += n0 + n1 + n2 + n3;
            }
        }
        for (; c < nchunks; c += stride) {
            uint32_t d0, n0;
            chunk_counts_tiled<DIM, POTTS>(S, g, c, d0, n0);
            d += d0;
            neg += n0;
        }
    } else if ((g.L & 15u) == 0u) {
        const uint32_t nchunks = g.N >> 4;
        uint32_t c = first;
        if (UNROLL == 4) {
            for (; c + 3u * stride < nchunks; c += 4u * stride) {
                uint32_t d0, n0, d1, n1, d2, n2, d3, n3;
                chunk_counts<DIM, POTTS>(S, g, c, d0, n0);
                chunk_counts<DIM, POTTS>(S, g, c + stride, d1, n1);
                chunk_counts<DIM, POTTS>(S, g, c + 2u * stride, d2, n2);
                chunk_counts<DIM, POTTS>(S, g, c + 3u * stride, d3, n3);
                d += d0 + d1 + d2 + d3;
                neg += n0 + n1 + n2 + n3;
            }
        }
        for (; c < nchunks; c += stride) {
            uint32_t d0, n0;
            chunk_counts<DIM, POTTS>(S, g, c, d0, n0);
            d += d0;
            neg += n0;
        }
    } else {
        uint32_t d0 = 0u, n0 = 0u;
        if (first < g.N) scalar_counts<DIM, POTTS>(S, g, first, stride, d0, n0);
        d = d0;
        neg = n0;
    }
    ndiff = d;
    nneg = neg;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// (B, M) of one lattice by one workgroup; every thread receives the result.
// Potts (q > 0): B = q (equal bonds) - d N, M = q (colour-0 sites) - N.
template <int WG, int DIM>
__device__ __forceinline__ void reduce_lattice_wg(const int8_t* S, const Geo& g, long long* red,
                                  int64_t& Bout, int64_t& Mout, uint32_t q = 0u)
{
    constexpr int NW = WG / WAVE;
    const uint32_t tid = threadIdx.x;
    uint64_t d, neg;
    if (q)
        lattice_counts<DIM, 1, true>(S, g, tid, WG, d, neg);
    else
        lattice_counts<DIM, 1, false>(S, g, tid, WG, d, neg);
    d = wave_sum_u64(d);
    neg = wave_sum_u64(neg);
    const uint32_t wv = tid / WAVE;
    __syncthreads();
    if ((tid & (WAVE - 1)) == 0) {
        red[wv] = (long long)d;
        red[NW + wv] = (long long)neg;
    }
    __syncthreads();
    int64_t sd = 0, sn = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        sd += red[w];
        sn += red[NW + w];
    }
    if (q) {
        Bout = (int64_t)q * sd - (int64_t)DIM * (int64_t)g.N;
        Mout = (int64_t)q * sn - (int64_t)g.N;
    } else {
        Bout = (int64_t)DIM * (int64_t)g.N - 2 * sd;
        Mout = (int64_t)g.N - 2 * sn;
    }
    __syncthreads();
}

// A spin byte with its member tag removed: the plain +-1 that bit 1 holds.
__device__ __forceinline__ uint32_t plain_word(uint32_t w)
{
    const uint32_t neg = (w >> 1) & 0x01010101u;                  // 1 where the spin is -1
    return 0x01010101u | (neg * 0xFEu);
}

__device__ __forceinline__ int8_t plain_byte(int8_t b) { return (b & 2) ? (int8_t)-1 : (int8_t)1; }

// Remove the member tags from lattice bytes [0, N): whole words first, then
// the last N mod 4 bytes one by one (the lattice may be a caller's buffer of
// exactly N bytes).  Items first, first + stride, ...
__device__ __forceinline__ void clear_tags(int8_t* S, uint32_t N, uint32_t first, uint32_t stride)
{
    uint32_t* W = reinterpret_cast<uint32_t*>(S);
    const uint32_t nw = N >> 2;
    for (uint32_t i = first; i < nw; i += stride) {
        const uint32_t w = W[i];
        const uint32_t clean = plain_word(w);
        if (clean != w) W[i] = clean;
    }
    const uint32_t k = 4u * nw + first;
    if (first < 4u && k < N) {
        const int8_t b = S[k];
        const int8_t clean = plain_byte(b);
        if (clean != b) S[k] = clean;
    }
}

// Remove the member tags from a whole lattice, by one workgroup.
template <int WG>
__device__ __forceinline__ void clear_tags_wg(int8_t* S, uint32_t N)
{
    clear_tags(S, N, threadIdx.x, WG);
    __syncthreads();
}

// ------------------------------------------------- one-workgroup growth path
// All updates of one lattice in one workgroup.  The frontier is a ring of
// `qmask + 1` entries in LDS; when a step's new sites do not fit, they go to
// the lattice's global overflow stack and come back when the ring runs low.
// Items are appended in whole steps: ballot/mbcnt inside each wave, a prefix
// over the waves' counts in LDS, one store per new site.

// Neighbour slots of site j (+x, -x, +y, -y[, +z, -z] as bits 0..2d-1)
// whose bond crosses the periodic boundary, and the same for the +mu slots
// only (the bonds that site j is the base of).
template <int DIM>
__device__ __forceinline__ uint32_t wrap_slots(const Geo& g, uint32_t j)
{
    const uint32_t L = g.L;
    const uint32_t q = g.div_L(j);
    const uint32_t x = j - q * L;
    uint32_t m = (x + 1u == L ? 1u : 0u) | (x == 0u ? 2u : 0u);
    if (DIM == 2) {
        m |= (q + 1u == L ? 4u : 0u) | (q == 0u ? 8u : 0u);
    } else {
        const uint32_t z = g.div_L(q);
        const uint32_t y = q - z * L;
        m |= (y + 1u == L ? 4u : 0u) | (y == 0u ? 8u : 0u) | (z + 1u == L ? 16u : 0u) |
             (z == 0u ? 32u : 0u);
    }
    return m;
}

// Workgroup-shared control words of the one-workgroup path.
struct WgCtl {
    int s0;                 // seed spin (Ising) or colour (Potts) of the current update
    uint32_t stop;          // 1: the launch's time budget is spent
    uint32_t idx;           // next replica (work counter)
    int32_t cb;             // byte written to claimed sites
    uint64_t t_start;       // wall clock at the workgroup's start
    uint32_t faces;         // odd L: expanded members listed on a last face
};

// Time budget of a launch, checked by thread 0 only and broadcast through
// LDS so that every thread of the workgroup takes the same decision.
__device__ __forceinline__ uint32_t budget_spent(const WgCtl* c, uint64_t budget)
{
    return (budget != 0u && wall_clock64() - c->t_start >= budget) ? 1u : 0u;
}

// Stop request of a lattice: a flag in host memory mapped into the device's
// address space, set by the host while kernels run, read at system scope.
// The loads and stores below go through global-address-space pointers: a
// generic pointer would make them flat instructions, which every later LDS
// wait of the wave would also wait for.
typedef __attribute__((address_space(1))) const uint32_t gcword;
typedef __attribute__((address_space(1))) int64_t gi64;

// Record of one update at dst (three 8-byte global stores).
__device__ __forceinline__ void store_record(wolff_record* dst, int64_t bond_sum, int64_t mag,
                                             int64_t csize)
{
    gi64* p = (gi64*)dst;
    p[0] = bond_sum;
    p[1] = mag;
    p[2] = csize;
}

// The raw request word (0: none); the caller compares it only where it
// needs the answer, so that the host-memory read can stay in flight.
__device__ __forceinline__ uint32_t abort_word(const uint32_t* flag)
{
    return flag != nullptr ? __hip_atomic_load((gcword*)flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)
                           : 0u;
}

__device__ __forceinline__ uint32_t abort_requested(const uint32_t* flag)
{
    return abort_word(flag) != 0u ? 1u : 0u;
}

// Up to max_updates (0: all left) updates of replica R, stopping early at an
// update boundary once the launch's time budget is spent.  Per update: seed
// site and seed spin/colour (step (i)), growth steps until the ring and the
// overflow stack are empty (steps (ii)-(iv)), the flip done by the claims,
// M updated exactly, B updated from the cluster (even-L Ising with
// measurement) or recounted over the lattice, and one record (step (v)).
template <int WG, int DIM>
__device__ __forceinline__ void run_rep(Rep* R, uint32_t max_updates, uint64_t budget, uint32_t qmask,
                        uint32_t* q, uint32_t* wave_cnt, long long* red, WgCtl* ctl)
{
    constexpr int NW = WG / WAVE;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (WAVE - 1);
    const uint32_t wv = tid / WAVE;

    int8_t* S = R->S;
    gbyte* SG = as_global(S);
    gword* ov = as_global(R->ov);
    const Geo g = R->geo;
    const uint32_t thr = R->thr, k0 = R->k0, k1 = R->k1;
    const uint32_t t0 = R->t;
    uint32_t n = R->n_left;
    if (max_updates != 0u && max_updates < n) n = max_updates;
    wolff_record* rec = R->rec + R->rec_count;
    int64_t M = R->M, B = R->B;
    bool b_valid = R->b_valid != 0u;
    uint32_t t_norm = R->t_norm;
    const bool measure = R->measure != 0u;
    const uint32_t pq = R->q;                                     // 0: Ising, else Potts q
    // With measurement on an even-L (bipartite) Ising lattice the bond sum
    // follows the cluster; otherwise it is recounted over the lattice per update.
    const bool incr = measure && pq == 0u;
    // odd L: the lattice is not bipartite across the periodic boundary, so
    // a bond that wraps around is left out of the expansion-time count and
    // counted once the cluster is complete, from its member on the last face
    const bool odd = (g.L & 1u) != 0u;
    uint32_t err = 0u;
    const uint32_t QC = qmask + 1u;
    uint32_t* tab = q + QC;                                       // claim table after the ring
    StatAcc st;                                                   // counting build only
    // bytes one recount of the lattice reads (chunks of 16 sites with their
    // +x word and +y (+z) chunks, or per site with its +mu neighbours)
    const uint64_t recount_bytes = (g.tiled || (g.L & 15u) == 0u)
                                       ? (uint64_t)(g.N / 16u) * (DIM == 2 ? 36u : 52u)
                                       : (uint64_t)g.N * (1u + DIM);

    // a stop request seen before the first update: run none (the state
    // stays exact; the request is polled again after every update)
    const uint32_t* abort_flag = R->abort;
    if (abort_flag != nullptr) {
        if (tid == 0) ctl->stop = abort_requested(abort_flag);
        __syncthreads();
        if (ctl->stop) n = 0u;
        __syncthreads();
    }

    uint32_t done = 0u;
    while (done < n) {
        const uint32_t u = done;
        const uint32_t t = t0 + u;
        if (incr && (!b_valid || t - t_norm >= TAG_EPOCHS)) {
            // recount (B, M), check them against the tracked values, and
            // normalise the lattice so that no byte carries this epoch's tag
            int64_t Bm, Mm;
            reduce_lattice_wg<WG, DIM>(S, g, red, Bm, Mm);
            if (Mm != M) err |= ERR_MAG;
            if (b_valid && Bm != B) err |= ERR_BOND;
            B = Bm;
            b_valid = true;
            clear_tags_wg<WG>(S, g.N);
            // the normalisation pass reads every byte and rewrites the words with tags (bounded by N)
            if (tid == 0) st.add(WOLFF_STAT_READ_BYTES, recount_bytes + g.N);
            if (tid == 0) st.add(WOLFF_STAT_WRITE_BYTES, g.N);
            t_norm = t;
        }
        const uint32_t key = incr ? tag_key(t) : NO_TAG;
        const uint32_t s = seed_site(k0, k1, t, g.N);             // step (i)
        if (tid == 0) {
            st.add(WOLFF_STAT_UPDATES, 1u);
            st.add(WOLFF_STAT_READ_BYTES, 1u);
            st.add(WOLFF_STAT_WRITE_BYTES, 1u);
            const uint32_t a = site_addr<DIM>(g, s);
            const uint32_t b0 = (uint8_t)SG[a];
            int s0;
            int8_t cbyte;
            if (pq) {
                s0 = (int)b0;
                cbyte = (int8_t)potts_new_colour(k0, k1, t, pq, b0);
            } else {
                s0 = (b0 & 2u) ? -1 : 1;
                cbyte = claimed_byte(s0, key);
            }
            SG[a] = cbyte;
            q[0] = s;
            ctl->s0 = s0;
            ctl->cb = cbyte;
            ctl->faces = 0u;
        }
        __syncthreads();
        const int s0 = ctl->s0;
        const int8_t cb = (int8_t)ctl->cb;
        const uint32_t emask = pq ? 0xFFu : 2u;
        const uint32_t evalue = pq ? (uint32_t)s0 : (s0 < 0 ? 2u : 0u);
        const int8_t xb = expanded_byte(s0, key);

        uint32_t head = 0u, tail = 1u, ovn = 0u;                    // the paper's in / ic
        uint64_t csize = 1u;
        uint32_t n_anti = 0u, n_inner = 0u;
        while (true) {
            uint32_t avail = tail - head;
            if (avail < (uint32_t)WG && ovn > 0u) {                 // refill the ring
                const uint32_t m = min(ovn, QC - avail);
                for (uint32_t i = tid; i < m; i += WG) {
                    q[(tail + i) & qmask] = ov[ovn - m + i];
                    st.add(WOLFF_STAT_READ_BYTES, 4u);
                }
                tail += m;
                ovn -= m;
                __syncthreads();
                avail = tail - head;
            }
            if (avail == 0u) break;                                  // step (iv) done
            const uint32_t nproc = min(avail, (uint32_t)WG);
            const bool active = tid < nproc;
            const uint32_t j = active ? q[(head + tid) & qmask] : 0u;
            head += nproc;

            uint32_t self = 0u, par = 0u;
            if (incr) {
                // A bond inside the cluster is counted by the endpoint expanded
                // later.  Two endpoints expanded in the same step differ in
                // parity: the even one is marked expanded before the step's
                // reads, the odd one after them.
                self = site_addr_parity<DIM>(g, j, par);
                if (active && par == 0u) SG[self] = xb;
                __syncthreads();
            }
            uint32_t nb[2 * DIM], sa[2 * DIM];
            neighbours<DIM>(g, j, nb, sa);
            uint32_t wm = 0u;                                         // odd L: slots that wrap around
            if (incr && odd && active) wm = wrap_slots<DIM>(g, j);
            bool won[2 * DIM];
#pragma unroll
            for (int m = 0; m < 2 * DIM; ++m) won[m] = false;
            uint32_t n_act = 0u;
            // a wave with no frontier site this step skips the gathers and the
            // Philox blocks (its SIMD's issue slots go to the waves that work)
            if (__ballot(active) != 0ull)
                expand_site_wg<DIM, WG>(active, j, nb, sa, SG, emask, evalue, cb, key, thr, k0, k1, t,
                                        s, won, tab, n_anti, n_inner, n_act, wm);
            if (tid == 0) st.add(WOLFF_STAT_STEPS, 1u);
            if (active) {
                uint32_t nw = 0u;
#pragma unroll
                for (int m = 0; m < 2 * DIM; ++m) nw += won[m] ? 1u : 0u;
                st.add(WOLFF_STAT_SITES, 1u);
                st.add(WOLFF_STAT_NEIGHBOUR_READS, 2u * DIM);
                st.add(WOLFF_STAT_READ_BYTES, 2u * DIM);                // one byte per neighbour
                st.add(WOLFF_STAT_PHILOX, 1u + DIM);                    // drawn during the gathers
                st.add(WOLFF_STAT_CLAIMS, n_act);
                st.add(WOLFF_STAT_WRITE_BYTES, nw + (incr ? 1u : 0u));  // flips, and the expanded tag
            }
            if (incr && odd) {
                // list the members on a last face (a +mu bond of theirs wraps
                // around) below the top of the overflow stack: the stack holds
                // unexpanded members, the list expanded ones, at most N together
                const bool face = (wm & 0x15u) != 0u;
                const uint64_t fm = __ballot(face);
                if (fm) {
                    uint32_t base = 0u;
                    if (lane == 0) base = atomicAdd(&ctl->faces, (uint32_t)__popcll(fm));
                    base = __shfl(base, 0, WAVE);
                    if (face) {
                        ov[g.N - 1u - (base + lane_prefix(fm))] = j;
                        st.add(WOLFF_STAT_WRITE_BYTES, 4u);
                    }
                }
            }
            uint32_t pos[2 * DIM];
            const uint32_t wtot = wave_compact<DIM>(won, pos);
            if (lane == 0) wave_cnt[wv] = wtot;
            __syncthreads();
            if (incr && active && par != 0u) SG[self] = xb;           // every read of the step is done
            // the step's claims are settled: empty the table for the next step
            {   // eight entries per thread: two 16-byte stores
                uint4* t4 = reinterpret_cast<uint4*>(tab) + 2u * tid;
                const uint4 e = make_uint4(TAB_EMPTY, TAB_EMPTY, TAB_EMPTY, TAB_EMPTY);
                t4[0] = e;
                t4[1] = e;
            }
            uint32_t before = 0u, total = 0u;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = wave_cnt[w];
                before += ((uint32_t)w < wv) ? c : 0u;
                total += c;
            }
            if (total <= QC - (tail - head)) {
#pragma unroll
                for (int m = 0; m < 2 * DIM; ++m)
                    if (won[m]) q[(tail + before + pos[m]) & qmask] = nb[m];
                tail += total;
            } else {
#pragma unroll
                for (int m = 0; m < 2 * DIM; ++m)
                    if (won[m]) {
                        ov[ovn + before + pos[m]] = nb[m];
                        st.add(WOLFF_STAT_WRITE_BYTES, 4u);
                    }
                ovn += total;
            }
            csize += total;
            __syncthreads();
        }

        if (pq)                                                     // exact: colour-0 count moves by +-|C|
            M += (int64_t)pq * (int64_t)csize * ((int64_t)(cb == 0) - (int64_t)(s0 == 0));
        else
            M -= 2 * (int64_t)s0 * (int64_t)csize;                  // exact |dM| = 2|C|
        if (incr) {
            if (odd) {
                // the wrap-around bonds inside the cluster, each from its
                // member on the last face
                const uint32_t nf = ctl->faces;
                for (uint32_t i = tid; i < nf; i += WG) {
                    const uint32_t jf = ov[g.N - 1u - i];
                    const uint32_t wf = wrap_slots<DIM>(g, jf);
                    st.add(WOLFF_STAT_READ_BYTES, 4u + (uint32_t)__popc(wf & 0x15u));
                    const uint32_t L = g.L;
                    uint32_t kk[DIM];
                    kk[0] = jf - (L - 1u);                            // +x of x = L - 1
                    kk[1] = jf - (L - 1u) * L;                        // +y of y = L - 1
                    if (DIM == 3) kk[DIM - 1] = jf - (L - 1u) * g.LL; // +z of z = L - 1
#pragma unroll
                    for (int mu = 0; mu < DIM; ++mu)
                        if ((wf >> (2 * mu)) & 1u)
                            n_inner += is_member((uint8_t)SG[site_addr<DIM>(g, kk[mu])], key) ? 1u : 0u;
                }
            }
            // Flipping C changes only the bonds between C and the rest: with
            // n_anti of them anti-aligned and 2d|C| - n_anti - 2 n_inner
            // aligned, dB = -4 (d |C| - n_anti - n_inner).
            const int64_t w = wave_sum_i64((int64_t)n_anti + (int64_t)n_inner);
            if (lane == 0) red[wv] = w;
            __syncthreads();
            int64_t sum = 0;
#pragma unroll
            for (int w2 = 0; w2 < NW; ++w2) sum += red[w2];
            B -= 4 * ((int64_t)DIM * (int64_t)csize - sum);
        } else if (measure) {
            int64_t Bm, Mm;
            reduce_lattice_wg<WG, DIM>(S, g, red, Bm, Mm, pq);
            B = Bm;
            if (Mm != M) err |= ERR_MAG;
            if (tid == 0) st.add(WOLFF_STAT_READ_BYTES, recount_bytes);
        }
        b_valid = measure;
        if (tid == 0) {
            store_record(rec + u, measure ? B : (int64_t)WOLFF_NOT_MEASURED, M, (int64_t)csize);
            st.add(WOLFF_STAT_WRITE_BYTES, 24u);
            st.add(WOLFF_STAT_READ_BYTES, abort_flag != nullptr ? 4u : 0u);
            ctl->stop = budget_spent(ctl, budget) | abort_requested(abort_flag);
        }
        __syncthreads();
        ++done;
        if (ctl->stop) break;                 // at an update boundary only
    }
    st.flush(R->stats);
    if (tid == 0) {
        R->t = t0 + done;
        R->n_left -= done;
        R->rec_count += done;
        R->M = M;
        R->B = B;
        R->b_valid = b_valid ? 1u : 0u;
        R->t_norm = t_norm;
        R->err |= err;
    }
}

// Persistent batched form: workgroup w starts with replica order[w] and then
// takes order[gridDim.x + atomicAdd(next)] until the list or the time budget
// (wall-clock ticks, 0 = none) is exhausted.  A replica is only ever
// advanced by one workgroup per launch, so its claims need no device-scope
// atomics (they are settled in LDS); the kernel boundary publishes its state
// to the next launch.
// The 512-thread kernels that take simple-cubic lattices are held to four
// waves per SIMD (128 VGPRs, a few spilled), so that two workgroups share a
// CU: on MI355X 3D L = 256 x 2048 replicas ran 14 % faster than at the 142
// VGPRs (three waves per SIMD, one workgroup per CU) the compiler picks by
// itself.  The square-lattice kernel fits four waves as it is (the bound
// made it 3 % slower).
template <int WG, int DIMS>
constexpr int batch_waves_per_eu()
{
    return (WG == 512 && DIMS != 2) ? 4 : 1;
}

template <int WG, int DIMS>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<WG, DIMS>())))
void batch_kernel(Rep* reps, const uint32_t* order,
                                                   uint32_t n_reps, uint32_t* next,
                                                   uint32_t max_updates, uint32_t qmask,
                                                   uint64_t budget)
{
    extern __shared__ __align__(16) uint32_t q[];
    __shared__ uint32_t wave_cnt[WG / WAVE];
    __shared__ long long red[2 * (WG / WAVE)];
    __shared__ WgCtl ctl;
    if (threadIdx.x == 0) {
        ctl.t_start = wall_clock64();
        ctl.stop = 0u;
    }
    for (uint32_t i = threadIdx.x; i < tab_entries(WG); i += WG) q[qmask + 1u + i] = TAB_EMPTY;
    __syncthreads();
    uint32_t idx = blockIdx.x;
    while (idx < n_reps) {
        // the replica is the same for the whole workgroup: keep its index and
        // every descriptor field in scalar registers
        const uint32_t r = __builtin_amdgcn_readfirstlane(order[idx]);
        Rep* R = reps + r;
        if (DIMS == 2 || (DIMS == 0 && R->dim == 2))
            run_rep<WG, 2>(R, max_updates, budget, qmask, q, wave_cnt, red, &ctl);
        else
            run_rep<WG, 3>(R, max_updates, budget, qmask, q, wave_cnt, red, &ctl);
        if (threadIdx.x == 0) {
            ctl.stop = budget_spent(&ctl, budget);
            ctl.idx = ctl.stop ? n_reps : gridDim.x + atomicAdd(next, 1u);
        }
        __syncthreads();
        idx = __builtin_amdgcn_readfirstlane(ctl.idx);
        __syncthreads();
    }
}

// Remove the member tags from a lattice, grid-wide (before the team path,
// which works on plain bytes, takes over a lattice, and at the end of a
// no-allocation run on a caller's lattice).
__global__ void plain_kernel(int8_t* S, uint32_t N)
{
    clear_tags(S, N, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ void reset_counter_kernel(uint32_t* c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0u;
}

// Initial state: iid +-1 (Ising) or iid colours (Potts) from the domain-2
// stream (site i named logically, stored at its address).
__global__ void init_kernel(int8_t* S, Geo g, int dim, uint32_t k0, uint32_t k1, uint32_t q)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < g.N; i += stride) {
        const U4 r = philox(i, 0u, 0u, DOMAIN_INIT, k0, k1);
        const uint32_t a = (dim == 2) ? site_addr<2>(g, i) : site_addr<3>(g, i);
        if (q)                                            // Potts colour floor(x0 q / 2^32)
            S[a] = (int8_t)__umulhi(r.x, q);
        else
            S[a] = (r.x < 0x80000000u) ? (int8_t)1 : (int8_t)-1;
    }
}

// (B, M) of one lattice by one workgroup, written to its descriptor.
template <int WG>
__global__ __launch_bounds__(WG) void measure_rep_kernel(Rep* R)
{
    __shared__ long long red[2 * (WG / WAVE)];
    int64_t B, M;
    const Geo g = R->geo;
    if (R->dim == 2)
        reduce_lattice_wg<WG, 2>(R->S, g, red, B, M, R->q);
    else
        reduce_lattice_wg<WG, 3>(R->S, g, red, B, M, R->q);
    if (threadIdx.x == 0) {
        R->B = B;
        R->M = M;
        R->b_valid = 1u;
    }
}

// ------------------------------------------------ multi-workgroup team path
// One update of one lattice by a team of workgroups.  team_seed_kernel draws
// the seed site, claims it and publishes it as entry 0 of the global queue.
// Every team workgroup expands sites from its own LDS ring; new sites beyond
// `keep` go to the global queue (slots reserved with one atomicAdd on tail,
// each entry tagged with the update's epoch so that a reader can tell a
// written slot from a reserved one); a workgroup whose ring is empty takes a
// chunk of slots with a CAS on head.  pending counts claimed sites not yet
// expanded: a workgroup adds (new - expanded) once per step, before its new
// sites become visible, so pending reaches 0 exactly when the cluster is
// complete (steps (iii)-(iv) of Section 2).  The last workgroup to leave
// writes the magnetisation and, without measurement, the record.
__global__ void team_seed_kernel(Rep* R, TeamCtl* ctl, unsigned long long* gq)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (abort_requested(R->abort)) {             // stop request: leave the update undone
        ctl->aborted = 1u;
        return;
    }
    ctl->aborted = 0u;
    const Geo g = R->geo;
    const uint32_t t = R->t;
    const uint32_t s = seed_site(R->k0, R->k1, t, g.N);
    int8_t* S = R->S;
    const uint32_t a = (R->dim == 2) ? site_addr<2>(g, s) : site_addr<3>(g, s);
    const int s0 = S[a];
    int c = 0;
    if (R->q) {                                   // Potts: the cluster's new colour
        c = (int)potts_new_colour(R->k0, R->k1, t, R->q, (uint32_t)s0);
        S[a] = (int8_t)c;
    } else {
        claim<SCOPE_AGENT>(S, a, s0);
    }
    uint32_t epoch = ctl->epoch + 1u;
    if (epoch == 0u) epoch = 1u;
    ctl->epoch = epoch;
    ctl->s = s;
    ctl->s0 = s0;
    ctl->cb = c;
    ctl->head = 0u;
    ctl->tail = 1u;
    ctl->pending = 1;
    ctl->exited = 0u;
    ctl->csize = 1ull;
    ctl->acc_diff = 0;
    ctl->acc_neg = 0;
    ctl->blocks_done = 0u;
    gq[0] = ((unsigned long long)epoch << 32) | s;
    if (WOLFF_STATS && R->stats) {
        atomicAdd(&R->stats[WOLFF_STAT_UPDATES], 1ull);
        atomicAdd(&R->stats[WOLFF_STAT_READ_BYTES], 1ull);
        atomicAdd(&R->stats[WOLFF_STAT_WRITE_BYTES], 8ull + 1ull);      // queue entry 0 and the flip
    }
}

template <int WG, int DIM>
__global__ __launch_bounds__(WG) void team_kernel(Rep* R, TeamCtl* ctl, unsigned long long* gq,
                                                  uint32_t qmask, uint32_t keep)
{
    constexpr int NW = WG / WAVE;
    extern __shared__ __align__(16) uint32_t q[];
    __shared__ uint32_t wave_cnt[NW];
    __shared__ uint32_t sh_take[3];   // first slot, count, done flag
    __shared__ uint32_t sh_push;

    if (ctl->aborted) return;                    // the seed kernel saw a stop request
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (WAVE - 1);
    const uint32_t wv = tid / WAVE;
    int8_t* S = R->S;
    const Geo g = R->geo;
    const uint32_t thr = R->thr, k0 = R->k0, k1 = R->k1, t = R->t;
    const uint32_t s = ctl->s;
    const int s0 = ctl->s0;
    const uint32_t epoch = ctl->epoch;
    const uint32_t pq = R->q;
    const uint32_t cnew = (uint32_t)ctl->cb;

    uint32_t head = 0u, tail = 0u;           // local ring
    uint64_t my_claims = 0u;
    StatAcc st;                              // counting build only
    while (true) {
        if (tail == head) {
            // take a chunk from the global queue, or leave when pending is 0
            if (tid == 0) {
                uint32_t first = 0u, cnt = 0u, done = 0u;
                uint32_t backoff = 1u, polls = 0u;
                while (true) {
                    st.add(WOLFF_STAT_READ_BYTES, 8u);          // head and tail
                    if (++polls > TEAM_SPIN_LIMIT) {           // never expected: flag and leave
                        __hip_atomic_fetch_or(&R->err, ERR_TEAM_WAIT, __ATOMIC_RELAXED, SCOPE_AGENT);
                        done = 1u;
                        break;
                    }
                    const uint32_t h = __hip_atomic_load(&ctl->head, __ATOMIC_RELAXED, SCOPE_AGENT);
                    const uint32_t tl = __hip_atomic_load(&ctl->tail, __ATOMIC_RELAXED, SCOPE_AGENT);
                    if (h < tl) {
                        uint32_t want = tl - h;
                        if (want > (uint32_t)WG) want = WG;
                        uint32_t expected = h;
                        st.add(WOLFF_STAT_ATOMIC_BYTES, 4u);
                        if (__hip_atomic_compare_exchange_strong(&ctl->head, &expected, h + want,
                                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                 SCOPE_AGENT)) {
                            first = h;
                            cnt = want;
                            break;
                        }
                        continue;
                    }
                    st.add(WOLFF_STAT_READ_BYTES, 4u);
                    st.add(WOLFF_STAT_IDLE_POLLS, 1u);
                    if (__hip_atomic_load(&ctl->pending, __ATOMIC_RELAXED, SCOPE_AGENT) == 0) {
                        done = 1u;
                        break;
                    }
                    // back off: up to 8 x 64 cycles between polls
                    for (uint32_t b = 0; b < backoff; ++b) __builtin_amdgcn_s_sleep(1);
                    if (backoff < 8u) backoff <<= 1;
                }
                sh_take[0] = first;
                sh_take[1] = cnt;
                sh_take[2] = done;
            }
            __syncthreads();
            const uint32_t first = sh_take[0], cnt = sh_take[1], done = sh_take[2];
            __syncthreads();
            if (done) break;
            if (tid < cnt) {
                // the slot was reserved by a running producer that writes it
                // right after its reservation; the wait is bounded anyway
                unsigned long long v = __hip_atomic_load(&gq[first + tid], __ATOMIC_RELAXED, SCOPE_AGENT);
                uint32_t polls = 0u;
                st.add(WOLFF_STAT_READ_BYTES, 8u);
                while ((uint32_t)(v >> 32) != epoch) {
                    if (++polls > TEAM_SPIN_LIMIT) {
                        __hip_atomic_fetch_or(&R->err, ERR_TEAM_WAIT, __ATOMIC_RELAXED, SCOPE_AGENT);
                        v = ((unsigned long long)epoch << 32) | s;   // a member already: expands to nothing
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    v = __hip_atomic_load(&gq[first + tid], __ATOMIC_RELAXED, SCOPE_AGENT);
                    st.add(WOLFF_STAT_READ_BYTES, 8u);
                }
                q[(tail + tid) & qmask] = (uint32_t)v;
            }
            tail += cnt;
            __syncthreads();
        }

        const uint32_t avail = tail - head;
        const uint32_t nproc = min(avail, (uint32_t)WG);
        const bool active = tid < nproc;
        const uint32_t j = active ? q[(head + tid) & qmask] : 0u;
        head += nproc;

        uint32_t nb[2 * DIM];
        bool won[2 * DIM];
        uint32_t n_act = 0u;
#pragma unroll
        for (int m = 0; m < 2 * DIM; ++m) won[m] = false;
        if (__ballot(active) != 0ull)           // idle waves skip the gathers and Philox blocks
            expand_site<DIM, SCOPE_AGENT>(active, j, g, S, s0, thr, k0, k1, t, s, nb, won, n_act, pq, cnew);
        if (tid == 0) st.add(WOLFF_STAT_STEPS, 1u);
        if (active) {
            st.add(WOLFF_STAT_SITES, 1u);
            st.add(WOLFF_STAT_NEIGHBOUR_READS, 2u * DIM);
            st.add(WOLFF_STAT_READ_BYTES, 2u * DIM);
            st.add(WOLFF_STAT_PHILOX, 1u + DIM);
            st.add(WOLFF_STAT_CLAIMS, n_act);
            st.add(WOLFF_STAT_ATOMIC_BYTES, 4u * n_act);      // 32-bit claim atomics
        }
        uint32_t pos[2 * DIM];
        const uint32_t wtot = wave_compact<DIM>(won, pos);
        if (lane == 0) wave_cnt[wv] = wtot;
        __syncthreads();
        uint32_t before = 0u, total = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t c = wave_cnt[w];
            before += ((uint32_t)w < wv) ? c : 0u;
            total += c;
        }
        // keep up to `keep` sites locally, publish the rest
        const uint32_t local_now = tail - head;
        uint32_t n_keep = 0u;
        if (local_now < keep) n_keep = min(total, keep - local_now);
        const uint32_t n_push = total - n_keep;
        if (tid == 0) {
            const int32_t delta = (int32_t)total - (int32_t)nproc;
            if (delta != 0) __hip_atomic_fetch_add(&ctl->pending, delta, __ATOMIC_RELAXED, SCOPE_AGENT);
            if (n_push > 0u)
                sh_push = __hip_atomic_fetch_add(&ctl->tail, n_push, __ATOMIC_RELAXED, SCOPE_AGENT);
            st.add(WOLFF_STAT_ATOMIC_BYTES, (delta != 0 ? 4u : 0u) + (n_push > 0u ? 4u : 0u));
        }
        __syncthreads();
        const uint32_t gbase = sh_push;
#pragma unroll
        for (int m = 0; m < 2 * DIM; ++m) {
            if (won[m]) {
                const uint32_t r = before + pos[m];
                if (r < n_keep) {
                    q[(tail + r) & qmask] = nb[m];
                } else {
                    const unsigned long long v = ((unsigned long long)epoch << 32) | nb[m];
                    __hip_atomic_store(&gq[gbase + (r - n_keep)], v, __ATOMIC_RELAXED, SCOPE_AGENT);
                    st.add(WOLFF_STAT_WRITE_BYTES, 8u);
                }
            }
        }
        tail += n_keep;
        my_claims += total;
        __syncthreads();
    }

    if (tid == 0) st.add(WOLFF_STAT_ATOMIC_BYTES, (my_claims ? 8u : 0u) + 4u);
    st.flush(R->stats);
    if (tid == 0) {
        if (my_claims)
            __hip_atomic_fetch_add(&ctl->csize, (unsigned long long)my_claims, __ATOMIC_RELAXED,
                                   SCOPE_AGENT);
        const uint32_t prev =
            __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_ACQ_REL, SCOPE_AGENT);
        if (prev == gridDim.x - 1u) {
            const unsigned long long csize =
                __hip_atomic_load(&ctl->csize, __ATOMIC_RELAXED, SCOPE_AGENT);
            const int64_t M = pq ? R->M + (int64_t)pq * (int64_t)csize *
                                              ((int64_t)(cnew == 0u) - (int64_t)(s0 == 0))
                                 : R->M - 2 * (int64_t)s0 * (int64_t)csize;
            R->M = M;
            if (R->measure == 0u) {
                R->b_valid = 0u;
                wolff_record r;
                r.bond_sum = (int64_t)WOLFF_NOT_MEASURED;
                r.mag = M;
                r.csize = (int64_t)csize;
                R->rec[R->rec_count] = r;
                R->rec_count += 1u;
                R->t = t + 1u;
            }
        }
    }
}

// Grid-wide (B, M) after a team update; the last block writes the record.
template <int DIM>
__global__ __launch_bounds__(256) void measure_grid_kernel(Rep* R, TeamCtl* ctl)
{
    constexpr int WG = 256, NW = WG / WAVE;
    __shared__ long long red[2 * NW];
    if (ctl->aborted) return;
    const Geo g = R->geo;
    const uint32_t pq = R->q;
    uint64_t d, neg;
    if (pq)
        lattice_counts<DIM, 4, true>(R->S, g, blockIdx.x * WG + threadIdx.x, gridDim.x * WG, d, neg);
    else
        lattice_counts<DIM, 4, false>(R->S, g, blockIdx.x * WG + threadIdx.x, gridDim.x * WG, d, neg);
    d = wave_sum_u64(d);
    neg = wave_sum_u64(neg);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        red[threadIdx.x / WAVE] = (long long)d;
        red[NW + threadIdx.x / WAVE] = (long long)neg;
    }
    __syncthreads();
    if (WOLFF_STATS && R->stats && blockIdx.x == 0 && threadIdx.x == 0) {
        // the whole recount: 16-site chunks with their +x word and +y (+z) chunks
        const uint64_t bytes = (g.tiled || (g.L & 15u) == 0u)
                                   ? (uint64_t)(g.N / 16u) * (DIM == 2 ? 36u : 52u)
                                   : (uint64_t)g.N * (1u + DIM);
        atomicAdd(&R->stats[WOLFF_STAT_READ_BYTES], (unsigned long long)bytes);
        atomicAdd(&R->stats[WOLFF_STAT_WRITE_BYTES], 24ull);
        atomicAdd(&R->stats[WOLFF_STAT_ATOMIC_BYTES], 16ull * gridDim.x + 4ull * gridDim.x);
    }
    if (threadIdx.x == 0) {
        long long sd = 0, sn = 0;
        for (int w = 0; w < NW; ++w) {
            sd += red[w];
            sn += red[NW + w];
        }
        __hip_atomic_fetch_add(&ctl->acc_diff, sd, __ATOMIC_RELAXED, SCOPE_AGENT);
        __hip_atomic_fetch_add(&ctl->acc_neg, sn, __ATOMIC_RELAXED, SCOPE_AGENT);
        const uint32_t prev =
            __hip_atomic_fetch_add(&ctl->blocks_done, 1u, __ATOMIC_ACQ_REL, SCOPE_AGENT);
        if (prev == gridDim.x - 1u) {
            const long long td = __hip_atomic_load(&ctl->acc_diff, __ATOMIC_RELAXED, SCOPE_AGENT);
            const long long tn = __hip_atomic_load(&ctl->acc_neg, __ATOMIC_RELAXED, SCOPE_AGENT);
            const int64_t B = pq ? (int64_t)pq * td - (int64_t)DIM * (int64_t)g.N
                                 : (int64_t)DIM * (int64_t)g.N - 2 * (int64_t)td;
            const int64_t Mm = pq ? (int64_t)pq * tn - (int64_t)g.N : (int64_t)g.N - 2 * (int64_t)tn;
            const int64_t M = R->M;
            if (Mm != M) R->err |= ERR_MAG;
            R->B = B;
            R->b_valid = 1u;
            wolff_record r;
            r.bond_sum = B;
            r.mag = M;
            r.csize = (int64_t)ctl->csize;
            R->rec[R->rec_count] = r;
            R->rec_count += 1u;
            R->t = R->t + 1u;
        }
    }
}

// explicit instantiations used by the host code
template __global__ void batch_kernel<64, 0>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<64, 2>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<64, 3>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<128, 0>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<128, 2>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<128, 3>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<256, 0>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<256, 2>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<256, 3>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<512, 0>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<512, 2>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<512, 3>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<1024, 0>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<1024, 2>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void batch_kernel<1024, 3>(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);
template __global__ void measure_rep_kernel<1024>(Rep*);
template __global__ void team_kernel<256, 2>(Rep*, TeamCtl*, unsigned long long*, uint32_t, uint32_t);
template __global__ void team_kernel<256, 3>(Rep*, TeamCtl*, unsigned long long*, uint32_t, uint32_t);
template __global__ void measure_grid_kernel<2>(Rep*, TeamCtl*);
template __global__ void measure_grid_kernel<3>(Rep*, TeamCtl*);

}  // namespace wolff
