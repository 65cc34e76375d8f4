// LDS-resident growth path of the Wolff update (Section 2, steps (i)-(v);
// the cluster grown frontier-parallel as in Section 4, step (iii')).
//
// The lattice of an Ising run lives in the LDS of a team of G workgroups
// for a whole launch, one bit per spin: workgroup g holds slab g, a range of
// whole rows (2D) or whole planes (3D).  Neighbour gathers and claims are LDS
// reads and LDS atomics; only a bond that leaves the slab goes through
// global memory, as a message to the slab that owns the far site.  With
// G = 1 (a lattice that fits one workgroup's LDS) nothing leaves the
// workgroup at all.
//
// Layout of a slab: rows of Lp = 32 * ceil(L / 32) bits, row r of the
// lattice (r = y in 2D, r = z L + y in 3D) at bit (r - r0) Lp of its slab,
// site x of a row at bit x; bit 1 = spin -1.  A site is named by its logical
// index j = x + L r, as everywhere else (random-stream counters, messages,
// records).
//
// Per update t, every workgroup draws the seed site s; its owner claims it
// (the claim flips the bit) and starts the frontier.  A workgroup expands
// sites from an LDS ring (spilling to a private global stack), claims local
// neighbours whose bond is active with an LDS atomic OR / AND that flips the
// bit (exactly one caller sees the old bit equal to the seed spin s0), and
// sends a message (site, s0) for every active bond whose far site is in
// another slab; the receiver claims it if its spin is s0.  Messages travel
// on single-producer rings: slab g reads one ring filled by slab g - 1 and
// one filled by slab g + 1, so a sender places its messages at counters it
// keeps itself (no slot reservation) and then publishes the ring's new end
// with a plain store; entries carry the update index, so a receiver that
// reads an end before the entries below it simply waits for their tags.
// A device-scope counter P = (t + 1) << 32 | outstanding units decides when
// the cluster is complete.  The units are one per busy workgroup (a
// workgroup with sites to expand), one per message not yet consumed, and
// credit: before a step that could send more messages than its workgroup's
// remaining credit, the workgroup adds a block of credit to P (the addition
// issued at the step's start and waited for before the step's messages are
// written, so its latency hides behind the expansion); a message spends one
// unit of credit, and the receiver removes it when it consumes the message,
// in the same addition that takes the receiver's busy unit if the message
// gave it sites.  A workgroup that runs out of work hands back its busy unit
// and its unspent credit.  So P never reaches 0 while work or a message is
// left, and a busy workgroup's steps leave P alone.  After P reaches
// 0 the team counts the bond sum (every slab its rows plus the rows it
// shares with the next slab, whose first row each slab publishes) and its
// negative spins, and the last workgroup at the update's grid barrier writes
// the record.  The barrier also orders the updates: no workgroup starts
// update t + 1 before all have finished update t.
#pragma once

#include "wolff_kernels.h"

namespace wolff {

// Geometry of the bit lattice and its slabs (host-computed).
struct LdsGeo {
    uint32_t L;
    uint32_t N;             // L^dim
    uint32_t Lp;            // bits per row (L rounded up to 32)
    uint32_t RW;            // words per row
    uint32_t rows;          // rows of the lattice: L (2D), L * L (3D)
    uint32_t slab_rows;     // rows per slab (3D: a multiple of L)
    uint32_t slab_words;    // slab_rows * RW
    uint32_t G;             // slabs (workgroups)
    Div dL;                 // division by L
    Div dslab;              // division of a row index by slab_rows
};

// Team state in device memory (zeroed once when the lattice first takes
// this path; every field is back to its idle value at the end of a launch).
struct LdsCtl {
    unsigned long long P;          // (epoch << 32) | outstanding units; epoch = t + 1
    uint32_t bar_count;            // grid barrier: arrivals
    uint32_t bar_gen;              // grid barrier: generation
    unsigned long long acc_diff;   // this update: differing bonds
    unsigned long long acc_neg;    // this update: negative spins
    unsigned long long acc_claims; // this update: sites claimed (|C|)
    unsigned long long acc_dm;     // this update: change of the magnetisation (two's complement)
    int64_t M;                     // magnetisation after the last update
    int64_t B;                     // bond sum after the last measured update
    uint32_t stop;                 // 1: stop before the next update (stop request)
    uint32_t err;                  // ERR_* bits seen by any workgroup
    uint32_t done;                 // updates completed in this launch
    uint32_t pad;
};

struct LdsArgs {
    Rep* R;
    LdsCtl* ctl;
    unsigned long long* inbox;     // 2G message rings of imask + 1 entries: ring 2g + 0 is
                                   // filled by slab g - 1, ring 2g + 1 by slab g + 1
    uint32_t* inbox_tail;          // 2G counters: entries written to each ring so far (each
                                   // stored only by the ring's one sender; 8-byte aligned)
    uint32_t imask;
    uint32_t* bnd;                 // G * bnd_words: first row (2D) / plane (3D) of every slab
    uint32_t bnd_words;
    uint32_t* ov;                  // G private overflow stacks of ov_stride entries
    uint32_t ov_stride;
    uint32_t qmask;                // LDS ring entries - 1
    LdsGeo lg;
};

constexpr uint32_t MSG_S0_NEG = 0x80000000u;   // message word: seed spin -1
// Bound on the polls of one wait (a poll is ~0.3 to 1 us: seconds in all,
// far above any legitimate wait).  A wait past it flags ERR_TEAM_WAIT and
// the stop request, so the launch ends at the next update boundary.
constexpr uint32_t LDS_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ void flag_wait_failure(LdsCtl* ctl);

__device__ __forceinline__ uint64_t ld_agent(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, SCOPE_AGENT);
}
// The ends of the two message rings slab g reads, in one load: ring 2g + 0
// (filled by slab g - 1) in the low word, ring 2g + 1 in the high word.
__device__ __forceinline__ uint64_t ld_tails(const uint32_t* tails, uint32_t g)
{
    return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(tails + 2u * g),
                             __ATOMIC_RELAXED, SCOPE_AGENT);
}
// Units of P a workgroup of WG threads adds at a time as message credit: at
// least what one step can spend (two far neighbours per site at most).
template <int WG>
constexpr uint32_t credit_block() { return 4u * (uint32_t)WG; }

__device__ __forceinline__ void flag_wait_failure(LdsCtl* ctl)
{
    __hip_atomic_fetch_or(&ctl->err, ERR_TEAM_WAIT, __ATOMIC_RELAXED, SCOPE_AGENT);
    __hip_atomic_store(&ctl->stop, 1u, __ATOMIC_RELAXED, SCOPE_AGENT);
}

// Grid barrier of the G workgroups of a launch (all co-resident).  Thread 0
// arrives; the last arrival runs `last()` (with every other workgroup's
// earlier writes visible) before it opens the barrier.  A wait past its
// bound sets ERR_TEAM_WAIT and leaves.
template <typename F>
__device__ __forceinline__ void grid_barrier(LdsCtl* ctl, uint32_t G, F last)
{
    __syncthreads();            // the workgroup's writes happen before thread 0 arrives
    if (threadIdx.x == 0) {
        if (G == 1) {
            last();
        } else {
            const uint32_t gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, SCOPE_AGENT);
            const uint32_t prev = __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL, SCOPE_AGENT);
            if (prev == G - 1u) {
                last();
                __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, SCOPE_AGENT);
                __hip_atomic_store(&ctl->bar_gen, gen + 1u, __ATOMIC_RELEASE, SCOPE_AGENT);
            } else {
                uint32_t polls = 0u;
                while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, SCOPE_AGENT) == gen) {
                    if (++polls > LDS_SPIN_LIMIT) {
                        flag_wait_failure(ctl);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
        }
    }
    __syncthreads();
}

// Bit address of site (x, row r) inside its slab (r0 = first row of the slab).
__device__ __forceinline__ uint32_t slab_bit(const LdsGeo& lg, uint32_t x, uint32_t r, uint32_t r0)
{
    return (r - r0) * lg.Lp + x;
}

__device__ __forceinline__ uint32_t bit_of(const uint32_t* bits, uint32_t a)
{
    return (bits[a >> 5] >> (a & 31u)) & 1u;
}

// Claim local bit a for a cluster of seed bit b0 (0: spin +1, 1: spin -1):
// flip it to !b0 with one LDS atomic; true for the one caller that found b0.
__device__ __forceinline__ bool claim_bit(uint32_t* bits, uint32_t a, uint32_t b0)
{
    const uint32_t m = 1u << (a & 31u);
    if (b0 == 0u) return (atomicOr(&bits[a >> 5], m) & m) == 0u;
    return (atomicAnd(&bits[a >> 5], ~m) & m) != 0u;
}

// Count differing bonds and negative spins of the slab's rows: the +x bond
// of every site, the +y bond (2D: to the next row, 3D: within the plane),
// and the +z bond (3D: to the next plane).  A bond to the next slab's first
// row / plane reads it from global memory, where that slab published it
// (G = 1 never does: every row is its own).  Items: words of the slab,
// thread-strided.
template <int WG, int DIM>
__device__ __forceinline__ void slab_counts(const uint32_t* bits, const LdsGeo& lg, uint32_t g,
                                            const uint32_t* next_first_global, uint64_t& ndiff,
                                            uint64_t& nneg, StatAcc& st)
{
    const uint32_t r0 = g * lg.slab_rows;
    const uint32_t nrows = min(lg.slab_rows, lg.rows - r0);
    const uint32_t RW = lg.RW, L = lg.L;
    const uint32_t tail_bits = L - (RW - 1u) * 32u;                  // valid bits of a row's last word
    const uint32_t tail_mask = tail_bits == 32u ? 0xFFFFFFFFu : ((1u << tail_bits) - 1u);
    uint64_t d = 0u, neg = 0u;
    for (uint32_t w = threadIdx.x; w < nrows * RW; w += WG) {
        const uint32_t lr = w / RW;
        const uint32_t wi = w - lr * RW;
        const uint32_t v = bits[w];
        const bool last_word = wi == RW - 1u;
        const uint32_t valid = last_word ? tail_mask : 0xFFFFFFFFu;
        neg += __popc(v & valid);
        // +x: bit i against bit i + 1 of the row (bit L - 1 against bit 0)
        uint32_t nx;
        if (!last_word) {
            nx = (v >> 1) | (bits[w + 1u] << 31);
        } else {
            const uint32_t first = bits[w - wi] & 1u;
            nx = (v >> 1) | (first << (tail_bits - 1u));
            if (tail_bits == 32u) nx = (v >> 1) | (first << 31);
        }
        d += __popc((v ^ nx) & valid);
        // +y / +z neighbours: row words
        const uint32_t r = r0 + lr;
        if (DIM == 2) {
            const uint32_t ry = (r + 1u == lg.rows) ? 0u : r + 1u;  // row of the +y neighbours
            const bool here = ry >= r0 && ry < r0 + nrows;
            const uint32_t vy = here ? bits[(ry - r0) * RW + wi]
                                     : ld_agent(&next_first_global[wi]);   // the next slab's first row
            st.add(WOLFF_STAT_READ_BYTES, here ? 0u : 4u);
            d += __popc((v ^ vy) & valid);
        } else {
            const uint32_t z = lg.dL.div(r);
            const uint32_t y = r - z * L;
            const uint32_t ry = (y + 1u == L) ? r + 1u - L : r + 1u;   // +y: within the plane
            d += __popc((v ^ bits[(ry - r0) * RW + wi]) & valid);
            const uint32_t rz = (r + L >= lg.rows) ? r + L - lg.rows : r + L;
            const bool here = rz >= r0 && rz < r0 + nrows;
            const uint32_t vz = here ? bits[(rz - r0) * RW + wi]
                                     : ld_agent(&next_first_global[y * RW + wi]);  // row y of the next slab's first plane
            st.add(WOLFF_STAT_READ_BYTES, here ? 0u : 4u);
            d += __popc((v ^ vz) & valid);
        }
    }
    ndiff = d;
    nneg = neg;
}

// Neighbour slot m of site j (+x, -x, +y, -y[, +z, -z]) as (row, column).
template <int DIM>
__device__ __forceinline__ void lds_neighbour(const LdsGeo& lg, uint32_t j, uint32_t m, uint32_t& nr,
                                              uint32_t& nc)
{
    const uint32_t L = lg.L;
    const uint32_t r = lg.dL.div(j);
    const uint32_t x = j - r * L;
    const uint32_t mu = m >> 1;
    const bool plus = (m & 1u) == 0u;
    if (mu == 0u) {
        nr = r;
        nc = plus ? ((x + 1u == L) ? 0u : x + 1u) : ((x == 0u) ? L - 1u : x - 1u);
        return;
    }
    nc = x;
    if (DIM == 2) {
        nr = plus ? ((r + 1u == L) ? 0u : r + 1u) : ((r == 0u) ? L - 1u : r - 1u);
    } else {
        const uint32_t z = lg.dL.div(r);
        const uint32_t y = r - z * L;
        if (mu == 1u)
            nr = plus ? ((y + 1u == L) ? r + 1u - L : r + 1u) : ((y == 0u) ? r + L - 1u : r - 1u);
        else
            nr = plus ? ((z + 1u == L) ? y : r + L) : ((z == 0u) ? r + lg.rows - L : r - L);
    }
}

// Claims of up to NS local bits for a cluster of seed bit b0; every atomic
// is issued before any result is used.
template <int NS>
__device__ __forceinline__ void claim_bits(uint32_t* bits, const uint32_t ba[NS], const bool act[NS],
                                           uint32_t b0, bool won[NS])
{
    uint32_t old[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        const uint32_t msk = 1u << (ba[m] & 31u);
        old[m] = 0u;
        if (act[m])
            old[m] = (b0 == 0u) ? atomicOr(&bits[ba[m] >> 5], msk) : atomicAnd(&bits[ba[m] >> 5], ~msk);
    }
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        const uint32_t msk = 1u << (ba[m] & 31u);
        won[m] = act[m] && (((old[m] & msk) != 0u) == (b0 != 0u));
    }
}

// Thread 0: a read of the ring ends issued at the start of a step, published
// to the workgroup one step later, after the first barrier of that step (so
// that no wave still reads the previous value and no wait is needed: the
// read is a step old, and the step's own stores are not issued yet).
struct TailRead {
    uint64_t v;
    bool ok;        // issued and not yet published
    bool fresh;     // issued during the current step
};

// Second half of a growth step, for NS neighbour slots per lane: compaction
// of the claimed sites and of the messages (to the previous / next slab),
// publication of the ring ends read a step earlier, the messages (paid from
// the credit), and the claimed sites appended to the ring or the overflow
// stack.  A busy workgroup's own sites are not counted in P (its one busy
// unit stands for all of them), so a step changes P only through credit.
template <int WG, int NS>
__device__ __forceinline__ void lds_publish(const LdsArgs& a, uint32_t* q, uint32_t* wave_cnt,
                                            uint32_t* wave_snd, uint32_t* sh, gword* ov, const bool won[NS],
                                            const bool snd[NS], const bool to_next[NS],
                                            const uint32_t nb[NS],
                                            unsigned long long epoch, uint32_t b0, uint32_t gprev,
                                            uint32_t gnext, uint32_t G, uint32_t QC, uint32_t& head,
                                            uint32_t& tail, uint32_t& ovn, uint32_t& claims,
                                            uint32_t& cprev, uint32_t& cnext, uint32_t& credit,
                                            TailRead& tr, StatAcc& st)
{
    constexpr int NW = WG / WAVE;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (WAVE - 1);
    const uint32_t wv = tid / WAVE;
    uint32_t pos[NS], spos[NS];
    uint32_t wtot = 0u;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        const uint64_t mask = __ballot(won[m]);
        pos[m] = wtot + lane_prefix(mask);
        wtot += (uint32_t)__popcll(mask);
    }
    uint32_t sprev = 0u, snext = 0u;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        const uint64_t mp = __ballot(snd[m] && !to_next[m]);
        const uint64_t mn = __ballot(snd[m] && to_next[m]);
        spos[m] = to_next[m] ? snext + lane_prefix(mn) : sprev + lane_prefix(mp);
        sprev += (uint32_t)__popcll(mp);
        snext += (uint32_t)__popcll(mn);
    }
    uint32_t before = 0u, total = wtot, pb = 0u, ptot = sprev, nbf = 0u, ntot = snext;
    if (NW > 1) {
        // the waves' counts through LDS (one wave has its totals already)
        if (lane == 0) {
            wave_cnt[wv] = wtot;
            wave_snd[wv] = sprev;
            wave_snd[NW + wv] = snext;
        }
        __syncthreads();
        total = ptot = ntot = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t c = wave_cnt[w], cp = wave_snd[w], cn = wave_snd[NW + w];
            const bool lower = (uint32_t)w < wv;
            before += lower ? c : 0u;
            pb += lower ? cp : 0u;
            nbf += lower ? cn : 0u;
            total += c;
            ptot += cp;
            ntot += cn;
        }
    }
    if (G > 1u && tid == 0) {
        if (tr.ok && !tr.fresh) {
            sh[3] = (uint32_t)tr.v;
            sh[7] = (uint32_t)(tr.v >> 32);
            tr.ok = false;
        }
        tr.fresh = false;
    }
    if (G > 1u) {
        // the messages go to the two rings this workgroup alone fills, at
        // the counters every thread keeps (the same in all); their units
        // come out of the credit already in P (thread 0 waited for the
        // credit's addition before the barrier above)
        if (ptot + ntot > 0u) {
            const unsigned long long word = epoch | (b0 ? MSG_S0_NEG : 0u);
            const uint32_t QI = a.imask + 1u;
#pragma unroll
            for (int m = 0; m < NS; ++m) {
                if (snd[m]) {
                    const size_t ring = to_next[m] ? 2u * (size_t)gnext : 2u * (size_t)gprev + 1u;
                    const uint32_t slot = to_next[m] ? cnext + nbf + spos[m] : cprev + pb + spos[m];
                    __hip_atomic_store(&a.inbox[ring * QI + (slot & a.imask)], word | nb[m],
                                       __ATOMIC_RELAXED, SCOPE_AGENT);
                    st.add(WOLFF_STAT_WRITE_BYTES, 8u);
                    st.add(WOLFF_STAT_MESSAGES, 1u);
                }
            }
            cprev += ptot;
            cnext += ntot;
            if (tid == 0) {
                if (ptot) __hip_atomic_store(&a.inbox_tail[2u * gprev + 1u], cprev, __ATOMIC_RELAXED, SCOPE_AGENT);
                if (ntot) __hip_atomic_store(&a.inbox_tail[2u * gnext], cnext, __ATOMIC_RELAXED, SCOPE_AGENT);
                st.add(WOLFF_STAT_WRITE_BYTES, (ptot ? 4u : 0u) + (ntot ? 4u : 0u));
                st.add(WOLFF_STAT_STEPS_SEND, 1u);
            }
        }
        if (tid == 0) credit -= ptot + ntot;
    }
    // append the claimed sites to the ring (or the overflow stack); the
    // counters move by selects, not through a reference chosen by branch
    // (which the compiler would keep in scratch memory)
    const bool fits = total <= QC - (tail - head);
    const uint32_t qbase = tail + before, obase = ovn + before;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        if (won[m]) {
            if (fits) {
                q[(qbase + pos[m]) & a.qmask] = nb[m];
            } else {
                ov[obase + pos[m]] = nb[m];
                st.add(WOLFF_STAT_WRITE_BYTES, 4u);
            }
        }
    }
    tail += fits ? total : 0u;
    ovn += fits ? 0u : total;
    claims += total;
}

// s_waitcnt with vmcnt(0) and the other counters unconstrained (expcnt 7,
// lgkmcnt 15).  On gfx950 vmcnt counts stores and atomics as well as loads,
// so this waits until every global access the wave issued was performed.
constexpr int WAITCNT_VM0 = 0x0F70;

// Thread 0, before the barrier that precedes a step's messages: the credit
// added (without a returned value) at the step's start must have been
// performed.  A returned value would make the compiler wait at the first
// reuse of its register, and with it for every access issued before.
__device__ __forceinline__ void credit_wait(uint64_t c0, StatAcc& st)
{
    __builtin_amdgcn_s_waitcnt(WAITCNT_VM0);
    if (WOLFF_STATS) st.add(WOLFF_STAT_CYCLES_SEND, clock64() - c0);
}

// Workgroup-shared words of the LDS path beside the slab and the ring.
template <int NW>
struct LdsShm {
    uint32_t wave_cnt[NW];
    uint32_t wave_snd[2 * NW];
    uint64_t red[2 * NW];
    uint32_t sh[16];
};

// All updates of one lattice (up to max_updates, or until the wall-clock
// budget since t_start is spent) by this workgroup and, with MULTI, the
// other G - 1 workgroups of the launch.  MULTI: the lattice spans several
// slabs (messages, P, grid barriers through a.ctl); otherwise this one
// workgroup holds it all, every team-only branch compiles away and a.ctl
// is not used.  TINY: frontiers one wave holds run level after level in
// that wave alone (see the step).
template <int WG, int DIM, bool MULTI, bool TINY>
__device__ __forceinline__ void lds_body(const LdsArgs& a, uint32_t max_updates, uint64_t budget,
                                         uint64_t t_start, uint32_t* lds, LdsShm<WG / WAVE>& shm)
{
    constexpr int NW = WG / WAVE;
    constexpr int D2 = 2 * DIM;
    constexpr uint32_t BOND_SITES = (uint32_t)(WG / D2);    // sites of a one-lane-per-bond step
    constexpr uint32_t TINY_SITES = (uint32_t)(WAVE / D2);  // sites one wave holds, one lane per bond
    uint32_t* wave_cnt = shm.wave_cnt;
    uint32_t* wave_snd = shm.wave_snd;
    uint64_t* red = shm.red;
    uint32_t* sh = shm.sh;
    StatAcc st;                       // counting build only

    const LdsGeo lg = a.lg;
    uint32_t* bits = lds;
    uint32_t* q = lds + ((lg.slab_words + 3u) & ~3u);
    const uint32_t QC = a.qmask + 1u;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (WAVE - 1);
    const uint32_t wv = tid / WAVE;
    const uint32_t g = MULTI ? blockIdx.x : 0u;
    const uint32_t G = MULTI ? lg.G : 1u;
    const uint32_t r0 = g * lg.slab_rows;
    const uint32_t nrows = min(lg.slab_rows, lg.rows - r0);
    const uint32_t L = lg.L;
    Rep* R = a.R;
    LdsCtl* ctl = a.ctl;
    const Geo geo = R->geo;
    const uint32_t thr = R->thr, k0 = R->k0, k1 = R->k1;
    const uint32_t t0 = R->t;
    uint32_t n = R->n_left;
    if (max_updates != 0u && max_updates < n) n = max_updates;
    const bool measure = R->measure != 0u;
    const uint32_t gprev = (g == 0u) ? G - 1u : g - 1u;
    const uint32_t gnext = (g + 1u == G) ? 0u : g + 1u;
    gword* ov = as_global(a.ov + (size_t)g * a.ov_stride);
    const unsigned long long* inbox = a.inbox + 2u * (size_t)g * (a.imask + 1u);
    const gbyte* SG = as_global(R->S);

    // the slab from the int8 lattice (any storage order; bit 1 of a byte is
    // its sign, member tags included)
    for (uint32_t w = tid; w < nrows * lg.RW; w += WG) {
        const uint32_t lr = w / lg.RW;
        const uint32_t x0 = (w - lr * lg.RW) * 32u;
        const uint32_t base = (r0 + lr) * L;
        uint32_t v = 0u;
        for (uint32_t b = 0; b < 32u && x0 + b < L; ++b) {
            const uint32_t j = base + x0 + b;
            const uint32_t addr = (DIM == 2) ? site_addr<2>(geo, j) : site_addr<3>(geo, j);
            v |= (((uint32_t)(uint8_t)SG[addr] >> 1) & 1u) << b;
            st.add(WOLFF_STAT_READ_BYTES, 1u);
        }
        bits[w] = v;
    }
    if (tid == 0) {
        // every message was consumed: the rings this slab reads start at
        // their ends; the counters of the two rings it fills are its own
        const uint64_t it = G > 1u ? ld_tails(a.inbox_tail, g) : 0u;
        sh[0] = sh[3] = (uint32_t)it;
        sh[6] = sh[7] = (uint32_t)(it >> 32);
        sh[8] = G > 1u ? ld_agent(&a.inbox_tail[2u * gnext]) : 0u;
        sh[9] = G > 1u ? ld_agent(&a.inbox_tail[2u * gprev + 1u]) : 0u;
    }
    // a stop request seen before the first update: run none
    if (MULTI) {
        grid_barrier(ctl, G, [&] {
            __hip_atomic_store(&ctl->stop, abort_requested(R->abort), __ATOMIC_RELAXED, SCOPE_AGENT);
            __hip_atomic_store(&ctl->P, (unsigned long long)t0 << 32, __ATOMIC_RELAXED, SCOPE_AGENT);
            ctl->M = R->M;
            ctl->B = R->B;
            ctl->acc_diff = ctl->acc_neg = ctl->acc_claims = 0ull;
            ctl->acc_dm = 0ull;
        });
        if (tid == 0) sh[5] = __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, SCOPE_AGENT);
    } else {
        if (tid == 0) sh[5] = abort_requested(R->abort);
    }
    __syncthreads();
    uint32_t ihead0 = sh[0], ihead1 = sh[6];          // next entries to read, by ring
    uint32_t cnext = sh[8], cprev = sh[9];            // entries written to the rings filled
    uint32_t credit = 0u;                             // thread 0: units of P not yet spent
    if (sh[5]) n = 0u;
    const uint64_t rec0 = R->rec_count;
    __syncthreads();

    // one workgroup (G = 1): M, B and the error bits in thread 0's registers
    int64_t M1 = R->M, B1 = R->B;
    uint32_t err1 = 0u;
    const uint32_t* abort_flag = R->abort;
    uint32_t done = 0u;
    for (; done < n; ++done) {
        const uint32_t t = t0 + done;
        // G = 1: the stop request is read now and used after the update, so
        // that the read's latency hides behind the growth
        uint32_t abort_raw = 0u;
        if (G == 1u && tid == 0) abort_raw = abort_word(abort_flag);
        const unsigned long long epoch = (unsigned long long)(t + 1u) << 32;
        const uint32_t s = seed_site(k0, k1, t, lg.N);                // step (i)
        const uint32_t srow = lg.dL.div(s);
        const uint32_t owner = lg.dslab.div(srow);
        uint32_t head = 0u, tail = 0u, ovn = 0u;
        uint32_t claims = 0u, nstep = 0u;
        TailRead tr{0u, false, false};
        credit = 0u;
        bool busy = false;                                        // thread 0: one unit of P held
        if (tid == 0 && g == 0u) st.add(WOLFF_STAT_UPDATES, 1u);
        if (g == owner) {
            if (tid == 0) {
                const uint32_t a0 = slab_bit(lg, s - srow * L, srow, r0);
                const uint32_t b0 = bit_of(bits, a0);
                claim_bit(bits, a0, b0);
                q[0] = s;
                sh[1] = b0;
                sh[2] = 1u;                                       // s0 known
                if (G > 1u)
                    __hip_atomic_store(&ctl->P, epoch | 1ull, __ATOMIC_RELAXED, SCOPE_AGENT);
                busy = true;                                      // the unit just stored
            }
            tail = 1u;
            claims = 1u;
        } else if (tid == 0) {
            sh[2] = 0u;                                           // s0 not known yet
        }
        __syncthreads();

        while (true) {
            uint32_t avail = tail - head;
            if (avail < (uint32_t)WG && ovn > 0u) {                 // refill the ring
                const uint32_t m = min(ovn, QC - avail);
                for (uint32_t i = tid; i < m; i += WG) {
                    q[(tail + i) & a.qmask] = ov[ovn - m + i];
                    st.add(WOLFF_STAT_READ_BYTES, 4u);
                }
                tail += m;
                ovn -= m;
                __syncthreads();
                avail = tail - head;
            }
            // messages from the other slabs: while the workgroup has work of
            // its own it reads the ends of its two rings (without waiting)
            // during every sixteenth step and sees the value one step later;
            // idle, it polls the ring ends and P.  (Reading every second step, or
            // every fourth, was measured slower on MI355X: 2D L = 4096 at T_c
            // 8.3 and 8.1 against 7.8 ms per update.)
            uint32_t itail0 = ihead0, itail1 = ihead1;
            if (G > 1u) {
                if (avail == 0u) {
                    if (tid == 0) {
                        const uint64_t c_idle = WOLFF_STATS ? clock64() : 0u;
                        if (busy || credit) {                     // out of work: hand back the busy unit and the credit
                            const long long back = (long long)credit + (busy ? 1ll : 0ll);
                            __hip_atomic_fetch_add(&ctl->P, (unsigned long long)(0ll - back),
                                                   __ATOMIC_RELAXED, SCOPE_AGENT);
                            st.add(WOLFF_STAT_ATOMIC_BYTES, 8u);
                            credit = 0u;
                            busy = false;
                        }
                        const uint64_t ih = ((uint64_t)ihead1 << 32) | ihead0;
                        uint64_t it = ld_tails(a.inbox_tail, g);
                        uint32_t fin = 0u;
                        uint32_t polls = 0u, backoff = 1u;
                        while (it == ih) {
                            const unsigned long long p = ld_agent(&ctl->P);
                            if ((p >> 32) > (epoch >> 32) || p == epoch) {
                                // P reached 0: every message was consumed
                                it = ld_tails(a.inbox_tail, g);
                                fin = it == ih ? 1u : 0u;
                                break;
                            }
                            if (++polls > LDS_SPIN_LIMIT ||
                                __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, SCOPE_AGENT)) {
                                if (polls > LDS_SPIN_LIMIT) flag_wait_failure(ctl);
                                fin = 1u;
                                break;
                            }
                            for (uint32_t b = 0; b < backoff; ++b) __builtin_amdgcn_s_sleep(1);
                            if (backoff < 8u) backoff <<= 1;
                            it = ld_tails(a.inbox_tail, g);
                        }
                        sh[3] = (uint32_t)it;
                        sh[7] = (uint32_t)(it >> 32);
                        tr.ok = false;                            // older than what was just read
                        sh[4] = fin;
                        st.add(WOLFF_STAT_IDLE_POLLS, polls + 1u);
                        st.add(WOLFF_STAT_READ_BYTES, 8u + 16u * (polls + 1u));
                        if (WOLFF_STATS) st.add(WOLFF_STAT_CYCLES_IDLE, clock64() - c_idle);
                    }
                    __syncthreads();
                    const uint32_t fin = sh[4];
                    itail0 = sh[3];
                    itail1 = sh[7];
                    __syncthreads();
                    if (fin) break;
                } else {
                    itail0 = sh[3];                               // the latest reads (may lag)
                    itail1 = sh[7];
                }
            } else if (avail == 0u) {
                break;                                            // one workgroup: the cluster is complete
            }

            if (itail0 != ihead0 || itail1 != ihead1) {
                // claim the sites of up to WG messages (the sender found the
                // bond active): lanes [0, m0) read ring 2g + 0, [m0, m0 + m1)
                // ring 2g + 1
                const uint32_t m0 = min(itail0 - ihead0, (uint32_t)WG);
                const uint32_t m1 = min(itail1 - ihead1, (uint32_t)WG - m0);
                const uint32_t m = m0 + m1;
                bool won = false;
                uint32_t k = 0u;
                if (tid < m) {
                    const bool r1 = tid >= m0;
                    const uint32_t idx = r1 ? ihead1 + (tid - m0) : ihead0 + tid;
                    const unsigned long long* slot =
                        &inbox[(r1 ? (size_t)(a.imask + 1u) : 0u) + (idx & a.imask)];
                    unsigned long long v = ld_agent(slot);
                    uint32_t polls = 0u;
                    st.add(WOLFF_STAT_READ_BYTES, 8u);
                    while ((v >> 32) != (epoch >> 32)) {          // counted, not yet visible
                        if (++polls > LDS_SPIN_LIMIT) {
                            flag_wait_failure(ctl);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        v = ld_agent(slot);
                        st.add(WOLFF_STAT_READ_BYTES, 8u);
                    }
                    if ((v >> 32) == (epoch >> 32)) {
                        const uint32_t w = (uint32_t)v;
                        k = w & ~MSG_S0_NEG;
                        const uint32_t b0 = (w & MSG_S0_NEG) ? 1u : 0u;
                        sh[1] = b0;                               // every message carries s0
                        const uint32_t kr = lg.dL.div(k);
                        won = claim_bit(bits, slab_bit(lg, k - kr * L, kr, r0), b0);
                        st.add(WOLFF_STAT_CLAIMS, 1u);
                    }
                }
                const uint64_t mask = __ballot(won);
                const uint32_t pos = lane_prefix(mask);
                if (lane == 0) wave_cnt[wv] = (uint32_t)__popcll(mask);
                __syncthreads();
                uint32_t before = 0u, total = 0u;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const uint32_t c = wave_cnt[w];
                    before += ((uint32_t)w < wv) ? c : 0u;
                    total += c;
                }
                if (total <= QC - (tail - head)) {
                    if (won) q[(tail + before + pos) & a.qmask] = k;
                    tail += total;
                } else {
                    if (won) ov[ovn + before + pos] = k;
                    st.add(WOLFF_STAT_WRITE_BYTES, won ? 4u : 0u);
                    ovn += total;
                }
                claims += total;
                ihead0 += m0;
                ihead1 += m1;
                if (tid == 0) {
                    sh[2] = 1u;
                    // the consumed messages leave P in the same addition that
                    // takes the busy unit if the workgroup now has sites
                    const bool wake = !busy && total > 0u;
                    const long long delta = (wake ? 1ll : 0ll) - (long long)m;
                    busy = busy || wake;
                    if (delta != 0) {
                        __hip_atomic_fetch_add(&ctl->P, (unsigned long long)delta, __ATOMIC_RELAXED, SCOPE_AGENT);
                        st.add(WOLFF_STAT_ATOMIC_BYTES, 8u);
                    }
                }
                __syncthreads();
                continue;
            }
            if (avail == 0u) continue;                            // (G > 1) poll again

            // ---- one growth step (steps (ii)-(iii)).  A wide frontier takes
            // one lane per site (every neighbour of the site in that lane,
            // up to WG sites); a narrow one takes one lane per bond (up to
            // WG / 2d sites), so that its Philox blocks, neighbour reads and
            // claims are spread over 2d times more lanes and the step's
            // chain is one block long instead of 1 + d.
            const uint32_t b0 = sh[1];
            const bool look = G > 1u && (nstep++ & 15u) == 0u;
            if (look && tid == 0) tr = TailRead{ld_tails(a.inbox_tail, g), true, true};
            // message credit for this step, added now and waited for just
            // before the step's messages are written
            bool refill = false;
            if (G > 1u && tid == 0 && credit < 2u * min(avail, (uint32_t)WG)) {
                __hip_atomic_fetch_add(&ctl->P, (unsigned long long)credit_block<WG>(),
                                       __ATOMIC_RELAXED, SCOPE_AGENT);
                credit += credit_block<WG>();
                refill = true;
                st.add(WOLFF_STAT_ATOMIC_BYTES, 8u);
            }
            const uint64_t c_step = (WOLFF_STATS && tid == 0) ? clock64() : 0u;
            uint64_t c_pub = c_step;
            if (tid == 0) st.add(WOLFF_STAT_STEPS, 1u);
            if (look && tid == 0) st.add(WOLFF_STAT_READ_BYTES, 8u);
            if (TINY && avail <= TINY_SITES && ovn == 0u) {
                // ---- a frontier that one wave holds, one lane per bond: wave 0
                // runs level after level alone, with no workgroup barrier, while
                // the frontier stays that small (split lattice: at most 16
                // levels, so that the ring ends are still read); the other waves
                // wait at the barrier below.  One wave's LDS accesses are
                // performed in order, so a level sees the bits and ring entries
                // the previous one wrote.
                if (wv == 0u) {
                    uint32_t av = avail, lv = 0u;
                    while (true) {
                        const uint32_t si = lane / (uint32_t)D2;
                        const uint32_t m = lane - si * (uint32_t)D2;
                        const bool active = si < av;
                        const uint32_t j = active ? q[(head + si) & a.qmask] : 0u;
                        head += av;
                        if (G > 1u && lv > 0u && tid == 0 && credit < 2u * av) {
                            __hip_atomic_fetch_add(&ctl->P, (unsigned long long)credit_block<WG>(),
                                                   __ATOMIC_RELAXED, SCOPE_AGENT);
                            credit += credit_block<WG>();
                            refill = true;
                            st.add(WOLFF_STAT_ATOMIC_BYTES, 8u);
                        }
                        uint32_t nr, nc;
                        lds_neighbour<DIM>(lg, j, m, nr, nc);
                        const uint32_t nbk = nc + nr * L;
                        const bool local = !MULTI || (nr >= r0 && nr < r0 + nrows);
                        const uint32_t ba = local ? slab_bit(lg, nc, nr, r0) : 0u;
                        const bool elig = active && (!local || bit_of(bits, ba) == b0);
                        uint32_t rr = 0xFFFFFFFFu;
                        if (active) {
                            const U4 w4 = philox((m & 1u) ? nbk : j, t, s, DOMAIN_BOND, k0, k1);
                            const uint32_t mu = m >> 1;
                            rr = (mu == 0u) ? w4.x : (mu == 1u) ? w4.y : w4.z;
                        }
                        const bool act = elig && rr < thr;
                        const bool won = act && local && claim_bit(bits, ba, b0);
                        const bool snd = act && !local;
                        const bool nxt = (m & 1u) == 0u;
                        st.add(WOLFF_STAT_SITES, (active && m == 0u) ? 1u : 0u);
                        st.add(WOLFF_STAT_NEIGHBOUR_READS, (active && local) ? 1u : 0u);
                        st.add(WOLFF_STAT_PHILOX, active ? 1u : 0u);
                        st.add(WOLFF_STAT_CLAIMS, (act && local) ? 1u : 0u);
                        if (G > 1u) {
                            const uint64_t mp = __ballot(snd && !nxt), mn = __ballot(snd && nxt);
                            const uint32_t ptot = (uint32_t)__popcll(mp), ntot = (uint32_t)__popcll(mn);
                            if (ptot + ntot > 0u) {
                                if (refill) {
                                    credit_wait(c_pub, st);           // the credit is in P
                                    refill = false;
                                }
                                if (snd) {
                                    const unsigned long long word = epoch | (b0 ? MSG_S0_NEG : 0u);
                                    const uint32_t QI = a.imask + 1u;
                                    const size_t ring = nxt ? 2u * (size_t)gnext : 2u * (size_t)gprev + 1u;
                                    const uint32_t slot = nxt ? cnext + lane_prefix(mn) : cprev + lane_prefix(mp);
                                    __hip_atomic_store(&a.inbox[ring * QI + (slot & a.imask)], word | nbk,
                                                       __ATOMIC_RELAXED, SCOPE_AGENT);
                                    st.add(WOLFF_STAT_WRITE_BYTES, 8u);
                                    st.add(WOLFF_STAT_MESSAGES, 1u);
                                }
                                cprev += ptot;
                                cnext += ntot;
                                if (tid == 0) {
                                    if (ptot) __hip_atomic_store(&a.inbox_tail[2u * gprev + 1u], cprev, __ATOMIC_RELAXED, SCOPE_AGENT);
                                    if (ntot) __hip_atomic_store(&a.inbox_tail[2u * gnext], cnext, __ATOMIC_RELAXED, SCOPE_AGENT);
                                    credit -= ptot + ntot;
                                    st.add(WOLFF_STAT_WRITE_BYTES, (ptot ? 4u : 0u) + (ntot ? 4u : 0u));
                                    st.add(WOLFF_STAT_STEPS_SEND, 1u);
                                }
                            }
                        }
                        // the claimed sites to the ring (it is empty: all av were taken)
                        const uint64_t wm = __ballot(won);
                        const uint32_t total = (uint32_t)__popcll(wm);
                        if (won) q[(tail + lane_prefix(wm)) & a.qmask] = nbk;
                        tail += total;
                        claims += total;
                        ++lv;
                        if (tid == 0) st.add(WOLFF_STAT_STEPS_NARROW, 1u);
                        av = total;
                        if (av == 0u || av > TINY_SITES || (G > 1u && lv >= 16u)) break;
                        if (tid == 0) st.add(WOLFF_STAT_STEPS, 1u);
                        // the next level's lanes read what other lanes of the
                        // wave wrote: order the wave's LDS accesses across levels
                        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                    }
                    if (tid == 0) {
                        if (refill) credit_wait(c_pub, st);       // credit a later step may spend
                        sh[8] = head;
                        sh[9] = tail;
                        sh[11] = claims;
                        sh[12] = cprev;
                        sh[13] = cnext;
                        sh[14] = lv;
                        tr.fresh = false;                         // published by a later step
                    }
                }
                if (WOLFF_STATS && tid == 0) c_pub = clock64();
                __syncthreads();
                head = sh[8];
                tail = sh[9];
                claims = sh[11];
                cprev = sh[12];
                cnext = sh[13];
                nstep += sh[14] - 1u;
            } else if (avail <= BOND_SITES) {
                const uint32_t si = tid / (uint32_t)D2;
                const uint32_t m = tid - si * (uint32_t)D2;
                const uint32_t nproc = min(avail, BOND_SITES);
                const bool active = si < nproc;
                const uint32_t j = active ? q[(head + si) & a.qmask] : 0u;
                head += nproc;
                uint32_t nr, nc;
                lds_neighbour<DIM>(lg, j, m, nr, nc);
                const uint32_t nbk = nc + nr * L;
                const bool local = !MULTI || (nr >= r0 && nr < r0 + nrows);
                const uint32_t ba = local ? slab_bit(lg, nc, nr, r0) : 0u;
                const bool elig = active && (!local || bit_of(bits, ba) == b0);
                uint32_t rr = 0xFFFFFFFFu;
                if (active) {
                    // bond (j, mu) for a +mu slot, (j - e_mu, mu) for a -mu slot;
                    // drawn for every live lane, so that the block does not wait
                    // for the neighbour's bit (1.7 % faster at 2D L = 4096 than
                    // drawing only for eligible lanes)
                    const U4 w4 = philox((m & 1u) ? nbk : j, t, s, DOMAIN_BOND, k0, k1);
                    const uint32_t mu = m >> 1;
                    rr = (mu == 0u) ? w4.x : (mu == 1u) ? w4.y : w4.z;
                }
                const bool act = elig && rr < thr;
                const bool won[1] = {act && local && claim_bit(bits, ba, b0)};
                const bool snd[1] = {act && !local};
                const bool to_next[1] = {(m & 1u) == 0u};
                const uint32_t nb1[1] = {nbk};
                st.add(WOLFF_STAT_SITES, (active && m == 0u) ? 1u : 0u);
                st.add(WOLFF_STAT_NEIGHBOUR_READS, (active && local) ? 1u : 0u);
                st.add(WOLFF_STAT_PHILOX, active ? 1u : 0u);
                st.add(WOLFF_STAT_CLAIMS, (act && local) ? 1u : 0u);
                if (tid == 0) st.add(WOLFF_STAT_STEPS_NARROW, 1u);
                if (WOLFF_STATS && tid == 0) c_pub = clock64();
                if (refill) credit_wait(c_pub, st);
                lds_publish<WG, 1>(a, q, wave_cnt, wave_snd, sh, ov, won, snd, to_next, nb1,
                                   epoch, b0, gprev, gnext, G, QC, head, tail, ovn, claims,
                                   cprev, cnext, credit, tr, st);
            } else {
                const uint32_t nproc = min(avail, (uint32_t)WG);
                const bool active = tid < nproc;
                const uint32_t j = active ? q[(head + tid) & a.qmask] : 0u;
                head += nproc;
                uint32_t nb[D2], ba[D2];
                bool local[D2], elig[D2];
#pragma unroll
                for (int m = 0; m < D2; ++m) {
                    uint32_t nr, nc;
                    lds_neighbour<DIM>(lg, j, (uint32_t)m, nr, nc);
                    nb[m] = nc + nr * L;
                    local[m] = !MULTI || (nr >= r0 && nr < r0 + nrows);
                    ba[m] = local[m] ? slab_bit(lg, nc, nr, r0) : 0u;
                    // a local neighbour is a candidate only if its spin is s0; a
                    // remote one is decided by its owner
                    elig[m] = active && (!local[m] || bit_of(bits, ba[m]) == b0);
                }
                // bond words: one block keyed by j for the +mu bonds, one keyed by
                // j - e_mu per -mu bond, the 1 + d blocks drawn together with
                // their rounds interleaved (a wide step almost always needs all
                // of them somewhere in the wave; drawing each only where a lane
                // needed it, one after the other, was 2.6 % slower at 2D
                // L = 4096 on MI355X)
                uint32_t rp[3] = {0u, 0u, 0u}, rm[3] = {0u, 0u, 0u};
                if (active) {
                    uint32_t ctr[1 + DIM];
                    U4 w[1 + DIM];
                    ctr[0] = j;
#pragma unroll
                    for (int mu = 0; mu < DIM; ++mu) ctr[1 + mu] = nb[2 * mu + 1];
                    philox_multi<1 + DIM>(ctr, t, s, DOMAIN_BOND, k0, k1, w);
                    rp[0] = w[0].x;
                    rp[1] = w[0].y;
                    rp[2] = w[0].z;
#pragma unroll
                    for (int mu = 0; mu < DIM; ++mu)
                        rm[mu] = (mu == 0) ? w[1 + mu].x : (mu == 1) ? w[1 + mu].y : w[1 + mu].z;
                }
                bool act[D2], won[D2], snd[D2], to_next[D2];
#pragma unroll
                for (int m = 0; m < D2; ++m) {
                    const uint32_t rr = (m & 1) ? rm[m / 2] : rp[m / 2];
                    act[m] = elig[m] && rr < thr && local[m];
                    snd[m] = elig[m] && rr < thr && !local[m];
                    to_next[m] = (m & 1) == 0;
                }
                // every claim's LDS atomic in flight at once
                claim_bits<D2>(bits, ba, act, b0, won);
                if (active) {
                    uint32_t nl = 0u, nc = 0u;
#pragma unroll
                    for (int m = 0; m < D2; ++m) {
                        nl += local[m] ? 1u : 0u;
                        nc += act[m] ? 1u : 0u;
                    }
                    const uint32_t nblk = 1u + (uint32_t)DIM;
                    st.add(WOLFF_STAT_SITES, 1u);
                    st.add(WOLFF_STAT_NEIGHBOUR_READS, nl);
                    st.add(WOLFF_STAT_PHILOX, nblk);
                    st.add(WOLFF_STAT_CLAIMS, nc);
                }
                if (WOLFF_STATS && tid == 0) c_pub = clock64();
                if (refill) credit_wait(c_pub, st);
                lds_publish<WG, D2>(a, q, wave_cnt, wave_snd, sh, ov, won, snd, to_next, nb,
                                    epoch, b0, gprev, gnext, G, QC, head, tail, ovn, claims,
                                    cprev, cnext, credit, tr, st);
            }
            __syncthreads();
            if (WOLFF_STATS && tid == 0) {
                const uint64_t c_end = clock64();
                st.add(WOLFF_STAT_CYCLES_GROW, c_end - c_step);
                st.add(WOLFF_STAT_CYCLES_EXPAND, c_pub - c_step);
                st.add(WOLFF_STAT_CYCLES_PUBLISH, c_end - c_pub);
            }
        }

        // ---- step (v): the record of update t
        const uint32_t b0 = sh[1];
        uint64_t ndiff = 0u, nneg = 0u;
        if (measure) {
            if (G > 1u) {
                // publish the first row / plane for the previous slab's count
                const uint32_t nb_words = (DIM == 2 ? 1u : L) * lg.RW;
                for (uint32_t w = tid; w < nb_words; w += WG) {
                    __hip_atomic_store(&a.bnd[(size_t)g * a.bnd_words + w], bits[w], __ATOMIC_RELAXED, SCOPE_AGENT);
                    st.add(WOLFF_STAT_WRITE_BYTES, 4u);
                }
                grid_barrier(ctl, G, [] {});
            }
            slab_counts<WG, DIM>(bits, lg, g, a.bnd + (size_t)gnext * a.bnd_words, ndiff, nneg, st);
        }
        uint64_t dsum = wave_sum_u64(ndiff), nsum = wave_sum_u64(nneg);
        if (lane == 0) {
            red[wv] = dsum;
            red[NW + wv] = nsum;
        }
        __syncthreads();
        if (G == 1u) {
            // one workgroup: thread 0 keeps M and B in registers and writes
            // the record; the stop request was read at the update's start
            if (tid == 0) {
                uint64_t sd = 0u, sn = 0u;
                for (int w = 0; w < NW; ++w) {
                    sd += red[w];
                    sn += red[NW + w];
                }
                M1 += (b0 ? 2ll : -2ll) * (long long)claims;          // M -= 2 s0 |C|
                if (measure) {
                    B1 = (int64_t)DIM * (int64_t)lg.N - 2 * (int64_t)sd;
                    if ((int64_t)lg.N - 2 * (int64_t)sn != M1) err1 |= ERR_MAG;
                }
                store_record(R->rec + rec0 + done, measure ? B1 : (int64_t)WOLFF_NOT_MEASURED, M1,
                             (int64_t)claims);
                st.add(WOLFF_STAT_WRITE_BYTES, 24u);
                st.add(WOLFF_STAT_READ_BYTES, 4u);                          // the stop request
                // the request word is first looked at here (the empty asm keeps
                // the compiler from testing it, and so waiting for it, earlier)
                asm volatile("" : "+v"(abort_raw));
                const bool spent = budget != 0u && wall_clock64() - t_start >= budget;
                sh[5] = (abort_raw != 0u || err1 != 0u || spent) ? 1u : 0u;
            }
        } else {
            if (tid == 0) {
                uint64_t sd = 0u, sn = 0u;
                for (int w = 0; w < NW; ++w) {
                    sd += red[w];
                    sn += red[NW + w];
                }
                if (measure) {
                    __hip_atomic_fetch_add(&ctl->acc_diff, (unsigned long long)sd, __ATOMIC_RELAXED, SCOPE_AGENT);
                    __hip_atomic_fetch_add(&ctl->acc_neg, (unsigned long long)sn, __ATOMIC_RELAXED, SCOPE_AGENT);
                    st.add(WOLFF_STAT_ATOMIC_BYTES, 16u);
                }
                if (claims) {
                    // a slab that claimed sites knows s0: M changes by -2 s0 per claim
                    const long long dm = (b0 ? 2ll : -2ll) * (long long)claims;
                    __hip_atomic_fetch_add(&ctl->acc_claims, (unsigned long long)claims, __ATOMIC_RELAXED, SCOPE_AGENT);
                    __hip_atomic_fetch_add(&ctl->acc_dm, (unsigned long long)dm, __ATOMIC_RELAXED, SCOPE_AGENT);
                    st.add(WOLFF_STAT_ATOMIC_BYTES, 16u);
                }
            }
            grid_barrier(ctl, G, [&] {
                // the last workgroup: |C|, M exactly (M -= 2 s0 |C|, summed over
                // the slabs that claimed), B and the M recount, the record, and
                // the stop request
                const unsigned long long csize = ld_agent(&ctl->acc_claims);
                const int64_t M = ctl->M + (int64_t)ld_agent(&ctl->acc_dm);
                int64_t B = ctl->B;
                if (measure) {
                    B = (int64_t)DIM * (int64_t)lg.N - 2 * (int64_t)ld_agent(&ctl->acc_diff);
                    const int64_t Mm = (int64_t)lg.N - 2 * (int64_t)ld_agent(&ctl->acc_neg);
                    if (Mm != M) ctl->err |= ERR_MAG;
                }
                ctl->M = M;
                ctl->B = B;
                store_record(R->rec + rec0 + done, measure ? B : (int64_t)WOLFF_NOT_MEASURED, M,
                             (int64_t)csize);
                st.add(WOLFF_STAT_WRITE_BYTES, 24u);
                __hip_atomic_store(&ctl->acc_diff, 0ull, __ATOMIC_RELAXED, SCOPE_AGENT);
                __hip_atomic_store(&ctl->acc_neg, 0ull, __ATOMIC_RELAXED, SCOPE_AGENT);
                __hip_atomic_store(&ctl->acc_claims, 0ull, __ATOMIC_RELAXED, SCOPE_AGENT);
                __hip_atomic_store(&ctl->acc_dm, 0ull, __ATOMIC_RELAXED, SCOPE_AGENT);
                const uint32_t failed = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, SCOPE_AGENT) != 0u;
                __hip_atomic_store(&ctl->stop, abort_requested(abort_flag) | (failed ? 1u : 0u),
                                   __ATOMIC_RELAXED, SCOPE_AGENT);
            });
            if (tid == 0) sh[5] = __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, SCOPE_AGENT);
        }
        __syncthreads();
        const uint32_t stop = sh[5];
        __syncthreads();
        if (stop) {
            ++done;
            break;
        }
    }

    // the slab back to the int8 lattice: plain +-1 bytes
    gbyte* SW = as_global(R->S);
    for (uint32_t w = tid; w < nrows * lg.RW; w += WG) {
        const uint32_t lr = w / lg.RW;
        const uint32_t x0 = (w - lr * lg.RW) * 32u;
        const uint32_t base = (r0 + lr) * L;
        const uint32_t v = bits[w];
        for (uint32_t b = 0; b < 32u && x0 + b < L; ++b) {
            const uint32_t j = base + x0 + b;
            const uint32_t addr = (DIM == 2) ? site_addr<2>(geo, j) : site_addr<3>(geo, j);
            SW[addr] = ((v >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
            st.add(WOLFF_STAT_WRITE_BYTES, 1u);
        }
    }
    st.flush(R->stats);
    if (MULTI) {
        grid_barrier(ctl, G, [&] {
            R->t = t0 + done;
            R->n_left -= done;
            R->rec_count = rec0 + done;
            R->M = ctl->M;
            R->B = ctl->B;
            if (done > 0u) R->b_valid = measure ? 1u : 0u;
            R->t_norm = t0 + done;
            R->err |= __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, SCOPE_AGENT);
            __hip_atomic_store(&ctl->err, 0u, __ATOMIC_RELAXED, SCOPE_AGENT);
        });
    } else {
        __syncthreads();                 // every thread is done with the descriptor
        if (tid == 0) {
            R->t = t0 + done;
            R->n_left -= done;
            R->rec_count = rec0 + done;
            R->M = M1;
            R->B = B1;
            if (done > 0u) R->b_valid = measure ? 1u : 0u;
            R->t_norm = t0 + done;
            R->err |= err1;
        }
        __syncthreads();
    }
}

// One lattice, on G workgroups (MULTI) or one.  Tiny frontiers run in one
// wave (TINY) on split lattices and on one-slab workgroups of up to 256
// threads, where the library puts lattices below 2^18 sites: measured on
// MI355X, 2D L = 32 (C1) 29.7 -> 24.0 us per update, 2D L = 4096 at T_c
// 7.55 -> 7.32 ms, 3D L = 256 0.294 -> 0.256 ms; on one-slab 512-thread
// workgroups (wide frontiers, 2D L = 512 and 1024) the wave path was 2-3 %
// slower, and in the batched form a C4 mix ran 14 % longer, so those leave
// it out.
template <int WG, int DIM, bool MULTI>
__global__ __launch_bounds__(WG) void lds_kernel(LdsArgs a, uint32_t max_updates)
{
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ LdsShm<WG / WAVE> shm;
    lds_body<WG, DIM, MULTI, MULTI || WG <= 256>(a, max_updates, 0u, 0u, lds, shm);
}

// Batched form of the LDS path for lattices that fit one workgroup: each
// workgroup takes replica order[blockIdx.x], then order[gridDim.x +
// atomicAdd(next)], and runs it with its lattice in LDS (geos[r]: its
// geometry) until the list or the wall-clock budget is exhausted, as the
// one-workgroup batched kernel does with the lattice in global memory.
// DIMS: 2, 3, or 0 for a list that mixes both.
template <int WG, int DIMS>
__global__ __launch_bounds__(WG) void lds_batch_kernel(Rep* reps, const LdsGeo* geos,
                                                       const uint32_t* order, uint32_t n_reps,
                                                       uint32_t* next, uint32_t max_updates,
                                                       uint32_t qmask, uint64_t budget)
{
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ LdsShm<WG / WAVE> shm;
    __shared__ uint64_t t_start_sh;
    __shared__ uint32_t idx_sh;
    if (threadIdx.x == 0) t_start_sh = wall_clock64();
    __syncthreads();
    const uint64_t t_start = t_start_sh;
    uint32_t idx = blockIdx.x;
    while (idx < n_reps) {
        const uint32_t r = __builtin_amdgcn_readfirstlane(order[idx]);
        LdsArgs a{};
        a.R = reps + r;
        a.ctl = nullptr;
        a.ov = reps[r].ov;
        a.ov_stride = 0u;
        a.qmask = qmask;
        a.lg = geos[r];
        if (DIMS == 2 || (DIMS == 0 && reps[r].dim == 2))
            lds_body<WG, 2, false, false>(a, max_updates, budget, t_start, lds, shm);
        else
            lds_body<WG, 3, false, false>(a, max_updates, budget, t_start, lds, shm);
        if (threadIdx.x == 0) {
            const bool spent = budget != 0u && wall_clock64() - t_start >= budget;
            idx_sh = spent ? n_reps : gridDim.x + atomicAdd(next, 1u);
        }
        __syncthreads();
        idx = __builtin_amdgcn_readfirstlane(idx_sh);
        __syncthreads();
    }
}

}  // namespace wolff
