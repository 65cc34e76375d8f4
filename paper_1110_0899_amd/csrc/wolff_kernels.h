// gfx950 kernels of the Wolff single-cluster update.
//
// Two growth paths share the bond keying and the per-site neighbour logic:
//  * one workgroup per lattice (batch_kernel): the frontier lives in an LDS
//    ring (spilling to a global overflow stack when it outgrows it); the
//    workgroup runs every update of its lattice inside one launch.  Because
//    no other workgroup touches the lattice during the launch, claims are
//    settled in an LDS hash table and written with plain byte stores.  The
//    same kernel runs one replica (single lattices) or thousands (the batched
//    form and the serving loop), Ising or q-state Potts.
//  * a team of workgroups per lattice (team_kernel, one launch per update):
//    each workgroup expands from its own LDS queue and trades work through a
//    tagged global queue with atomic head/tail counters and a pending count
//    that decides termination; claims are agent-scope atomics (Ising: an
//    OR/AND on the spin's word, Potts: a compare-and-swap of the colour).
#pragma once

#include "wolff_device.h"
#include "../../include/wolff.h"

namespace wolff {

// Per-lattice descriptor in device memory, read at the start of a launch and
// written back at its end.
struct Rep {
    int8_t* S;              // spins, N bytes (allocation padded to a multiple of 4)
    uint32_t* ov;           // overflow stack of the one-workgroup path, N entries
    wolff_record* rec;      // record array
    uint64_t rec_count;     // records written so far
    Geo geo;
    int32_t dim;
    uint32_t thr;           // floor(p * 2^32)
    uint32_t k0, k1;        // Philox key
    uint32_t t;             // next update index
    uint32_t n_left;        // updates still to run
    uint32_t measure;       // 1: bond sum in every record
    uint32_t err;           // error bits (ERR_*)
    uint32_t t_norm;        // no member tag in S is older than update t_norm
    uint32_t b_valid;       // 1: B holds the bond sum of the current lattice
    uint32_t q;             // 0: Ising (+-1 bytes); q >= 2: q-state Potts (colour bytes)
    uint32_t pad_q;
    int64_t M;              // magnetisation after the last update
    int64_t B;              // bond sum (valid when b_valid)
    const uint32_t* abort;  // host-mapped stop request, read once per update (NULL: none)
    unsigned long long* stats;  // counting build: WOLFF_STAT_COUNT counters (NULL: none)
};

// Per-update control block of the team path.
struct TeamCtl {
    uint32_t head;          // next global queue slot to hand out
    uint32_t tail;          // global queue slots reserved by producers
    int32_t pending;        // sites claimed but not yet expanded, all workgroups
    uint32_t exited;        // workgroups done with this update
    uint32_t epoch;         // tag of this update's queue entries (never 0)
    uint32_t s;             // seed site
    int32_t s0;             // seed spin (Ising) or colour (Potts) before the update
    int32_t cb;             // Potts: the cluster's new colour
    unsigned long long csize;
    long long acc_diff;     // measurement: differing bonds (Potts: equal bonds)
    long long acc_neg;      // measurement: negative spins (Potts: colour-0 sites)
    uint32_t blocks_done;
    uint32_t aborted;       // 1: the update was not started (stop request seen)
};

}  // namespace wolff
