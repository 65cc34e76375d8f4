/*
 * wolff.h -- C ABI of the MI355X (gfx950) Wolff single-cluster library.
 *
 * The library runs the Wolff single-cluster update of the Ising model
 * (Komura & Okabe, arXiv:1110.0899) on one GPU:
 *   H = -J sum_<ij> S_i S_j on the periodic square (dim = 2) or simple-cubic
 *   (dim = 3) lattice of linear size L (Section 2, Hamiltonian); each update
 *   picks a random seed site, grows its cluster by adding parallel
 *   neighbours with probability p = 1 - exp(-2J/T) (Section 2, steps (i)-(v);
 *   grown frontier-parallel as in Section 4, step (iii')) and flips it.
 *
 * Random numbers (the paper's LCG has unstated parameters; this library fixes
 * its own counter-based stream, so results are reproducible and independent
 * of the traversal order):
 *   Philox4x32-10 (Salmon et al., SC'11), key = (seed & 0xffffffff, seed >> 32)
 *   initial spin of site i   : +1 if word 0 of philox((i, 0, 0, 2)) < 2^31, else -1
 *   seed site of update t    : floor(((x1 << 32) | x0) * N / 2^64), x = philox((0, t, 0, 1))
 *   bond (b, mu) in update t : word mu of philox((b, t, s, 0)), s = seed site of t;
 *                              the bond joins b and b + e_mu and is active iff
 *                              the word is < thr = floor(p * 2^32) (binary64).
 *   The cluster is the connected component of s in the graph of active bonds
 *   between sites whose spin equals s0 (the seed's spin before the update).
 * Sites are numbered i = x + L*y (+ L*L*z), x fastest.
 *
 * Conventions for every call:
 *   - Return value: WOLFF_OK (0) or a negative WOLFF_E* code; no C++
 *     exception crosses this interface.  wolff_last_error() gives a message
 *     for the calling thread's most recent failure.
 *   - Host pointers are owned by the caller and only read/written during
 *     the call.  Device memory is owned by the library.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Work is enqueued on the handle's HIP stream (its own non-blocking
 *     stream unless wolff_set_stream was called); calls that return host
 *     data synchronise that stream first.
 */
#ifndef WOLFF_H
#define WOLFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define WOLFF_OK          0
#define WOLFF_EINVAL     -1   /* bad argument (dim, L, J, T, null pointer, size)   */
#define WOLFF_ENOMEM     -2   /* device or host allocation failed                   */
#define WOLFF_EDEVICE    -3   /* HIP runtime error (message in wolff_last_error)    */
#define WOLFF_ERANGE     -4   /* update index would pass 2^32 - 2                   */
#define WOLFF_ESTATE     -5   /* a device-side consistency check failed             */
#define WOLFF_EABORTED   -6   /* updates stopped on request (wolff_abort)           */

/* bond_sum value of a record taken with measurement switched off */
#define WOLFF_NOT_MEASURED INT64_MIN

/* Record of one update (Section 5, "+ measurement"): E = -J * bond_sum,
 * bond_sum = sum_i sum_mu S_i S_{i+e_mu}; mag = sum_i S_i; csize = |C|
 * (the paper's counter ic at the end of the update, seed included). */
typedef struct {
    int64_t bond_sum;
    int64_t mag;
    int64_t csize;
} wolff_record;

typedef struct {
    int32_t  dim;
    int32_t  L;
    uint64_t n_sites;        /* N = L^dim                                      */
    double   J;
    double   T;
    uint64_t seed;
    uint32_t threshold;      /* thr = floor((1 - exp(-2J/T)) * 2^32); Potts:
                                floor((1 - exp(-J/T)) * 2^32)                 */
    int32_t  path;           /* WOLFF_PATH_* the next wolff_run will use       */
    uint64_t t;              /* index of the next update                       */
    int64_t  mag;            /* magnetisation after the last update            */
    int64_t  bond_sum;       /* bond sum after the last measured update        */
    uint64_t records_pending;/* records not yet drained by wolff_observables   */
    int32_t  q;              /* 0: Ising; q >= 2: q-state Potts (wolff_create_potts) */
    int32_t  reserved;
} wolff_info;

typedef struct wolff_sim wolff_sim;

/* Create a lattice of L^dim spins, iid +-1 from `seed` (update index t = 0):
 * the problem of Section 2 (the Ising Hamiltonian with coupling J on the
 * periodic square or simple-cubic lattice of linear size L, at temperature
 * T; Section 5 runs it at the critical temperatures).
 * dim in {2, 3}; L >= 2; L^dim < 2^32; J > 0 and T > 0 finite (WOLFF_EINVAL
 * otherwise).  Allocates about 5 bytes per site of device memory (spins and
 * the overflow stack of the one-workgroup path), plus 8 bytes per site for
 * the multi-workgroup queue on the first team-path run (WOLFF_ENOMEM when
 * it does not fit).  Synchronises before returning.  *out is set only on
 * success; the handle owns all its device memory. */
int wolff_create(int dim, int L, double J, double T, uint64_t seed, wolff_sim **out);

/* Device buffers that the caller allocates (e.g. torch tensors) and keeps
 * alive until wolff_destroy; the library frees none of them. */
typedef struct {
    int8_t       *spins;          /* >= ((L^dim + 3) / 4) * 4 bytes, 16-byte aligned:
                                     the lattice in site order (x fastest), int8
                                     +1 / -1.  Between calls (once the handle's
                                     stream is idle) it holds the spins at the
                                     handle's update index. */
    uint32_t     *overflow;       /* >= 4 L^dim bytes, 4-byte aligned: the frontier
                                     overflow stack of the one-workgroup path */
    wolff_record *records;        /* record_capacity records, 8-byte aligned: the
                                     record of the k-th update since the buffer
                                     was last drained is records[k] */
    uint64_t      record_capacity;/* >= 1 */
    void         *team_queue;     /* NULL, or >= 8 L^dim bytes, 8-byte aligned: the
                                     multi-workgroup queue (NULL: the library
                                     allocates it on the first team-path run) */
    uint64_t      t0;             /* update index of the state in `spins` when
                                     WOLFF_BUFFERS_KEEP_SPINS is set */
    uint32_t      flags;          /* 0 or WOLFF_BUFFERS_KEEP_SPINS */
    uint32_t      reserved;       /* 0 */
} wolff_buffers;

/* flags: the spins buffer already holds the state (+1 / -1 bytes) at update
 * index t0; without it the library fills it iid from the seed (t = 0). */
#define WOLFF_BUFFERS_KEEP_SPINS 1u

/* wolff_create on caller-owned device buffers (the problem statement of
 * Section 2, as wolff_create).  The lattice is stored in site order in
 * `spins`, so the caller's tensor is the lattice itself.  wolff_run fails
 * with WOLFF_EINVAL when its records would not fit in the record buffer
 * beside the pending ones (drain them with wolff_observables).
 * WOLFF_EINVAL for a NULL or misaligned buffer, a record capacity of 0 or
 * unknown flags; WOLFF_ERANGE for t0 > 2^32 - 2; otherwise as wolff_create. */
int wolff_create_ex(int dim, int L, double J, double T, uint64_t seed,
                    const wolff_buffers *buffers, wolff_sim **out);

/* ------------------------------------------------ no-allocation variant */
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * updates as wolff_create_ex + wolff_set_path(WOLFF_PATH_SINGLE) +
 * wolff_set_measure(measure) + wolff_run(n_updates) + wolff_synchronize on
 * the same buffers, records and spins identical, but the call allocates
 * nothing: the lattice descriptor and the frontier overflow stack live in a
 * fixed device array of the library (about 4 MiB + 1 KiB, held by every
 * device the library runs on until the process ends).
 *   spins     device pointer, 16-byte aligned, >= L^dim bytes: the lattice in
 *             site order as int8 +1 / -1.  With WOLFF_BUFFERS_KEEP_SPINS in
 *             flags it holds the state at update index t0 on entry;
 *             otherwise it is filled iid from `seed` and t0 is ignored (the
 *             run starts at update 0).  On return it holds the state after
 *             the last update, as plain +1 / -1 bytes.
 *   records   device pointer, 8-byte aligned, >= n_updates records: the
 *             record of update k of this call is records[k] (may be NULL
 *             when n_updates is 0).
 *   measure   0: "update only" records (bond_sum = WOLFF_NOT_MEASURED).
 *   hip_stream  the stream the work is ordered on (NULL: the null stream);
 *             the call waits for it before returning.
 * L^dim must be <= WOLFF_NOALLOC_MAX_SITES (WOLFF_EINVAL otherwise, before
 * anything runs).  Every call on one device uses the same fixed array:
 * calls that overlap on a device (other threads, other streams) race and
 * must be serialised by the caller.  Ising only (no Potts).  Errors as
 * wolff_create_ex and wolff_run; WOLFF_ESTATE if a device-side check
 * failed. */
#define WOLFF_NOALLOC_MAX_SITES (1u << 20)
int wolff_run_noalloc(int dim, int L, double J, double T, uint64_t seed,
                      int8_t *spins, uint64_t t0, uint32_t flags, int measure,
                      uint64_t n_updates, wolff_record *records, void *hip_stream);

/* The q-state Potts model, H = -J sum_<ij> delta(s_i, s_j), colours
 * 0 .. q-1 (the extension Section 6 calls straightforward), 2 <= q <= 127:
 * bonds between equal colours are active with p = 1 - exp(-J/T) (the Ising
 * bond keying and threshold compare), and each cluster takes a new colour
 * uniform over the q - 1 others, drawn from word 0 of philox((0, t, 0, 3)).
 * Initial colours floor(x0 q / 2^32), x = philox((i, 0, 0, 2)).  Records:
 * bond_sum = sum over bonds of (q delta - 1), so E = -J (bond_sum + d N) / q;
 * mag = q (number of colour-0 sites) - N.  Spins are colours (int8) in
 * wolff_get_spins / wolff_set_spins.  With q = 2 and J twice the Ising J
 * the update, spins (colour 0 = +1) and records are the Ising ones.
 * Both growth paths serve Potts lattices (the team path claims a site with
 * a compare-and-swap of its colour); the bond sum is recounted over the
 * lattice after every measured update.  Otherwise as wolff_create. */
int wolff_create_potts(int dim, int L, int q, double J, double T, uint64_t seed,
                       wolff_sim **out);

/* Release the handle and its device memory (waits for its stream). NULL is
 * ok.  Buffers given to wolff_create_ex stay the caller's. */
int wolff_destroy(wolff_sim *s);

/* Enqueue n_updates Wolff updates (Section 2, steps (i)-(v), the cluster
 * grown frontier-parallel as in Section 4, step (iii')); asynchronous.
 * Appends one record per update.  WOLFF_ERANGE if t + n_updates > 2^32 - 2;
 * WOLFF_EABORTED (nothing enqueued) if a stop request from wolff_abort cut
 * earlier work short and was not yet reported. */
int wolff_run(wolff_sim *s, uint64_t n_updates);

/* Wait for the stream, then move up to `cap` pending records (the energy
 * and magnetisation measured after every update, Section 5, "+
 * measurement"), oldest first, into out[]; *n_out receives the number
 * moved.  Returns WOLFF_ESTATE if a device-side consistency check (a
 * recount of the magnetisation or of the bond sum disagreeing with the
 * tracked value) failed, WOLFF_EABORTED (after moving the records of the
 * updates that ran) if a stop request cut the work short. */
int wolff_observables(wolff_sim *s, wolff_record *out, uint64_t cap, uint64_t *n_out);

/* Wait for all work enqueued on the handle's stream (the end of step (v)
 * of Section 2 for every enqueued update).  WOLFF_EABORTED once if a stop
 * request cut the work short. */
int wolff_synchronize(wolff_sim *s);

/* Ask the updates enqueued on this handle to stop at the next update
 * boundary: the update in progress completes, the ones after it do not
 * start (a running one-workgroup launch polls the request after every
 * update, a team-path update before it starts).  Safe to call from another
 * host thread while the device works.  The state stays exact: spins, the
 * update index (the first update that did not run) and the records of the
 * updates that ran.  The next call that waits for the handle's stream
 * (wolff_synchronize, wolff_observables, wolff_get_info, wolff_get_spins,
 * wolff_set_spins, wolff_set_measure, wolff_run) clears the request and
 * returns WOLFF_EABORTED once if updates were skipped; the handle stays
 * usable.  For callers that need to end long runs early (Section 5's runs
 * of 10^4 updates per configuration). */
int wolff_abort(wolff_sim *s);

/* Current parameters (Section 2: L, d, J, T and the bond threshold of step
 * (ii)) and state (update index, the last measured E and M of Section 5);
 * synchronises.  WOLFF_EABORTED as wolff_synchronize (after filling *out). */
int wolff_get_info(wolff_sim *s, wolff_info *out);

/* Copy the N spins (int8, +-1 Ising / colours Potts, site order) of the
 * lattice after the latest update (Section 2, step (v)) to host memory; n
 * must equal N (WOLFF_EINVAL otherwise).  Synchronises. */
int wolff_get_spins(wolff_sim *s, int8_t *host, uint64_t n);

/* Replace the spins (n == N, values +-1; Potts: colours in [0, q)) and set
 * the next update index to t (checkpoint resume: the state of the Markov
 * chain of Section 2 is exactly (spins, t)).  Pending records are dropped
 * and the observables recomputed.  WOLFF_EINVAL for other values,
 * WOLFF_ERANGE for t > 2^32 - 2. */
int wolff_set_spins(wolff_sim *s, const int8_t *host, uint64_t n, uint64_t t);

/* The two columns of Section 5's Tables 1 and 2.
 * 1: bond_sum after every update (the paper's "+ measurement"): the
 * one-workgroup path updates it exactly from counts taken while the
 * cluster grows (Ising; it recounts it over the lattice every 32 updates as
 * a check); the LDS path recounts its bit lattice in LDS; the team path and
 * Potts lattices recount it over the lattice after every update; 0: "update
 * only", bond_sum = WOLFF_NOT_MEASURED.
 * mag and csize are exact in both modes.  Default 1. */
int wolff_set_measure(wolff_sim *s, int on);

/* Use the caller's HIP stream (a hipStream_t, e.g. torch's current stream)
 * for all later work; NULL returns to the handle's own stream.  Waits for
 * the previous stream first.  (Plumbing: no passage of the paper.) */
int wolff_set_stream(wolff_sim *s, void *hip_stream);

/* Growth path (the frontier-parallel growth of Section 4; Section 6 and
 * Table 3 treat small frontiers separately, as this choice does):
 * WOLFF_PATH_LDS (Ising only) keeps the lattice in LDS as one bit per spin
 * for a whole launch of many updates, split into slabs of whole rows (2D)
 * or planes (3D), one workgroup per slab (a lattice of at most 2^20 spins
 * fits one workgroup); gathers and claims are LDS accesses and only bonds
 * that cross a slab boundary go through global memory; WOLFF_EINVAL for
 * lattices it cannot hold (a row or plane above the slab size, or more than
 * 64 slabs).
 * WOLFF_PATH_SINGLE runs every update in one workgroup (LDS
 * frontier queue, one launch for many updates); WOLFF_PATH_TEAM runs each
 * update on `workgroups` cooperating workgroups (0 = library default) that
 * share an atomic-counter frontier.  WOLFF_PATH_AUTO takes the LDS path
 * for Ising lattices it holds in one or two workgroups, and for those of at
 * least 2^22 sites it holds at all; otherwise the path with the lower estimated
 * cost per update of the other two, from the mean cluster size of the
 * latest records (at most 256) returned by wolff_observables, the lattice
 * size and the measurement mode (both costs grow with the cluster's
 * breadth-first depth; one workgroup adds a cost per site and its lattice
 * recount).  Before any records are returned (and after wolff_set_spins)
 * that choice takes the single path for lattices under 2^20 sites, the
 * team path otherwise.  Every path gives the same records and spins. */
#define WOLFF_PATH_AUTO   0
#define WOLFF_PATH_SINGLE 1
#define WOLFF_PATH_TEAM   2
#define WOLFF_PATH_LDS    3
int wolff_set_path(wolff_sim *s, int path, int workgroups);

/* Workgroup size and LDS frontier ring entries of the one-workgroup path
 * (the paper's block size and shared-memory queue, Section 4; WOLFF_EINVAL
 * outside the ranges)
 * - same ranges as wolff_batch_set_tiles.  Default: 64 threads up to 4096
 * sites, 128 up to 16384, 256 below 2^20 (2048 entries), 512 from 2^20
 * sites (4096 entries). */
int wolff_set_tiles(wolff_sim *s, int wg, int queue_entries);

/* LDS-resident path (WOLFF_PATH_LDS): the most spins one workgroup holds
 * as bits in LDS (its slab of whole rows / planes); a power of two in
 * [2^10, 2^20], default 2^20.  Smaller slabs spread a lattice over more
 * workgroups (the paper's blocks, Section 4).  WOLFF_EINVAL otherwise. */
int wolff_set_lds_slab(wolff_sim *s, uint32_t slab_bits);

/* LDS-resident path: threads per workgroup (the paper's block size,
 * Section 4), 64, 128, 256, 512 or 1024; 0 restores the default (512 for
 * a lattice on several slabs; on one slab 128 for square lattices up to
 * 1024 spins, 256 up to 16384, 512 above).  WOLFF_EINVAL otherwise. */
int wolff_set_lds_tiles(wolff_sim *s, int wg);

/* Team path: replay a captured HIP graph of `chunk` updates (step (v) of
 * Section 2 repeated on the device without host launches; the seed,
 * growth and measurement launches of each) instead of launching them one by
 * one; 0 launches every kernel directly.  Default 16.  Graphs are not used
 * while kernel timing (wolff_profile) is on. */
int wolff_set_graph(wolff_sim *s, int chunk);

/* Kernel timing with HIP events on the handle's stream (the per-update
 * times of Section 5, Tables 1 and 2).  While on, every
 * launch of the cluster-growth kernel and of the measurement kernel is
 * bracketed by events; wolff_profile_read synchronises and returns the summed
 * milliseconds and launch counts since the last reset. */
int wolff_profile(wolff_sim *s, int on);
int wolff_profile_read(wolff_sim *s, double *grow_ms, uint64_t *grow_launches,
                       double *measure_ms, uint64_t *measure_launches);

/* Counting build (the library built with -DWOLFF_STATS=1, libwolff_stats.so):
 * the kernels count, per lattice, the work and the global memory accesses
 * they issue (Section 6 names the random, uncoalesced global accesses of
 * the growth as its bottleneck; these counters measure them).  Bytes are
 * those of the accesses issued (the access width times the count), not the
 * DRAM traffic, which caches reduce.  wolff_stats_read waits for the
 * handle's stream, copies min(n, WOLFF_STAT_COUNT) counters to out (summed
 * since creation or the last reset) and, with reset != 0, zeroes them.
 * WOLFF_EINVAL in the normal build. */
#define WOLFF_STAT_UPDATES         0  /* updates run                                    */
#define WOLFF_STAT_SITES           1  /* frontier sites expanded (the sum of |C|)       */
#define WOLFF_STAT_STEPS           2  /* growth steps, summed over workgroups           */
#define WOLFF_STAT_STEPS_NARROW    3  /* LDS path: steps with one lane per bond         */
#define WOLFF_STAT_NEIGHBOUR_READS 4  /* neighbour spin reads (global or LDS)           */
#define WOLFF_STAT_PHILOX          5  /* Philox4x32-10 blocks computed for live lanes   */
#define WOLFF_STAT_CLAIMS          6  /* claim operations issued                        */
#define WOLFF_STAT_READ_BYTES      7  /* global memory bytes read                       */
#define WOLFF_STAT_WRITE_BYTES     8  /* global memory bytes written                    */
#define WOLFF_STAT_ATOMIC_BYTES    9  /* global memory atomics (operand bytes)          */
#define WOLFF_STAT_MESSAGES       10  /* LDS path: messages to another slab             */
#define WOLFF_STAT_IDLE_POLLS     11  /* polls of a workgroup waiting for work          */
#define WOLFF_STAT_CYCLES_GROW    12  /* LDS path: thread-0 shader cycles in growth     */
#define WOLFF_STAT_CYCLES_IDLE    13  /* LDS path: thread-0 shader cycles polling idle  */
#define WOLFF_STAT_CYCLES_EXPAND  14  /* LDS path: thread-0 cycles from a step's start to
                                         its compaction (reads, Philox, claims)          */
#define WOLFF_STAT_CYCLES_PUBLISH 15  /* LDS path: thread-0 cycles in compaction,
                                         messages and append, end barrier included       */
#define WOLFF_STAT_STEPS_SEND     16  /* LDS path: steps that sent messages             */
#define WOLFF_STAT_CYCLES_SEND    17  /* LDS path: thread-0 cycles steps waited for
                                         their message credit to be added to the
                                         team's outstanding-work counter                */
#define WOLFF_STAT_COUNT          18
int wolff_stats_read(wolff_sim *s, uint64_t *out, int n, int reset);

/* Static description of an error code (never NULL).  (Plumbing: no
 * passage of the paper.) */
const char *wolff_strerror(int code);

/* Message of the calling thread's most recent failure ("" if none); valid
 * until that thread's next failing call.  (Plumbing.) */
const char *wolff_last_error(void);

/* ------------------------------------------------------- batched replicas */
/* Many independent lattices (any mix of dim, L, J, T, seed) advanced by one
 * persistent launch per wolff_batch_run: each workgroup takes whole replicas
 * from an atomic work counter, longest expected work first.  Every replica
 * follows exactly the stream it would follow alone through wolff_sim (each
 * runs the update of Section 2).  Section 5's studies run many (L, T)
 * points, e.g. the Binder-ratio scan of its Fig. 2, and its Section 1
 * notes that many lattices are simulated independently; this form runs
 * them in one launch.  Not a passage of the paper's method itself. */
typedef struct {
    int32_t  dim;
    int32_t  L;
    double   J;
    double   T;
    uint64_t seed;
    uint64_t n_updates;      /* updates this replica still has to run        */
    int32_t  start;          /* initial spins: 0 iid +-1 from seed (as in
                                wolff_create), +1 all up, -1 all down; Potts:
                                iid colours, all colour 0, all colour 1       */
    int32_t  flags;          /* 0, or WOLFF_JOB_UPDATE_ONLY: records carry
                                bond_sum = WOLFF_NOT_MEASURED (the paper's
                                "update only"); mag and csize stay exact      */
    int32_t  q;              /* 0: Ising; 2..127: q-state Potts (as
                                wolff_create_potts)                            */
    int32_t  reserved;       /* 0                                              */
} wolff_job;

#define WOLFF_JOB_UPDATE_ONLY 1

typedef struct wolff_batch wolff_batch;

/* Allocate and initialise n_jobs replicas (synchronises).  WOLFF_EINVAL
 * for a bad job (same rules as wolff_create) or n_jobs < 1, WOLFF_ERANGE
 * for n_updates > 2^32 - 2, WOLFF_ENOMEM when the lattices do not fit. */
int wolff_batch_create(const wolff_job *jobs, int n_jobs, wolff_batch **out);
/* Release the batch and its device memory (waits for its stream). */
int wolff_batch_destroy(wolff_batch *b);

/* Advance every replica with updates left by at most max_updates (0 = all
 * that are left) in one launch (Section 2, steps (i)-(v), per replica);
 * asynchronous. */
int wolff_batch_run(wolff_batch *b, uint64_t max_updates);

/* Pending records of replica `job` (synchronises), oldest first (Section
 * 5, "+ measurement"); WOLFF_ESTATE if a device-side check failed for it. */
int wolff_batch_records(wolff_batch *b, int job, wolff_record *out, uint64_t cap,
                        uint64_t *n_out);

/* Updates still to run for replica `job`, and its next update index. */
int wolff_batch_progress(wolff_batch *b, int job, uint64_t *left, uint64_t *t);

/* Spins of replica `job` (n must equal its N; synchronises). */
int wolff_batch_get_spins(wolff_batch *b, int job, int8_t *host, uint64_t n);

/* Measurement for every replica, as wolff_set_measure (Section 5's two
 * columns); synchronises. */
int wolff_batch_set_measure(wolff_batch *b, int on);

/* 1 (default): each wolff_batch_run replays a captured HIP graph of its
 * launches (one graph per distinct launch configuration); 0: direct launches. */
int wolff_batch_set_graph(wolff_batch *b, int on);
/* As wolff_set_stream. */
int wolff_batch_set_stream(wolff_batch *b, void *hip_stream);

/* Workgroup size / LDS queue of the batched kernel, picked by the tuner:
 * wg in {64, 128, 256, 512, 1024}, queue entries a power of two in
 * [wg, 8192] (queue and claim table, 8 entries per thread, 4 bytes each,
 * within 64 KiB of LDS); WOLFF_EINVAL otherwise. */
int wolff_batch_set_tiles(wolff_batch *b, int wg, int queue_entries);
/* Replicas of the Ising model whose lattice fits one workgroup's LDS (at
 * most 2^20 bits with rows padded to a multiple of 32: square lattices up
 * to L = 1024, simple-cubic up to L = 96) run on the LDS-resident path (as WOLFF_PATH_LDS with one slab:
 * the lattice as bits in LDS for the whole launch), in two launches by LDS
 * size that run concurrently with the one-workgroup launch of the other
 * replicas (the batched form of Section 4's frontier growth, same records).
 * on = 0 puts every replica on the one-workgroup kernel.  Default 1.
 * Takes effect at the next wolff_batch_run.  (A launch configuration, not a
 * passage of the paper.) */
int wolff_batch_set_lds(wolff_batch *b, int on);

/* Elapsed milliseconds of the last wolff_batch_run's kernel (HIP events on
 * the batch's stream; synchronises), and the number of launches it made. */
int wolff_batch_last_ms(wolff_batch *b, double *ms);

/* Counting build: the WOLFF_STAT_* counters (see wolff_stats_read) summed
 * over every replica of the batch.  WOLFF_EINVAL in the normal build. */
int wolff_batch_stats_read(wolff_batch *b, uint64_t *out, int n, int reset);

/* ------------------------------------------------------------ serving loop */
/* Serving form (not a passage of the paper: each job runs the update of
 * Section 2 and returns the records of Section 5).
 * A request loop that keeps lattices resident in HBM and advances every
 * resident job in time-bounded quanta, each one persistent launch of the
 * batched kernel (continuous batching).  Jobs are admitted first-in
 * first-out while a workgroup slot and their HBM footprint are free
 * (footprint = spins + overflow stack + records: about 5 N + 24 n_updates
 * bytes); a job submitted while others run joins the next quantum, so its
 * updates overlap with theirs on the device.  Every job's records are
 * exactly those of the same job run alone (the random stream is keyed by the
 * job's own seed and update index, never by its neighbours in the batch).
 * A finished job's records move to host memory and its HBM is released. */
typedef struct wolff_server wolff_server;

#define WOLFF_JOB_QUEUED  0
#define WOLFF_JOB_RUNNING 1
#define WOLFF_JOB_DONE    2
#define WOLFF_JOB_FAILED  3   /* a device consistency check failed for the job */

typedef struct {
    uint64_t queued;         /* submitted, not admitted                     */
    uint64_t running;        /* resident on the device                      */
    uint64_t done;           /* finished, records not yet taken             */
    uint64_t slots;          /* most jobs resident at once                  */
    uint64_t resident_bytes; /* HBM held by resident jobs                   */
    uint64_t budget_bytes;   /* HBM admission budget                        */
    uint64_t quanta;         /* launches so far                             */
    uint64_t updates;        /* updates completed over all jobs             */
    uint64_t added_spins;    /* sum of cluster sizes over those updates     */
    double   gpu_ms;         /* summed kernel time of the quanta            */
} wolff_server_stats;

/* hbm_budget_bytes: admission budget (0 = 80 % of the free device memory);
 * max_slots: most resident jobs (0 = workgroups resident at once). */
int wolff_server_create(uint64_t hbm_budget_bytes, int max_slots, wolff_server **out);
int wolff_server_destroy(wolff_server *srv);

/* Queue a job (start and flags as in wolff_job); *job_id identifies it.
 * WOLFF_EINVAL for bad parameters or a footprint above the whole budget. */
int wolff_server_submit(wolff_server *srv, const wolff_job *job, uint64_t *job_id);

/* One scheduling iteration: admit queued jobs that fit, run one quantum of
 * about quantum_ms (every resident job advances by whole updates until the
 * quantum is spent or it finishes), retire finished jobs.  Synchronous.
 * *n_finished receives the number of jobs that finished in this step. */
int wolff_server_step(wolff_server *srv, double quantum_ms, uint64_t *n_finished);

/* Run each quantum's jobs that fit one workgroup's LDS (Ising, at most 2^20
 * bits with rows padded to 32) on the batched LDS path, as
 * wolff_batch_set_lds does for a batch (as many as are resident at once;
 * the rest and every other job on the one-workgroup kernel); on = 0: all
 * on the one-workgroup kernel.  Default 1.  Records are the same either
 * way.  (A launch configuration, not a passage of the paper.) */
int wolff_server_set_lds(wolff_server *srv, int on);

/* State (WOLFF_JOB_*) and updates done of one job. */
int wolff_server_status(wolff_server *srv, uint64_t job_id, int *state, uint64_t *updates_done);

/* Ids of jobs finished since the previous call (up to cap). */
int wolff_server_finished(wolff_server *srv, uint64_t *ids, uint64_t cap, uint64_t *n_out);

/* Records of a finished job (oldest first, up to cap); the job is forgotten
 * once all its records have been taken. */
int wolff_server_take(wolff_server *srv, uint64_t job_id, wolff_record *out, uint64_t cap,
                      uint64_t *n_out);

int wolff_server_get_stats(wolff_server *srv, wolff_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* WOLFF_H */
