// Host runtime and C ABI of libwolff (declared in include/wolff.h).
// One translation unit: the kernels are included so that the launch sites
// below see their definitions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "wolff_kernels.hip"
#include "wolff_lds.hip"

using wolff::Geo;
using wolff::Rep;
using wolff::TeamCtl;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            return fail(e_ == hipErrorOutOfMemory ? WOLFF_ENOMEM : WOLFF_EDEVICE,       \
                        std::string(#expr) + ": " + hipGetErrorString(e_));             \
        }                                                                               \
    } while (0)

// Every fill and copy of a handle's device memory is ordered on the handle's
// stream.  The library's own streams are non-blocking: they do not wait for
// work on the null stream, so a hipMemset / hipMemcpy issued there could
// land after a kernel that the handle's stream runs later.  Copies that
// return host data (or read host data) wait for the stream before returning.
static hipError_t copy_wait(hipStream_t st, void* dst, const void* src, size_t bytes,
                            hipMemcpyKind kind)
{
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

extern "C" const char* wolff_strerror(int code)
{
    switch (code) {
    case WOLFF_OK: return "ok";
    case WOLFF_EINVAL: return "invalid argument";
    case WOLFF_ENOMEM: return "out of memory";
    case WOLFF_EDEVICE: return "HIP runtime error";
    case WOLFF_ERANGE: return "update index out of range";
    case WOLFF_ESTATE: return "device consistency check failed";
    case WOLFF_EABORTED: return "stopped on request";
    default: return "unknown error";
    }
}

extern "C" const char* wolff_last_error(void) { return g_last_error.c_str(); }

static std::string err_message(uint32_t bits)
{
    std::string m;
    if (bits & wolff::ERR_MAG) m += "magnetisation recount disagrees with the cluster sizes; ";
    if (bits & wolff::ERR_TEAM_WAIT) m += "a multi-workgroup wait passed its bound; ";
    if (bits & wolff::ERR_BOND) m += "bond-sum recount disagrees with the tracked value; ";
    if (m.empty()) m = "device error flag set";
    return m;
}

// -------------------------------------------------------------- parameters
// thr = floor(p * 2^32) in binary64 with p = 1 - exp(-2J/T) (Ising, Section
// 2, step (ii)) or p = 1 - exp(-J/T) (q-state Potts, q > 0).
static uint32_t bond_threshold(double J, double T, int q = 0)
{
    const double p = 1.0 - std::exp(-(q ? 1.0 : 2.0) * J / T);
    const double scaled = std::ldexp(p, 32);
    if (!(scaled > 0.0)) return 0u;
    if (scaled >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)std::floor(scaled);
}

static bool valid_q(int q) { return q == 0 || (q >= 2 && q <= 127); }

// Byte of a uniform start: Ising +1 / -1, Potts colour 0 / colour 1.
static int start_byte(int q, int start) { return q ? (start > 0 ? 0x00 : 0x01) : (start > 0 ? 0x01 : 0xFF); }

static wolff::Div make_div(uint32_t d)
{
    wolff::Div v;
    if ((d & (d - 1u)) == 0u) {
        uint32_t sh = 0;
        while ((1u << sh) < d) ++sh;
        v.shift = sh;
        v.magic_hi = v.magic_lo = 0u;
    } else {
        v.shift = 0xFFFFFFFFu;
        const uint64_t M = UINT64_MAX / d + 1u;     // floor(2^64 / d) + 1
        v.magic_hi = (uint32_t)(M >> 32);
        v.magic_lo = (uint32_t)M;
    }
    return v;
}

// Geometry; storage is tiled (128-site tiles) when L is a multiple of 16.
static Geo make_geo(int dim, uint32_t L)
{
    Geo g{};
    g.L = L;
    g.LL = L * L;
    g.N = (dim == 2) ? g.LL : g.LL * L;
    g.dL = make_div(L);
    g.tiled = (L % 16u == 0u) ? 1u : 0u;
    if (g.tiled) {
        g.ntx = L / 16u;
        g.nty = (dim == 2) ? L / 8u : L / 4u;
        g.ntz = (dim == 2) ? 1u : L / 2u;
    } else {
        g.ntx = g.nty = g.ntz = 1u;
    }
    g.dntx = make_div(g.ntx);
    g.dnty = make_div(g.nty);
    return g;
}

// Geometry of a lattice stored in site order (no tiles), for lattices in a
// caller's buffer.
static Geo make_site_order_geo(int dim, uint32_t L)
{
    Geo g = make_geo(dim, L);
    g.tiled = 0u;
    g.ntx = g.nty = g.ntz = 1u;
    g.dntx = make_div(1u);
    g.dnty = make_div(1u);
    return g;
}

// Storage address of logical site i (host copy of the device mapping).
static uint64_t host_site_addr(const Geo& g, int dim, uint64_t i)
{
    if (!g.tiled) return i;
    const uint64_t L = g.L;
    const uint64_t x = i % L, y = (i / L) % L, z = i / (L * L);
    if (dim == 2) return ((((y >> 3) * g.ntx + (x >> 4)) << 7) | ((y & 7u) << 4) | (x & 15u));
    return (((((z >> 1) * g.nty + (y >> 2)) * g.ntx + (x >> 4)) << 7) | ((z & 1u) << 6) |
            ((y & 3u) << 4) | (x & 15u));
}

// Device spins (storage order) -> host spins (site order), and back.
// Ising bytes may carry member tags; bit 1 is the sign of every byte.
// Potts bytes (q > 0) are the colours.
static int copy_spins_out(hipStream_t st, const Geo& g, int dim, const int8_t* dev, int8_t* host,
                          uint64_t n, int q = 0)
{
    if (!g.tiled) {
        HIP_TRY(copy_wait(st, host, dev, n, hipMemcpyDeviceToHost));
        if (!q)
            for (uint64_t i = 0; i < n; ++i) host[i] = (host[i] & 2) ? -1 : 1;
        return WOLFF_OK;
    }
    std::vector<int8_t> tmp(n);
    HIP_TRY(copy_wait(st, tmp.data(), dev, n, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
        const int8_t b = tmp[host_site_addr(g, dim, i)];
        host[i] = q ? b : ((b & 2) ? -1 : 1);
    }
    return WOLFF_OK;
}

static int copy_spins_in(hipStream_t st, const Geo& g, int dim, const int8_t* host, int8_t* dev,
                         uint64_t n)
{
    if (!g.tiled) {
        HIP_TRY(copy_wait(st, dev, host, n, hipMemcpyHostToDevice));
        return WOLFF_OK;
    }
    std::vector<int8_t> tmp(n);
    for (uint64_t i = 0; i < n; ++i) tmp[host_site_addr(g, dim, i)] = host[i];
    HIP_TRY(copy_wait(st, dev, tmp.data(), n, hipMemcpyHostToDevice));
    return WOLFF_OK;
}

static int check_params(int dim, int L, double J, double T, uint64_t* N)
{
    if (dim != 2 && dim != 3) return fail(WOLFF_EINVAL, "dim must be 2 or 3");
    if (L < 2) return fail(WOLFF_EINVAL, "L must be >= 2");
    if (!(std::isfinite(J) && J > 0.0)) return fail(WOLFF_EINVAL, "J must be finite and > 0");
    if (!(std::isfinite(T) && T > 0.0)) return fail(WOLFF_EINVAL, "T must be finite and > 0");
    uint64_t n = 1;
    for (int a = 0; a < dim; ++a) {
        n *= (uint64_t)L;
        if (n >= (1ull << 32)) return fail(WOLFF_EINVAL, "L^dim must be < 2^32");
    }
    *N = n;
    return WOLFF_OK;
}

static constexpr uint64_t T_LIMIT = 0xFFFFFFFEull;   // t + 1 must fit the 32-bit counter word

static uint64_t padded_bytes(uint64_t N) { return (N + 255u) & ~uint64_t(255); }

// -------------------------------------------------------- kernel dispatch
static int g_num_cus = 0;

static int device_cus()
{
    if (g_num_cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            g_num_cus = prop.multiProcessorCount;
        if (g_num_cus <= 0) g_num_cus = 256;
    }
    return g_num_cus;
}

using BatchFn = void (*)(Rep*, const uint32_t*, uint32_t, uint32_t*, uint32_t, uint32_t, uint64_t);

// Dynamic LDS of the batched kernel: frontier ring + claim table.
static size_t batch_lds_bytes(int wg, uint32_t qentries)
{
    return ((size_t)qentries + wolff::tab_entries(wg)) * sizeof(uint32_t);
}

// Batched kernel for a workgroup size and a dimension (2, 3, or 0 for a
// batch that mixes both; the single-dimension variants need fewer registers).
static BatchFn batch_fn(int wg, int dims)
{
#define WOLFF_PICK(W)                                                                   \
    return dims == 2 ? wolff::batch_kernel<W, 2> : dims == 3 ? wolff::batch_kernel<W, 3> \
                                                             : wolff::batch_kernel<W, 0>
    switch (wg) {
    case 64: WOLFF_PICK(64);
    case 128: WOLFF_PICK(128);
    case 512: WOLFF_PICK(512);
    case 1024: WOLFF_PICK(1024);
    default: WOLFF_PICK(256);
    }
#undef WOLFF_PICK
}

static hipError_t launch_batch(int wg, int dims, uint32_t grid, uint32_t qentries, hipStream_t st,
                               Rep* reps, const uint32_t* order, uint32_t n, uint32_t* next,
                               uint32_t max_updates, uint64_t budget = 0)
{
    const size_t lds = batch_lds_bytes(wg, qentries);
    const uint32_t qmask = qentries - 1u;
    hipLaunchKernelGGL(wolff::reset_counter_kernel, dim3(1), dim3(64), 0, st, next);
    hipLaunchKernelGGL(batch_fn(wg, dims), dim3(grid), dim3(wg), lds, st, reps, order, n, next,
                       max_updates, qmask, budget);
    return hipGetLastError();
}

// Workgroups of the batched kernel resident at once on the device.
static int batch_occupancy(int wg, int dims, int qentries)
{
    int per_cu = 0;
    const size_t lds = batch_lds_bytes(wg, (uint32_t)qentries);
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(batch_fn(wg, dims)), wg, lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu * device_cus();
}

// Workgroup sizes 64..1024 (powers of two); ring entries a power of two in
// [wg, 8192]; the ring and the claim table within 64 KiB of LDS.
static bool valid_tiles(int wg, int q)
{
    if (wg != 64 && wg != 128 && wg != 256 && wg != 512 && wg != 1024) return false;
    if (q < wg || q > 8192 || (q & (q - 1)) != 0) return false;
    return batch_lds_bytes(wg, (uint32_t)q) <= 65536;
}

// ====================================================================== sim
struct EventPair {
    hipEvent_t a, b;
};

struct wolff_sim {
    int dim = 2;
    int L = 0;
    int q = 0;                            // 0: Ising; q >= 2: q-state Potts
    uint64_t N = 0;
    double J = 1.0, T = 1.0;
    uint64_t seed = 0;
    uint32_t thr = 0;
    Geo geo{};

    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;

    // caller-owned device buffers (wolff_create_ex): the library frees none
    // of S, ov, d_rec, and gq when the caller supplied it
    bool ext_buffers = false;
    bool ext_queue = false;
    // stop request: a word of pinned host memory mapped into the device's
    // address space (abort_host on the host side, abort_dev on the device side)
    uint32_t* abort_host = nullptr;
    uint32_t* abort_dev = nullptr;

    int8_t* S = nullptr;
    uint32_t* ov = nullptr;
    unsigned long long* gq = nullptr;
    Rep* d_rep = nullptr;
    uint32_t* d_order = nullptr;
    uint32_t* d_next = nullptr;
    TeamCtl* d_ctl = nullptr;
    wolff_record* d_rec = nullptr;
    uint64_t rec_cap = 0;
    uint64_t rec_written = 0;    // records the device has been asked to write
    uint64_t rec_read = 0;

    uint64_t t = 0;
    int measure = 1;
    bool tagged = false;                  // S may hold member tags of the one-workgroup path
    int path = WOLFF_PATH_AUTO;
    double csize_mean = -1.0;             // mean |C| of the latest records returned (-1: none yet)
    int team_wgs = 0;
    int single_wg = 256;
    int single_q = 2048;

    // LDS-resident path: team state, inboxes, boundary rows, overflow stacks
    // (allocated on the first run on this path)
    wolff::LdsCtl* lctl = nullptr;
    unsigned long long* linbox = nullptr;
    uint32_t* ltail = nullptr;
    uint32_t* lbnd = nullptr;
    uint32_t* lov = nullptr;
    size_t lbytes_inbox = 0, lbytes_tail = 0;
    uint32_t lds_slab_bits = 1u << 20;    // most spins of one workgroup's slab
    int lds_wg = 0;                       // LDS-path workgroup size (0: by lattice size)

    int graph_chunk = 16;                 // updates per captured graph (0 = no graphs)
    hipGraphExec_t graph = nullptr;       // team-path chunk of graph_chunk updates
    int graph_key[3] = {-1, -1, -1};      // (chunk, measure, team size) it was captured with
    hipStream_t graph_stream = nullptr;

    unsigned long long* d_stats = nullptr;   // counting build: WOLFF_STAT_COUNT counters

    bool profiling = false;
    std::vector<EventPair> ev_grow, ev_meas, ev_free;
    double grow_ms = 0.0, meas_ms = 0.0;
    uint64_t grow_n = 0, meas_n = 0;
};

// WOLFF_PATH_AUTO compares the cost per update of the two growth paths,
// estimated from the mean cluster size c of the latest records returned.
// Both are latency-bound by the cluster's breadth-first depth (one step, or
// one device-wide round trip, per level), modelled as a power of c: on the
// team path it is the whole cost; one workgroup takes about half as long
// per level but also adds only ~250 (2D) or ~200 (3D) sites per
// microsecond, and pays for its lattice recount (every 32 measured updates
// with the incremental bond sum (Ising); every measured update
// otherwise).  The constants are fits to MI355X timings of both paths, at
// their default tiles, at the critical points (square lattices
// L = 512 ... 4096, simple-cubic L = 64 ... 256, mean clusters from 4e3 to
// 2.6e6 sites; within about 10 % of the fit, 20 % at 3D L = 64).
static double depth_us(int dim, double c)
{
    c = std::max(c, 1.0);
    return dim == 2 ? 4.2 * std::pow(c, 0.555) : 9.4 * std::pow(c, 0.4);
}

static double single_cost_us(const wolff_sim* s)
{
    double recount = 0.0;
    if (s->measure) {
        const bool incremental = !s->q;
        recount = incremental ? (double)s->N / (32.0 * 5000.0)
                              : (double)s->N / (s->dim == 2 ? 11000.0 : 6000.0);
    }
    const double rate = s->dim == 2 ? 250.0 : 200.0;       // sites per microsecond
    return 13.0 + 0.5 * depth_us(s->dim, s->csize_mean) + s->csize_mean / rate + recount;
}

static double team_cost_us(const wolff_sim* s)
{
    return 15.0 + depth_us(s->dim, s->csize_mean) + (s->measure ? 8.0 + (double)s->N / 1e6 : 0.0);
}

// ----------------------------------------------------- LDS-resident path
// Slabs of at most LDS_SLAB_BITS bits (128 KiB) per workgroup, whole rows
// (2D) or whole planes (3D), as few slabs as fit; at most LDS_MAX_SLABS
// workgroups, all resident at once.  The ring of LDS_RING entries follows
// the slab in LDS.
static constexpr uint32_t LDS_SLAB_BITS = 1u << 20;
static constexpr uint32_t LDS_RING = 2048;
static constexpr uint32_t LDS_MAX_SLABS = 64;

struct LdsPlan {
    wolff::LdsGeo lg;
    int wg;
    uint32_t imask;         // entries of one message ring - 1
    uint32_t bnd_words;
    uint32_t ov_stride;
    size_t lds_bytes;
};

static bool lds_plan(int dim, uint32_t L, uint32_t slab_bits, LdsPlan* out)
{
    wolff::LdsGeo lg{};
    lg.L = L;
    lg.N = dim == 2 ? L * L : L * L * L;
    lg.RW = (L + 31u) / 32u;
    lg.Lp = 32u * lg.RW;
    lg.rows = dim == 2 ? L : L * L;
    const uint64_t unit_bits = (uint64_t)lg.Lp * (dim == 2 ? 1u : L);   // a row or a plane
    if (unit_bits > slab_bits) return false;
    const uint32_t per_slab = (uint32_t)std::min<uint64_t>(L, slab_bits / unit_bits);
    const uint32_t G = (L + per_slab - 1u) / per_slab;
    if (G > LDS_MAX_SLABS) return false;
    const uint32_t units = (L + G - 1u) / G;                      // balanced slabs
    lg.G = (L + units - 1u) / units;
    lg.slab_rows = units * (dim == 2 ? 1u : L);
    lg.slab_words = lg.slab_rows * lg.RW;
    lg.dL = make_div(L);
    lg.dslab = make_div(lg.slab_rows);
    LdsPlan p{};
    p.lg = lg;
    const uint64_t N = lg.N;
    // measured on MI355X at the critical points: 512 threads per slab for a
    // split lattice (2D L = 4096: 10.0 ms per update against 11.2 with 256,
    // 10.5 with 1024; 3D L = 256: 0.34 ms against 0.41); one slab: 128 for
    // square lattices up to 1024 spins (2D L = 32: 24.4 us, 24.7 with 256,
    // 29 with 64), 256 up to 16384 (2D L = 45, 64: 36, 55 us against 38, 61
    // with 128; 3D L = 12, 16: 16, 22 us against 18, 27), 512 above (2D
    // L = 181, 256, 512, 1024: 0.19, 0.27, 0.64, 1.56 ms against 0.21,
    // 0.30, 0.73, 1.79 with 256; 3D L = 32, 40: 47, 65 us against 51, 75)
    p.wg = lg.G > 1u ? 512 : (dim == 2 && N <= 1024) ? 128 : N <= 16384 ? 256 : 512;
    // a message ring carries the bonds across one slab boundary in one
    // direction, each at most once per update: L^(d-1) entries
    uint32_t cap = 64u;
    const uint64_t need = dim == 2 ? L : (uint64_t)L * L;
    while (cap < need) cap <<= 1;
    p.imask = cap - 1u;
    p.bnd_words = (dim == 2 ? 1u : L) * lg.RW;
    p.ov_stride = lg.slab_rows * L;
    p.lds_bytes = ((size_t)((lg.slab_words + 3u) & ~3u) + LDS_RING) * sizeof(uint32_t);
    *out = p;
    return true;
}

using LdsFn = void (*)(wolff::LdsArgs, uint32_t);

// The LDS-path kernel for a workgroup size, a dimension and a slab count
// (one slab: the single-workgroup instance).
static LdsFn lds_fn(int wg, int dim, uint32_t G)
{
#define WOLFF_PICK_LDS(W)                                                               \
    if (G > 1u) return dim == 2 ? wolff::lds_kernel<W, 2, true> : wolff::lds_kernel<W, 3, true>; \
    return dim == 2 ? wolff::lds_kernel<W, 2, false> : wolff::lds_kernel<W, 3, false>
    switch (wg) {
    case 64: WOLFF_PICK_LDS(64);
    case 128: WOLFF_PICK_LDS(128);
    case 512: WOLFF_PICK_LDS(512);
    case 1024: WOLFF_PICK_LDS(1024);
    default: WOLFF_PICK_LDS(256);
    }
#undef WOLFF_PICK_LDS
}

static bool lds_fits(const wolff_sim* s)
{
    LdsPlan p;
    return s->q == 0 && lds_plan(s->dim, (uint32_t)s->L, s->lds_slab_bits, &p) &&
           (int)p.lg.G <= device_cus();
}

// Ising lattices the LDS path holds in one or two workgroups, or in more
// when the lattice has at least 2^22 sites: there it was the fastest path
// at every measured size and temperature window on MI355X (square lattices
// L = 32 ... 4096, simple-cubic L = 32 ... 256 at their critical points;
// simple-cubic L = 128 on two slabs 0.275 against 0.294 ms per update on
// one workgroup).  Lattices below 2^22 sites split into more slabs (a
// lowered slab size) stay with the cost model below.
static bool lds_preferred(const wolff_sim* s)
{
    LdsPlan p;
    if (!lds_fits(s) || !lds_plan(s->dim, (uint32_t)s->L, s->lds_slab_bits, &p)) return false;
    return p.lg.G <= 2u || s->N >= (1ull << 22);
}

static int resolved_path(const wolff_sim* s)
{
    if (s->path != WOLFF_PATH_AUTO) return s->path;
    if (lds_preferred(s)) return WOLFF_PATH_LDS;
    if (s->csize_mean < 0.0)      // no records yet: by lattice size
        return s->N < (1ull << 20) ? WOLFF_PATH_SINGLE : WOLFF_PATH_TEAM;
    return single_cost_us(s) <= team_cost_us(s) ? WOLFF_PATH_SINGLE : WOLFF_PATH_TEAM;
}

static int team_size(const wolff_sim* s)
{
    if (s->team_wgs > 0) return s->team_wgs;
    return std::max(8, device_cus() / 4);
}

static void free_lds(wolff_sim* s);

static void free_sim(wolff_sim* s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto* v : {&s->ev_grow, &s->ev_meas, &s->ev_free})
        for (auto& e : *v) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    if (!s->ext_buffers) {
        if (s->S) (void)hipFree(s->S);
        if (s->ov) (void)hipFree(s->ov);
        if (s->d_rec) (void)hipFree(s->d_rec);
    }
    if (s->gq && !s->ext_queue) (void)hipFree(s->gq);
    if (s->d_rep) (void)hipFree(s->d_rep);
    if (s->d_order) (void)hipFree(s->d_order);
    if (s->d_next) (void)hipFree(s->d_next);
    if (s->d_ctl) (void)hipFree(s->d_ctl);
    if (s->d_stats) (void)hipFree(s->d_stats);
    free_lds(s);
    if (s->abort_host) (void)hipHostFree(s->abort_host);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    delete s;
}

static int get_event_pair(wolff_sim* s, EventPair* out)
{
    if (!s->ev_free.empty()) {
        *out = s->ev_free.back();
        s->ev_free.pop_back();
        return WOLFF_OK;
    }
    HIP_TRY(hipEventCreate(&out->a));
    HIP_TRY(hipEventCreate(&out->b));
    return WOLFF_OK;
}

static int harvest_events(wolff_sim* s)
{
    for (int which = 0; which < 2; ++which) {
        auto& v = which == 0 ? s->ev_grow : s->ev_meas;
        for (auto& e : v) {
            float ms = 0.0f;
            HIP_TRY(hipEventSynchronize(e.b));
            HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
            if (which == 0) {
                s->grow_ms += ms;
                s->grow_n += 1;
            } else {
                s->meas_ms += ms;
                s->meas_n += 1;
            }
            s->ev_free.push_back(e);
        }
        v.clear();
    }
    return WOLFF_OK;
}

// Copy the host-side fields of the descriptor (stream must be idle).
static int push_rep(wolff_sim* s, const Rep& r)
{
    HIP_TRY(copy_wait(s->stream, s->d_rep, &r, sizeof(Rep), hipMemcpyHostToDevice));
    return WOLFF_OK;
}

static int pull_rep(wolff_sim* s, Rep* r)
{
    HIP_TRY(copy_wait(s->stream, r, s->d_rep, sizeof(Rep), hipMemcpyDeviceToHost));
    return WOLFF_OK;
}

// After the stream has drained: if a stop request is pending, clear it and,
// when it stopped updates, take the update index and the record count from
// the device (the updates that ran are exact; the rest never started).
// Returns WOLFF_EABORTED once for a request that stopped updates.
static int settle_abort(wolff_sim* s, const Rep& r)
{
    if (__atomic_load_n(s->abort_host, __ATOMIC_ACQUIRE) == 0u) return WOLFF_OK;
    __atomic_store_n(s->abort_host, 0u, __ATOMIC_RELEASE);
    if ((uint64_t)r.t == s->t) return WOLFF_OK;           // everything had run already
    const uint64_t skipped = s->t - (uint64_t)r.t;
    s->t = r.t;
    s->rec_written = r.rec_count;
    return fail(WOLFF_EABORTED, "stopped on request: " + std::to_string(skipped) +
                                    " enqueued updates did not run");
}

// pull_rep, then settle a pending stop request.  *stopped receives the
// result of settle_abort (WOLFF_OK or WOLFF_EABORTED).
static int pull_rep_settled(wolff_sim* s, Rep* r, int* stopped)
{
    int rc = pull_rep(s, r);
    if (rc) return rc;
    *stopped = settle_abort(s, *r);
    return WOLFF_OK;
}

static int measure_now(wolff_sim* s)
{
    hipLaunchKernelGGL(wolff::measure_rep_kernel<1024>, dim3(1), dim3(1024), 0, s->stream, s->d_rep);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));
    return WOLFF_OK;
}

static int create_sim(int dim, int L, int q, double J, double T, uint64_t seed,
                      const wolff_buffers* ext, wolff_sim** out)
{
    if (!out) return fail(WOLFF_EINVAL, "out is NULL");
    if (!valid_q(q)) return fail(WOLFF_EINVAL, "q must be 2..127 (or 0 for Ising)");
    uint64_t N = 0;
    int rc = check_params(dim, L, J, T, &N);
    if (rc) return rc;
    if (ext) {
        if (!ext->spins || !ext->overflow || !ext->records)
            return fail(WOLFF_EINVAL, "wolff_buffers: spins, overflow and records are required");
        if (ext->record_capacity < 1) return fail(WOLFF_EINVAL, "wolff_buffers: record_capacity < 1");
        if ((ext->flags & ~(uint32_t)WOLFF_BUFFERS_KEEP_SPINS) != 0u)
            return fail(WOLFF_EINVAL, "wolff_buffers: unknown flags");
        if (ext->t0 > T_LIMIT) return fail(WOLFF_ERANGE, "wolff_buffers: t0 exceeds 2^32 - 2");
        if ((uintptr_t)ext->spins % 16u || (uintptr_t)ext->overflow % 4u ||
            (uintptr_t)ext->records % 8u || (uintptr_t)ext->team_queue % 8u)
            return fail(WOLFF_EINVAL, "wolff_buffers: misaligned buffer (spins need 16-byte, "
                                      "overflow 4-byte, records and team_queue 8-byte alignment)");
    }
    wolff_sim* s = new (std::nothrow) wolff_sim();
    if (!s) return fail(WOLFF_ENOMEM, "host allocation failed");
    s->dim = dim;
    s->L = L;
    s->q = q;
    s->N = N;
    s->J = J;
    s->T = T;
    s->seed = seed;
    s->thr = bond_threshold(J, T, q);
    // one-workgroup path: small lattices have frontiers of a few sites per
    // step, where fewer waves per barrier shorten the step; from 2^20 sites
    // the frontiers of critical clusters fill 512 threads (measured on
    // MI355X: 64 threads best up to 4096 sites, 128 up to 16384, 256 below
    // 2^20, then 512 with a 4096-entry ring: -6 % per update at 2D L = 1024,
    // -35 % at L = 4096, -24 % at 3D L = 256)
    s->single_wg = N <= 4096 ? 64 : N <= 16384 ? 128 : N < (1ull << 20) ? 256 : 512;
    s->single_q = N < (1ull << 20) ? 2048 : 4096;
    // a caller's lattice is in site order; the library's own is tiled when
    // L is a multiple of 16
    s->geo = ext ? make_site_order_geo(dim, (uint32_t)L) : make_geo(dim, (uint32_t)L);
    const uint64_t t0 = (ext && (ext->flags & WOLFF_BUFFERS_KEEP_SPINS)) ? ext->t0 : 0u;

#define CREATE_TRY(expr)                                                                \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            int code_ = e_ == hipErrorOutOfMemory ? WOLFF_ENOMEM : WOLFF_EDEVICE;       \
            free_sim(s);                                                                \
            return fail(code_, std::string(#expr) + ": " + hipGetErrorString(e_));      \
        }                                                                               \
    } while (0)

    CREATE_TRY(hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking));
    s->stream = s->own_stream;
    CREATE_TRY(hipHostMalloc((void**)&s->abort_host, sizeof(uint32_t),
                             hipHostMallocMapped | hipHostMallocCoherent));
    *s->abort_host = 0u;
    CREATE_TRY(hipHostGetDevicePointer((void**)&s->abort_dev, s->abort_host, 0));
    if (ext) {
        s->ext_buffers = true;
        s->S = ext->spins;
        s->ov = ext->overflow;
        s->d_rec = ext->records;
        s->rec_cap = ext->record_capacity;
        if (ext->team_queue) {
            s->ext_queue = true;
            s->gq = reinterpret_cast<unsigned long long*>(ext->team_queue);
            CREATE_TRY(hipMemsetAsync(s->gq, 0, N * sizeof(unsigned long long), s->stream));
        }
    } else {
        CREATE_TRY(hipMalloc(&s->S, padded_bytes(N)));
        CREATE_TRY(hipMemsetAsync(s->S, 0, padded_bytes(N), s->stream));
        CREATE_TRY(hipMalloc(&s->ov, N * sizeof(uint32_t)));
        s->rec_cap = 1024;
        CREATE_TRY(hipMalloc(&s->d_rec, s->rec_cap * sizeof(wolff_record)));
    }
    CREATE_TRY(hipMalloc(&s->d_rep, sizeof(Rep)));
    CREATE_TRY(hipMalloc(&s->d_order, sizeof(uint32_t)));
    CREATE_TRY(hipMalloc(&s->d_next, sizeof(uint32_t)));
    CREATE_TRY(hipMalloc(&s->d_ctl, sizeof(TeamCtl)));
    CREATE_TRY(hipMemsetAsync(s->d_ctl, 0, sizeof(TeamCtl), s->stream));
    CREATE_TRY(hipMemsetAsync(s->d_order, 0, sizeof(uint32_t), s->stream));
    if (WOLFF_STATS) {
        CREATE_TRY(hipMalloc(&s->d_stats, WOLFF_STAT_COUNT * sizeof(unsigned long long)));
        CREATE_TRY(hipMemsetAsync(s->d_stats, 0, WOLFF_STAT_COUNT * sizeof(unsigned long long), s->stream));
    }

    if (!(ext && (ext->flags & WOLFF_BUFFERS_KEEP_SPINS))) {
        hipLaunchKernelGGL(wolff::init_kernel, dim3(std::min<uint64_t>((N + 255) / 256, 65536)),
                           dim3(256), 0, s->stream, s->S, s->geo, dim, (uint32_t)seed,
                           (uint32_t)(seed >> 32), (uint32_t)q);
        CREATE_TRY(hipGetLastError());
    }

    Rep r{};
    r.q = (uint32_t)q;
    r.S = s->S;
    r.ov = s->ov;
    r.rec = s->d_rec;
    r.rec_count = 0;
    r.geo = s->geo;
    r.dim = dim;
    r.thr = s->thr;
    r.k0 = (uint32_t)seed;
    r.k1 = (uint32_t)(seed >> 32);
    r.t = (uint32_t)t0;
    r.t_norm = (uint32_t)t0;
    r.n_left = 0xFFFFFFFFu;
    r.measure = 1;
    r.err = 0;
    r.abort = s->abort_dev;
    r.stats = s->d_stats;
    s->t = t0;
    CREATE_TRY(copy_wait(s->stream, s->d_rep, &r, sizeof(Rep), hipMemcpyHostToDevice));
    if ((rc = measure_now(s)) != WOLFF_OK) {
        free_sim(s);
        return rc;
    }
#undef CREATE_TRY
    *out = s;
    return WOLFF_OK;
}

extern "C" int wolff_create(int dim, int L, double J, double T, uint64_t seed, wolff_sim** out)
{
    return create_sim(dim, L, 0, J, T, seed, nullptr, out);
}

extern "C" int wolff_create_potts(int dim, int L, int q, double J, double T, uint64_t seed,
                                  wolff_sim** out)
{
    if (q == 0) return fail(WOLFF_EINVAL, "q must be 2..127");
    return create_sim(dim, L, q, J, T, seed, nullptr, out);
}

extern "C" int wolff_create_ex(int dim, int L, double J, double T, uint64_t seed,
                               const wolff_buffers* ext, wolff_sim** out)
{
    if (!ext) return fail(WOLFF_EINVAL, "wolff_buffers is NULL");
    return create_sim(dim, L, 0, J, T, seed, ext, out);
}

extern "C" int wolff_destroy(wolff_sim* s)
{
    free_sim(s);
    return WOLFF_OK;
}

// Make room for n more records on the device (synchronises if it grows).
static int reserve_records(wolff_sim* s, uint64_t n)
{
    const uint64_t need = s->rec_written + n;
    if (need <= s->rec_cap) return WOLFF_OK;
    if (s->ext_buffers)
        return fail(WOLFF_EINVAL, "the caller's record buffer holds " + std::to_string(s->rec_cap) +
                                      " records and " + std::to_string(s->rec_written - s->rec_read) +
                                      " are pending: drain them with wolff_observables");
    uint64_t cap = s->rec_cap;
    while (cap < need) cap *= 2;
    {   // the device's record count is the truth if a stop request cut work short
        Rep cur;
        int stopped = WOLFF_OK;
        int rc0 = pull_rep_settled(s, &cur, &stopped);
        if (rc0) return rc0;
        if (stopped) return stopped;
    }
    wolff_record* nrec = nullptr;
    HIP_TRY(hipMalloc(&nrec, cap * sizeof(wolff_record)));
    const uint64_t live = s->rec_written - s->rec_read;
    if (live) {
        const hipError_t e = copy_wait(s->stream, nrec, s->d_rec + s->rec_read,
                                       live * sizeof(wolff_record), hipMemcpyDeviceToDevice);
        if (e != hipSuccess) {   // the old buffer and its records stay in place
            (void)hipFree(nrec);
            return fail(WOLFF_EDEVICE, std::string("record buffer copy: ") + hipGetErrorString(e));
        }
    }
    HIP_TRY(hipFree(s->d_rec));
    s->d_rec = nrec;
    s->rec_cap = cap;
    s->rec_written = live;
    s->rec_read = 0;
    Rep r;
    int rc = pull_rep(s, &r);
    if (rc) return rc;
    r.rec = nrec;
    r.rec_count = live;
    return push_rep(s, r);
}

static int ensure_team_queue(wolff_sim* s)
{
    if (s->gq) return WOLFF_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    unsigned long long* q = nullptr;
    HIP_TRY(hipMalloc(&q, s->N * sizeof(unsigned long long)));
    const hipError_t e = hipMemsetAsync(q, 0, s->N * sizeof(unsigned long long), s->stream);
    if (e != hipSuccess) {       // kept only once zeroed: a later call must not find it half set up
        (void)hipFree(q);
        return fail(WOLFF_EDEVICE, std::string("team queue fill: ") + hipGetErrorString(e));
    }
    s->gq = q;
    return WOLFF_OK;
}

static void free_lds(wolff_sim* s)
{
    for (void* p : {(void*)s->lctl, (void*)s->linbox, (void*)s->ltail, (void*)s->lbnd, (void*)s->lov})
        if (p) (void)hipFree(p);
    s->lctl = nullptr;
    s->linbox = nullptr;
    s->ltail = nullptr;
    s->lbnd = nullptr;
    s->lov = nullptr;
}

// Team state of the LDS-resident path: allocated and zeroed on first use;
// zeroed again whenever the update index is set (the inbox entries carry
// the update index as their tag, so older entries must not survive a
// rewind).
static int lds_reset(wolff_sim* s)
{
    if (!s->lctl) return WOLFF_OK;
    HIP_TRY(hipMemsetAsync(s->lctl, 0, sizeof(wolff::LdsCtl), s->stream));
    HIP_TRY(hipMemsetAsync(s->linbox, 0, s->lbytes_inbox, s->stream));
    HIP_TRY(hipMemsetAsync(s->ltail, 0, s->lbytes_tail, s->stream));
    return WOLFF_OK;
}

static int alloc_lds(wolff_sim* s, const LdsPlan& p)
{
    const uint32_t G = p.lg.G;
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->lbytes_inbox = 2u * (size_t)G * (p.imask + 1u) * sizeof(unsigned long long);
    s->lbytes_tail = 2u * (size_t)G * sizeof(uint32_t);
    HIP_TRY(hipMalloc(&s->lctl, sizeof(wolff::LdsCtl)));
    HIP_TRY(hipMalloc(&s->linbox, s->lbytes_inbox));
    HIP_TRY(hipMalloc(&s->ltail, s->lbytes_tail));
    HIP_TRY(hipMalloc(&s->lbnd, (size_t)G * p.bnd_words * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&s->lov, (size_t)G * p.ov_stride * sizeof(uint32_t)));
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(lds_fn(p.wg, s->dim, p.lg.G)),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes));
    return lds_reset(s);
}

// The buffers are kept only when all of them were set up: a later call
// takes a non-null control block as "ready".
static int ensure_lds(wolff_sim* s, const LdsPlan& p)
{
    if (s->lctl) return WOLFF_OK;
    const int rc = alloc_lds(s, p);
    if (rc) free_lds(s);
    return rc;
}

static int run_lds(wolff_sim* s, uint64_t n)
{
    LdsPlan p;
    if (!lds_plan(s->dim, (uint32_t)s->L, s->lds_slab_bits, &p))
        return fail(WOLFF_EINVAL, "lattice too large for the LDS path");
    if (s->lds_wg) p.wg = s->lds_wg;
    int rc = ensure_lds(s, p);
    if (rc) return rc;
    wolff::LdsArgs a{};
    a.R = s->d_rep;
    a.ctl = s->lctl;
    a.inbox = s->linbox;
    a.inbox_tail = s->ltail;
    a.imask = p.imask;
    a.bnd = s->lbnd;
    a.bnd_words = p.bnd_words;
    a.ov = s->lov;
    a.ov_stride = p.ov_stride;
    a.qmask = LDS_RING - 1u;
    a.lg = p.lg;
    // launches of about 2^27 sites of work (the expected clusters plus the
    // slab load and write-back), at most 65536 updates
    const double cl = s->csize_mean >= 0.0 ? s->csize_mean : (double)s->N;
    const double work = cl + (double)s->N / 64.0 + 64.0;
    const uint64_t chunk = (uint64_t)std::max(1.0, std::min(65536.0, (double)(1ull << 27) / work));
    const LdsFn fn = lds_fn(p.wg, s->dim, p.lg.G);
    for (uint64_t done = 0; done < n;) {
        const uint32_t m = (uint32_t)std::min<uint64_t>(chunk, n - done);
        EventPair ev{};
        if (s->profiling) {
            if ((rc = get_event_pair(s, &ev))) return rc;
            HIP_TRY(hipEventRecord(ev.a, s->stream));
        }
        hipLaunchKernelGGL(fn, dim3(p.lg.G), dim3(p.wg), p.lds_bytes, s->stream, a, m);
        HIP_TRY(hipGetLastError());
        if (s->profiling) {
            HIP_TRY(hipEventRecord(ev.b, s->stream));
            s->ev_grow.push_back(ev);
        }
        done += m;
    }
    s->tagged = false;                 // the slabs are written back as plain +-1 bytes
    return WOLFF_OK;
}

static int run_team_update(wolff_sim* s)
{
    const int G = team_size(s);
    constexpr int WG = 256;
    const uint32_t qentries = 2048;
    const uint32_t keep = 2 * WG;
    EventPair ev{};
    hipLaunchKernelGGL(wolff::team_seed_kernel, dim3(1), dim3(64), 0, s->stream, s->d_rep, s->d_ctl, s->gq);
    if (s->profiling) {
        int rc = get_event_pair(s, &ev);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ev.a, s->stream));
    }
    if (s->dim == 2)
        hipLaunchKernelGGL((wolff::team_kernel<WG, 2>), dim3(G), dim3(WG), qentries * sizeof(uint32_t),
                           s->stream, s->d_rep, s->d_ctl, s->gq, qentries - 1u, keep);
    else
        hipLaunchKernelGGL((wolff::team_kernel<WG, 3>), dim3(G), dim3(WG), qentries * sizeof(uint32_t),
                           s->stream, s->d_rep, s->d_ctl, s->gq, qentries - 1u, keep);
    HIP_TRY(hipGetLastError());
    if (s->profiling) {
        HIP_TRY(hipEventRecord(ev.b, s->stream));
        s->ev_grow.push_back(ev);
    }
    if (s->measure) {
        EventPair em{};
        if (s->profiling) {
            int rc = get_event_pair(s, &em);
            if (rc) return rc;
            HIP_TRY(hipEventRecord(em.a, s->stream));
        }
        // a few blocks per CU, each thread loops over its chunks: the per-block
        // atomics of the final reduction stay few
        const uint64_t items = ((s->L & 15) == 0) ? s->N / 16 : s->N;
        const uint32_t blocks = (uint32_t)std::max<uint64_t>(
            1, std::min<uint64_t>((items + 1023) / 1024, (uint64_t)device_cus() * 2));
        if (s->dim == 2)
            hipLaunchKernelGGL(wolff::measure_grid_kernel<2>, dim3(blocks), dim3(256), 0, s->stream, s->d_rep, s->d_ctl);
        else
            hipLaunchKernelGGL(wolff::measure_grid_kernel<3>, dim3(blocks), dim3(256), 0, s->stream, s->d_rep, s->d_ctl);
        HIP_TRY(hipGetLastError());
        if (s->profiling) {
            HIP_TRY(hipEventRecord(em.b, s->stream));
            s->ev_meas.push_back(em);
        }
    }
    return WOLFF_OK;
}

static int ensure_team_graph(wolff_sim* s)
{
    const int key[3] = {s->graph_chunk, s->measure, team_size(s)};
    if (s->graph && s->graph_stream == s->stream && key[0] == s->graph_key[0] &&
        key[1] == s->graph_key[1] && key[2] == s->graph_key[2])
        return WOLFF_OK;
    if (s->graph) {
        HIP_TRY(hipStreamSynchronize(s->stream));
        HIP_TRY(hipGraphExecDestroy(s->graph));
        s->graph = nullptr;
    }
    HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed));
    int rc = WOLFF_OK;
    for (int u = 0; u < s->graph_chunk && rc == WOLFF_OK; ++u) rc = run_team_update(s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    HIP_TRY(e);
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(ei);
    s->graph = x;
    s->graph_stream = s->stream;
    for (int i = 0; i < 3; ++i) s->graph_key[i] = key[i];
    return WOLFF_OK;
}

extern "C" int wolff_set_tiles(wolff_sim* s, int wg, int queue_entries)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    if (!valid_tiles(wg, queue_entries)) return fail(WOLFF_EINVAL, "unsupported tile sizes");
    s->single_wg = wg;
    s->single_q = queue_entries;
    return WOLFF_OK;
}

extern "C" int wolff_set_lds_slab(wolff_sim* s, uint32_t slab_bits)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    if (slab_bits < 1024u || slab_bits > LDS_SLAB_BITS || (slab_bits & (slab_bits - 1u)) != 0u)
        return fail(WOLFF_EINVAL, "slab_bits must be a power of two in [2^10, 2^20]");
    if (slab_bits == s->lds_slab_bits) return WOLFF_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    free_lds(s);                               // sizes follow the slab count
    s->lds_slab_bits = slab_bits;
    if (s->path == WOLFF_PATH_LDS && !lds_fits(s)) s->path = WOLFF_PATH_AUTO;
    return WOLFF_OK;
}

extern "C" int wolff_set_lds_tiles(wolff_sim* s, int wg)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    if (wg != 0 && wg != 64 && wg != 128 && wg != 256 && wg != 512 && wg != 1024)
        return fail(WOLFF_EINVAL, "wg must be 0, 64, 128, 256, 512 or 1024");
    if (wg == s->lds_wg) return WOLFF_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    free_lds(s);                               // the kernel's LDS attribute is set on first use
    s->lds_wg = wg;
    return WOLFF_OK;
}

extern "C" int wolff_set_graph(wolff_sim* s, int chunk)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    if (chunk < 0 || chunk > 4096) return fail(WOLFF_EINVAL, "chunk must be in [0, 4096]");
    s->graph_chunk = chunk;
    return WOLFF_OK;
}

extern "C" int wolff_run(wolff_sim* s, uint64_t n)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    if (n == 0) return WOLFF_OK;
    if (s->t + n > T_LIMIT) return fail(WOLFF_ERANGE, "t + n_updates exceeds 2^32 - 2");
    int rc;
    if (__atomic_load_n(s->abort_host, __ATOMIC_ACQUIRE) != 0u) {
        // a stop request is pending: settle it before enqueueing anything
        Rep cur;
        int stopped = WOLFF_OK;
        if ((rc = pull_rep_settled(s, &cur, &stopped))) return rc;
        if (stopped) return stopped;
    }
    if ((rc = reserve_records(s, n))) return rc;
    const int path = resolved_path(s);
    if (path == WOLFF_PATH_LDS) {
        if ((rc = run_lds(s, n))) return rc;
    } else if (path == WOLFF_PATH_TEAM) {
        if ((rc = ensure_team_queue(s))) return rc;
        if (s->tagged) {
            // the team path reads plain bytes: drop the one-workgroup path's tags
            const uint32_t nw = (uint32_t)((s->N + 3) / 4);
            hipLaunchKernelGGL(wolff::plain_kernel, dim3(std::min<uint32_t>((nw + 255) / 256, 4096)),
                               dim3(256), 0, s->stream, s->S, (uint32_t)s->N);
            HIP_TRY(hipGetLastError());
            s->tagged = false;
        }
        uint64_t u = 0;
        const uint64_t chunk = (uint64_t)s->graph_chunk;
        if (!s->profiling && chunk > 0 && n >= chunk) {
            // the three launches of `chunk` updates, captured once and replayed;
            // every kernel argument is a device pointer whose contents carry
            // the state, so one graph serves every later chunk
            if ((rc = ensure_team_graph(s))) return rc;
            for (; u + chunk <= n; u += chunk) HIP_TRY(hipGraphLaunch(s->graph, s->stream));
        }
        for (; u < n; ++u)
            if ((rc = run_team_update(s))) return rc;
    } else {
        if (s->measure && !s->q) s->tagged = true;   // measured Ising updates leave member tags
        // one workgroup runs the updates; chunk so that one launch stays short
        // (about 2^26 sites of work: the expected cluster, plus the lattice
        // recount every 32 measured updates), at most 65536 updates
        const double cl = s->csize_mean >= 0.0 ? s->csize_mean : (double)s->N;
        const double work = cl + (s->measure ? (double)s->N / 32.0 : 0.0) + 64.0;
        const uint64_t chunk = (uint64_t)std::max(1.0, std::min(65536.0, (double)(1ull << 26) / work));
        for (uint64_t done = 0; done < n;) {
            const uint32_t m = (uint32_t)std::min<uint64_t>(chunk, n - done);
            EventPair ev{};
            if (s->profiling) {
                if ((rc = get_event_pair(s, &ev))) return rc;
                HIP_TRY(hipEventRecord(ev.a, s->stream));
            }
            HIP_TRY(launch_batch(s->single_wg, s->dim, 1, (uint32_t)s->single_q, s->stream, s->d_rep,
                                 s->d_order, 1, s->d_next, m));
            if (s->profiling) {
                HIP_TRY(hipEventRecord(ev.b, s->stream));
                s->ev_grow.push_back(ev);
            }
            done += m;
        }
        if (s->ext_buffers && s->tagged) {
            // the caller's lattice holds plain +-1 bytes between calls
            const uint32_t nw = (uint32_t)((s->N + 3) / 4);
            hipLaunchKernelGGL(wolff::plain_kernel, dim3(std::min<uint32_t>((nw + 255) / 256, 4096)),
                               dim3(256), 0, s->stream, s->S, (uint32_t)s->N);
            HIP_TRY(hipGetLastError());
            s->tagged = false;
        }
    }
    s->t += n;
    s->rec_written += n;
    return WOLFF_OK;
}

extern "C" int wolff_synchronize(wolff_sim* s)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (__atomic_load_n(s->abort_host, __ATOMIC_ACQUIRE) == 0u) return WOLFF_OK;
    Rep r;
    int stopped = WOLFF_OK;
    int rc = pull_rep_settled(s, &r, &stopped);
    return rc ? rc : stopped;
}

extern "C" int wolff_abort(wolff_sim* s)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    __atomic_store_n(s->abort_host, 1u, __ATOMIC_RELEASE);
    return WOLFF_OK;
}

extern "C" int wolff_observables(wolff_sim* s, wolff_record* out, uint64_t cap, uint64_t* n_out)
{
    if (!s || (!out && cap > 0)) return fail(WOLFF_EINVAL, "NULL argument");
    Rep r;
    int stopped = WOLFF_OK;
    int rc = pull_rep_settled(s, &r, &stopped);
    if (rc) return rc;
    const uint64_t live = s->rec_written - s->rec_read;
    const uint64_t k = std::min(cap, live);
    if (k) {
        HIP_TRY(copy_wait(s->stream, out, s->d_rec + s->rec_read, k * sizeof(wolff_record),
                          hipMemcpyDeviceToHost));
        // the latest records (at most 256) steer WOLFF_PATH_AUTO: a long
        // thermalisation series from an ordered start would otherwise carry
        // its first, lattice-sized clusters into the estimate
        const uint64_t from = k > 256 ? k - 256 : 0;
        double sum = 0.0;
        for (uint64_t i = from; i < k; ++i) sum += (double)out[i].csize;
        s->csize_mean = sum / (double)(k - from);
    }
    s->rec_read += k;
    if (n_out) *n_out = k;
    bool push = false;
    if (s->rec_read == s->rec_written) {
        s->rec_read = s->rec_written = 0;
        r.rec_count = 0;
        push = true;
    }
    const uint32_t bad_bits = r.err;
    const bool bad = bad_bits != 0u;
    if (bad) {
        r.err = 0u;
        push = true;
    }
    if (push && (rc = push_rep(s, r))) return rc;
    if (bad) return fail(WOLFF_ESTATE, err_message(bad_bits));
    if (stopped) return fail(WOLFF_EABORTED, "stopped on request; the records of the updates "
                                             "that ran were returned");
    return WOLFF_OK;
}

extern "C" int wolff_get_info(wolff_sim* s, wolff_info* out)
{
    if (!s || !out) return fail(WOLFF_EINVAL, "NULL argument");
    Rep r;
    int stopped = WOLFF_OK;
    int rc = pull_rep_settled(s, &r, &stopped);
    if (rc) return rc;
    out->dim = s->dim;
    out->L = s->L;
    out->n_sites = s->N;
    out->J = s->J;
    out->T = s->T;
    out->seed = s->seed;
    out->threshold = s->thr;
    out->path = resolved_path(s);
    out->q = s->q;
    out->reserved = 0;
    out->t = r.t;
    out->mag = r.M;
    out->bond_sum = r.B;
    out->records_pending = s->rec_written - s->rec_read;
    return stopped;
}

extern "C" int wolff_get_spins(wolff_sim* s, int8_t* host, uint64_t n)
{
    if (!s || !host) return fail(WOLFF_EINVAL, "NULL argument");
    if (n != s->N) return fail(WOLFF_EINVAL, "n must equal the number of sites");
    int rc = copy_spins_out(s->stream, s->geo, s->dim, s->S, host, n, s->q);
    if (rc || __atomic_load_n(s->abort_host, __ATOMIC_ACQUIRE) == 0u) return rc;
    Rep r;
    int stopped = WOLFF_OK;
    rc = pull_rep_settled(s, &r, &stopped);
    return rc ? rc : stopped;
}

extern "C" int wolff_set_spins(wolff_sim* s, const int8_t* host, uint64_t n, uint64_t t)
{
    if (!s || !host) return fail(WOLFF_EINVAL, "NULL argument");
    if (n != s->N) return fail(WOLFF_EINVAL, "n must equal the number of sites");
    if (t > T_LIMIT) return fail(WOLFF_ERANGE, "t exceeds 2^32 - 2");
    if (s->q) {
        for (uint64_t i = 0; i < n; ++i)
            if (host[i] < 0 || host[i] >= s->q) return fail(WOLFF_EINVAL, "colours must be in [0, q)");
    } else {
        for (uint64_t i = 0; i < n; ++i)
            if (host[i] != 1 && host[i] != -1) return fail(WOLFF_EINVAL, "spins must be +1 or -1");
    }
    Rep r;
    int stopped = WOLFF_OK;
    int rc = pull_rep_settled(s, &r, &stopped);
    if (rc) return rc;
    if ((rc = copy_spins_in(s->stream, s->geo, s->dim, host, s->S, n))) return rc;
    r.t = (uint32_t)t;
    r.t_norm = (uint32_t)t;
    r.rec_count = 0;
    s->tagged = false;
    s->csize_mean = -1.0;
    r.err = 0;
    s->t = t;
    s->rec_read = s->rec_written = 0;
    if ((rc = push_rep(s, r))) return rc;
    if ((rc = lds_reset(s))) return rc;
    if ((rc = measure_now(s))) return rc;
    return stopped;
}

extern "C" int wolff_set_measure(wolff_sim* s, int on)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    Rep r;
    int stopped = WOLFF_OK;
    int rc = pull_rep_settled(s, &r, &stopped);
    if (rc) return rc;
    s->measure = on ? 1 : 0;
    r.measure = (uint32_t)s->measure;
    if ((rc = push_rep(s, r))) return rc;
    return stopped;
}

extern "C" int wolff_set_stream(wolff_sim* s, void* hip_stream)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->stream = hip_stream ? (hipStream_t)hip_stream : s->own_stream;
    return WOLFF_OK;
}

extern "C" int wolff_set_path(wolff_sim* s, int path, int workgroups)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    if (path != WOLFF_PATH_AUTO && path != WOLFF_PATH_SINGLE && path != WOLFF_PATH_TEAM &&
        path != WOLFF_PATH_LDS)
        return fail(WOLFF_EINVAL, "unknown path");
    if (path == WOLFF_PATH_LDS && !lds_fits(s))
        return fail(WOLFF_EINVAL, "the LDS path takes Ising lattices whose slabs fit the device "
                                  "(rows or planes of at most 2^20 bits, at most 64 slabs)");
    if (workgroups < 0 || workgroups > 65536) return fail(WOLFF_EINVAL, "bad workgroup count");
    s->path = path;
    s->team_wgs = workgroups;
    return WOLFF_OK;
}

extern "C" int wolff_profile(wolff_sim* s, int on)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    int rc = harvest_events(s);
    if (rc) return rc;
    s->profiling = on != 0;
    s->grow_ms = s->meas_ms = 0.0;
    s->grow_n = s->meas_n = 0;
    return WOLFF_OK;
}

extern "C" int wolff_profile_read(wolff_sim* s, double* grow_ms, uint64_t* grow_launches,
                                  double* measure_ms, uint64_t* measure_launches)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    int rc = harvest_events(s);
    if (rc) return rc;
    if (grow_ms) *grow_ms = s->grow_ms;
    if (grow_launches) *grow_launches = s->grow_n;
    if (measure_ms) *measure_ms = s->meas_ms;
    if (measure_launches) *measure_launches = s->meas_n;
    return WOLFF_OK;
}

// Counters of a counting build (all zero and WOLFF_EINVAL otherwise).
static int read_stats(hipStream_t st, unsigned long long* d, uint64_t* out, int n, int reset)
{
    if (!WOLFF_STATS || d == nullptr)
        return fail(WOLFF_EINVAL, "the library was built without WOLFF_STATS (libwolff_stats.so counts)");
    if (!out || n < 0) return fail(WOLFF_EINVAL, "bad output buffer");
    unsigned long long h[WOLFF_STAT_COUNT];
    HIP_TRY(copy_wait(st, h, d, sizeof(h), hipMemcpyDeviceToHost));
    for (int i = 0; i < n && i < WOLFF_STAT_COUNT; ++i) out[i] = h[i];
    if (reset) {
        HIP_TRY(hipMemsetAsync(d, 0, sizeof(h), st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return WOLFF_OK;
}

extern "C" int wolff_stats_read(wolff_sim* s, uint64_t* out, int n, int reset)
{
    if (!s) return fail(WOLFF_EINVAL, "sim is NULL");
    return read_stats(s->stream, s->d_stats, out, n, reset);
}

// ==================================================================== batch
// One LDS class of a batch: replicas (longest expected work first), the
// kernel's workgroup size and dimension variant, and its LDS bytes.
struct BatchLdsClass {
    std::vector<uint32_t> order;
    uint32_t* d_order = nullptr;
    int wg = 256;
    int dims = 0;
    size_t lds_bytes = 0;
};

// LDS classes of the batched LDS path: slabs of at most 8 KiB (square
// lattices up to L = 256, simple-cubic up to L = 32; 256-thread
// workgroups, several per CU) and the rest of the one-workgroup lattices
// (up to 128 KiB, 512-thread workgroups, one per CU: the mixed replica
// set's heaviest replicas are square L = 512 near T = 2).  -1: not on the
// LDS path (Potts, or more than 2^20 spins).
static constexpr uint32_t BATCH_LDS_RING = 2048;
static int batch_lds_class(const wolff_job& j, wolff::LdsGeo* geo)
{
    if (j.q != 0) return -1;
    LdsPlan p;
    if (!lds_plan(j.dim, (uint32_t)j.L, LDS_SLAB_BITS, &p) || p.lg.G != 1u) return -1;
    *geo = p.lg;
    return p.lg.slab_words <= 2048u ? 0 : 1;
}

static size_t batch_lds_bytes_for(const wolff::LdsGeo& g)
{
    return ((size_t)((g.slab_words + 3u) & ~3u) + BATCH_LDS_RING) * sizeof(uint32_t);
}

using LdsBatchFn = void (*)(Rep*, const wolff::LdsGeo*, const uint32_t*, uint32_t, uint32_t*, uint32_t,
                            uint32_t, uint64_t);

static LdsBatchFn lds_batch_fn(int wg, int dims)
{
#define WOLFF_PICK_LB(W)                                                                \
    return dims == 2 ? wolff::lds_batch_kernel<W, 2>                                     \
                     : dims == 3 ? wolff::lds_batch_kernel<W, 3> : wolff::lds_batch_kernel<W, 0>
    if (wg == 512) { WOLFF_PICK_LB(512); }
    WOLFF_PICK_LB(256);
#undef WOLFF_PICK_LB
}

struct wolff_batch {
    std::vector<wolff_job> jobs;
    std::vector<Rep> reps;          // host copy (pointers, geometry, parameters)
    std::vector<uint64_t> left;     // host mirror of updates left
    std::vector<uint64_t> t;        // host mirror of next update index
    std::vector<uint64_t> rec_read; // records drained per replica
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    int8_t* S = nullptr;            // one slab for all lattices
    uint32_t* ov = nullptr;
    wolff_record* rec = nullptr;
    std::vector<uint64_t> S_off, ov_off, rec_off;
    Rep* d_reps = nullptr;
    uint32_t* d_order = nullptr;
    uint32_t* d_next = nullptr;
    std::vector<uint32_t> order;    // longest expected work first
    int wg = 256;
    int qentries = 2048;
    int dims = 0;                   // 2 or 3 if every replica has that dimension, else 0
    int measure = 1;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    bool timed = false;
    bool use_graph = true;
    // captured (counter reset + persistent launch), keyed by its launch arguments
    std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
    // Ising replicas whose lattice fits one workgroup's LDS run on the LDS
    // path (lds_batch_kernel) in two classes by LDS size; the others (and
    // all of them when use_lds is off) on the one-workgroup kernel above.
    // The classes run as concurrent launches forked from the batch stream.
    bool use_lds = true;
    wolff::LdsGeo* d_geos = nullptr;
    std::vector<uint32_t> order_glob;            // replicas outside the LDS classes
    uint32_t* d_order_glob = nullptr;
    int dims_glob = 0;
    BatchLdsClass lcls[2];
    uint32_t* d_next_aux = nullptr;              // work counters: [0] global class, [1..2] LDS classes
    hipStream_t aux[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
    unsigned long long* d_stats = nullptr;      // counting build: summed over the replicas
};

static void free_batch(wolff_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (hipStream_t st : b->aux)
        if (st) (void)hipStreamSynchronize(st);
    if (b->d_geos) (void)hipFree(b->d_geos);
    if (b->d_stats) (void)hipFree(b->d_stats);
    if (b->d_order_glob) (void)hipFree(b->d_order_glob);
    for (auto& c : b->lcls)
        if (c.d_order) (void)hipFree(c.d_order);
    if (b->d_next_aux) (void)hipFree(b->d_next_aux);
    for (hipStream_t st : b->aux)
        if (st) (void)hipStreamDestroy(st);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipEvent_t e : b->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (b->S) (void)hipFree(b->S);
    if (b->ov) (void)hipFree(b->ov);
    if (b->rec) (void)hipFree(b->rec);
    if (b->d_reps) (void)hipFree(b->d_reps);
    if (b->d_order) (void)hipFree(b->d_order);
    if (b->d_next) (void)hipFree(b->d_next);
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    if (b->ev_a) (void)hipEventDestroy(b->ev_a);
    if (b->ev_b) (void)hipEventDestroy(b->ev_b);
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
    delete b;
}

extern "C" int wolff_batch_create(const wolff_job* jobs, int n_jobs, wolff_batch** out)
{
    if (!jobs || n_jobs <= 0 || !out) return fail(WOLFF_EINVAL, "bad job list");
    wolff_batch* b = new (std::nothrow) wolff_batch();
    if (!b) return fail(WOLFF_ENOMEM, "host allocation failed");
#define BATCH_TRY(expr)                                                                 \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            int code_ = e_ == hipErrorOutOfMemory ? WOLFF_ENOMEM : WOLFF_EDEVICE;       \
            free_batch(b);                                                              \
            return fail(code_, std::string(#expr) + ": " + hipGetErrorString(e_));      \
        }                                                                               \
    } while (0)
    uint64_t s_total = 0, ov_total = 0, rec_total = 0;
    std::vector<uint64_t> Ns(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        uint64_t N = 0;
        int rc = check_params(jobs[i].dim, jobs[i].L, jobs[i].J, jobs[i].T, &N);
        if (rc) {
            free_batch(b);
            return fail(rc, "job " + std::to_string(i) + ": " + g_last_error);
        }
        if (jobs[i].start < -1 || jobs[i].start > 1 || (jobs[i].flags & ~WOLFF_JOB_UPDATE_ONLY) != 0 ||
            !valid_q(jobs[i].q)) {
            free_batch(b);
            return fail(WOLFF_EINVAL, "job " + std::to_string(i) + ": bad start, flags or q field");
        }
        if (jobs[i].n_updates > T_LIMIT) {
            free_batch(b);
            return fail(WOLFF_ERANGE, "job " + std::to_string(i) + ": too many updates");
        }
        Ns[i] = N;
        b->S_off.push_back(s_total);
        b->ov_off.push_back(ov_total);
        b->rec_off.push_back(rec_total);
        s_total += padded_bytes(N);
        ov_total += N;
        rec_total += std::max<uint64_t>(jobs[i].n_updates, 1);
    }
    b->jobs.assign(jobs, jobs + n_jobs);
    b->dims = jobs[0].dim;
    for (int i = 1; i < n_jobs; ++i)
        if (jobs[i].dim != b->dims) b->dims = 0;
    BATCH_TRY(hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking));
    b->stream = b->own_stream;
    BATCH_TRY(hipMalloc(&b->S, s_total));
    BATCH_TRY(hipMemsetAsync(b->S, 0, s_total, b->stream));
    BATCH_TRY(hipMalloc(&b->ov, ov_total * sizeof(uint32_t)));
    BATCH_TRY(hipMalloc(&b->rec, rec_total * sizeof(wolff_record)));
    BATCH_TRY(hipMalloc(&b->d_reps, n_jobs * sizeof(Rep)));
    BATCH_TRY(hipMalloc(&b->d_order, n_jobs * sizeof(uint32_t)));
    BATCH_TRY(hipMalloc(&b->d_next, sizeof(uint32_t)));
    BATCH_TRY(hipEventCreate(&b->ev_a));
    BATCH_TRY(hipEventCreate(&b->ev_b));
    if (WOLFF_STATS) {
        BATCH_TRY(hipMalloc(&b->d_stats, WOLFF_STAT_COUNT * sizeof(unsigned long long)));
        BATCH_TRY(hipMemsetAsync(b->d_stats, 0, WOLFF_STAT_COUNT * sizeof(unsigned long long), b->stream));
    }
    b->reps.resize(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        const wolff_job& j = jobs[i];
        Rep& r = b->reps[i];
        r = Rep{};
        r.S = b->S + b->S_off[i];
        r.ov = b->ov + b->ov_off[i];
        r.rec = b->rec + b->rec_off[i];
        r.rec_count = 0;
        r.geo = make_geo(j.dim, (uint32_t)j.L);
        r.dim = j.dim;
        r.q = (uint32_t)j.q;
        r.thr = bond_threshold(j.J, j.T, j.q);
        r.k0 = (uint32_t)j.seed;
        r.k1 = (uint32_t)(j.seed >> 32);
        r.t = 0;
        r.n_left = (uint32_t)j.n_updates;
        r.measure = (j.flags & WOLFF_JOB_UPDATE_ONLY) ? 0u : 1u;
        r.stats = b->d_stats;
        if (j.start == 0) {
            hipLaunchKernelGGL(wolff::init_kernel, dim3(std::min<uint64_t>((Ns[i] + 255) / 256, 65536)),
                               dim3(256), 0, b->stream, r.S, r.geo, j.dim, r.k0, r.k1, r.q);
            BATCH_TRY(hipGetLastError());
        } else {
            BATCH_TRY(hipMemsetAsync(r.S, start_byte(j.q, j.start), Ns[i], b->stream));
        }
        b->left.push_back(j.n_updates);
        b->t.push_back(0);
        b->rec_read.push_back(0);
    }
    BATCH_TRY(copy_wait(b->stream, b->d_reps, b->reps.data(), n_jobs * sizeof(Rep),
                        hipMemcpyHostToDevice));
    for (int i = 0; i < n_jobs; ++i) {
        hipLaunchKernelGGL(wolff::measure_rep_kernel<1024>, dim3(1), dim3(1024), 0, b->stream,
                           b->d_reps + i);
        BATCH_TRY(hipGetLastError());
    }
    // longest expected work first: more sites first, colder first at equal size
    b->order.resize(n_jobs);
    for (int i = 0; i < n_jobs; ++i) b->order[i] = (uint32_t)i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](uint32_t x, uint32_t y) {
        const double wx = (double)Ns[x] * (double)b->reps[x].thr * (double)std::max<uint64_t>(jobs[x].n_updates, 1);
        const double wy = (double)Ns[y] * (double)b->reps[y].thr * (double)std::max<uint64_t>(jobs[y].n_updates, 1);
        return wx > wy;
    });
    BATCH_TRY(copy_wait(b->stream, b->d_order, b->order.data(), n_jobs * sizeof(uint32_t),
                        hipMemcpyHostToDevice));
    {   // LDS classes, each in the longest-first order above
        std::vector<wolff::LdsGeo> geos(n_jobs);
        std::vector<int> cls(n_jobs);
        for (int i = 0; i < n_jobs; ++i) {
            geos[i] = wolff::LdsGeo{};
            cls[i] = batch_lds_class(jobs[i], &geos[i]);
        }
        for (uint32_t r : b->order) {
            if (cls[r] < 0)
                b->order_glob.push_back(r);
            else
                b->lcls[cls[r]].order.push_back(r);
        }
        b->dims_glob = b->order_glob.empty() ? 0 : jobs[b->order_glob[0]].dim;
        for (uint32_t r : b->order_glob)
            if (jobs[r].dim != b->dims_glob) b->dims_glob = 0;
        BATCH_TRY(hipMalloc(&b->d_geos, n_jobs * sizeof(wolff::LdsGeo)));
        BATCH_TRY(copy_wait(b->stream, b->d_geos, geos.data(), n_jobs * sizeof(wolff::LdsGeo),
                            hipMemcpyHostToDevice));
        BATCH_TRY(hipMalloc(&b->d_next_aux, 3 * sizeof(uint32_t)));
        if (!b->order_glob.empty()) {
            BATCH_TRY(hipMalloc(&b->d_order_glob, b->order_glob.size() * sizeof(uint32_t)));
            BATCH_TRY(copy_wait(b->stream, b->d_order_glob, b->order_glob.data(),
                                b->order_glob.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        }
        for (int c = 0; c < 2; ++c) {
            BatchLdsClass& C = b->lcls[c];
            if (C.order.empty()) continue;
            C.wg = c == 0 ? 256 : 512;
            C.dims = jobs[C.order[0]].dim;
            for (uint32_t r : C.order) {
                if (jobs[r].dim != C.dims) C.dims = 0;
                C.lds_bytes = std::max(C.lds_bytes, batch_lds_bytes_for(geos[r]));
            }
            BATCH_TRY(hipMalloc(&C.d_order, C.order.size() * sizeof(uint32_t)));
            BATCH_TRY(copy_wait(b->stream, C.d_order, C.order.data(), C.order.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice));
            BATCH_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(lds_batch_fn(C.wg, C.dims)),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)C.lds_bytes));
        }
    }
    BATCH_TRY(hipStreamSynchronize(b->stream));
#undef BATCH_TRY
    *out = b;
    return WOLFF_OK;
}

extern "C" int wolff_batch_destroy(wolff_batch* b)
{
    free_batch(b);
    return WOLFF_OK;
}

extern "C" int wolff_batch_set_tiles(wolff_batch* b, int wg, int queue_entries)
{
    if (!b) return fail(WOLFF_EINVAL, "batch is NULL");
    if (!valid_tiles(wg, queue_entries)) return fail(WOLFF_EINVAL, "unsupported tile sizes");
    b->wg = wg;
    b->qentries = queue_entries;
    return WOLFF_OK;
}

extern "C" int wolff_batch_set_measure(wolff_batch* b, int on)
{
    if (!b) return fail(WOLFF_EINVAL, "batch is NULL");
    std::vector<Rep> cur(b->reps.size());
    HIP_TRY(copy_wait(b->stream, cur.data(), b->d_reps, cur.size() * sizeof(Rep), hipMemcpyDeviceToHost));
    b->measure = on ? 1 : 0;
    for (auto& r : cur) r.measure = (uint32_t)b->measure;
    HIP_TRY(copy_wait(b->stream, b->d_reps, cur.data(), cur.size() * sizeof(Rep), hipMemcpyHostToDevice));
    return WOLFF_OK;
}

extern "C" int wolff_batch_set_graph(wolff_batch* b, int on)
{
    if (!b) return fail(WOLFF_EINVAL, "batch is NULL");
    b->use_graph = on != 0;
    return WOLFF_OK;
}

extern "C" int wolff_batch_set_stream(wolff_batch* b, void* hip_stream)
{
    if (!b) return fail(WOLFF_EINVAL, "batch is NULL");
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->stream = hip_stream ? (hipStream_t)hip_stream : b->own_stream;
    return WOLFF_OK;
}

// One LDS-class launch of the batched LDS path on stream st.
static hipError_t launch_lds_class(wolff_batch* b, int c, hipStream_t st, uint32_t max_updates)
{
    const BatchLdsClass& C = b->lcls[c];
    const LdsBatchFn fn = lds_batch_fn(C.wg, C.dims);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), C.wg,
                                                     C.lds_bytes) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const uint32_t n = (uint32_t)C.order.size();
    const uint32_t grid = (uint32_t)std::min<uint64_t>(n, (uint64_t)per_cu * device_cus());
    uint32_t* next = b->d_next_aux + 1 + c;
    hipLaunchKernelGGL(wolff::reset_counter_kernel, dim3(1), dim3(64), 0, st, next);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(C.wg), C.lds_bytes, st, b->d_reps, b->d_geos, C.d_order, n,
                       next, max_updates, BATCH_LDS_RING - 1u, (uint64_t)0);
    return hipGetLastError();
}

// The LDS classes and the rest as concurrent launches: the first on the
// batch stream, the others on auxiliary streams that fork from it and
// join back into it.
static int run_batch_split(wolff_batch* b, uint32_t max_updates)
{
    std::vector<int> parts;                       // -1: the global class; 0, 1: LDS classes
    if (!b->order_glob.empty()) parts.push_back(-1);
    for (int c = 0; c < 2; ++c)
        if (!b->lcls[c].order.empty()) parts.push_back(c);
    for (size_t k = 1; k < parts.size(); ++k) {
        if (!b->aux[k - 1]) HIP_TRY(hipStreamCreateWithFlags(&b->aux[k - 1], hipStreamNonBlocking));
        if (!b->ev_join[k - 1]) HIP_TRY(hipEventCreateWithFlags(&b->ev_join[k - 1], hipEventDisableTiming));
    }
    if (!b->ev_fork) HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(b->ev_a, b->stream));
    HIP_TRY(hipEventRecord(b->ev_fork, b->stream));
    for (size_t k = 0; k < parts.size(); ++k) {
        hipStream_t st = k == 0 ? b->stream : b->aux[k - 1];
        if (k > 0) HIP_TRY(hipStreamWaitEvent(st, b->ev_fork, 0));
        if (parts[k] < 0) {
            const uint32_t n = (uint32_t)b->order_glob.size();
            const uint64_t resident = (uint64_t)batch_occupancy(b->wg, b->dims_glob, b->qentries);
            const uint32_t grid = (uint32_t)std::min<uint64_t>(n, resident);
            HIP_TRY(launch_batch(b->wg, b->dims_glob, grid, (uint32_t)b->qentries, st, b->d_reps,
                                 b->d_order_glob, n, b->d_next_aux, max_updates));
        } else {
            HIP_TRY(launch_lds_class(b, parts[k], st, max_updates));
        }
        if (k > 0) HIP_TRY(hipEventRecord(b->ev_join[k - 1], st));
    }
    for (size_t k = 1; k < parts.size(); ++k) HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_join[k - 1], 0));
    HIP_TRY(hipEventRecord(b->ev_b, b->stream));
    return WOLFF_OK;
}

extern "C" int wolff_batch_set_lds(wolff_batch* b, int on)
{
    if (!b) return fail(WOLFF_EINVAL, "batch is NULL");
    b->use_lds = on != 0;
    return WOLFF_OK;
}

extern "C" int wolff_batch_run(wolff_batch* b, uint64_t max_updates)
{
    if (!b) return fail(WOLFF_EINVAL, "batch is NULL");
    if (max_updates > T_LIMIT) return fail(WOLFF_EINVAL, "max_updates too large");
    uint32_t active = 0;
    for (size_t i = 0; i < b->jobs.size(); ++i) active += b->left[i] > 0;
    if (active == 0) return WOLFF_OK;
    if (b->use_lds && (!b->lcls[0].order.empty() || !b->lcls[1].order.empty())) {
        const int rc = run_batch_split(b, (uint32_t)max_updates);
        if (rc) return rc;
        b->timed = true;
        for (size_t i = 0; i < b->jobs.size(); ++i) {
            const uint64_t m = (max_updates == 0) ? b->left[i] : std::min<uint64_t>(b->left[i], max_updates);
            b->left[i] -= m;
            b->t[i] += m;
        }
        return WOLFF_OK;
    }
    const uint64_t resident = (uint64_t)batch_occupancy(b->wg, b->dims, b->qentries);
    const uint32_t n = (uint32_t)b->jobs.size();
    const uint32_t grid = (uint32_t)std::min<uint64_t>(n, resident);
    HIP_TRY(hipEventRecord(b->ev_a, b->stream));
    if (b->use_graph) {
        const std::vector<uint64_t> key = {(uint64_t)b->wg, (uint64_t)b->dims, (uint64_t)b->qentries, grid, max_updates,
                                           (uint64_t)(uintptr_t)b->stream};
        auto it = b->graphs.find(key);
        if (it == b->graphs.end()) {
            HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
            const hipError_t el = launch_batch(b->wg, b->dims, grid, (uint32_t)b->qentries, b->stream,
                                               b->d_reps, b->d_order, n, b->d_next,
                                               (uint32_t)max_updates);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(b->stream, &g);
            HIP_TRY(el);
            HIP_TRY(ec);
            hipGraphExec_t ex = nullptr;
            const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(ei);
            it = b->graphs.emplace(key, ex).first;
        }
        HIP_TRY(hipGraphLaunch(it->second, b->stream));
    } else {
        HIP_TRY(launch_batch(b->wg, b->dims, grid, (uint32_t)b->qentries, b->stream, b->d_reps, b->d_order,
                             n, b->d_next, (uint32_t)max_updates));
    }
    HIP_TRY(hipEventRecord(b->ev_b, b->stream));
    b->timed = true;
    for (size_t i = 0; i < b->jobs.size(); ++i) {
        const uint64_t m = (max_updates == 0) ? b->left[i] : std::min<uint64_t>(b->left[i], max_updates);
        b->left[i] -= m;
        b->t[i] += m;
    }
    return WOLFF_OK;
}

extern "C" int wolff_batch_last_ms(wolff_batch* b, double* ms)
{
    if (!b || !ms) return fail(WOLFF_EINVAL, "NULL argument");
    if (!b->timed) {
        *ms = 0.0;
        return WOLFF_OK;
    }
    float f = 0.0f;
    HIP_TRY(hipEventSynchronize(b->ev_b));
    HIP_TRY(hipEventElapsedTime(&f, b->ev_a, b->ev_b));
    *ms = f;
    return WOLFF_OK;
}

extern "C" int wolff_batch_stats_read(wolff_batch* b, uint64_t* out, int n, int reset)
{
    if (!b) return fail(WOLFF_EINVAL, "batch is NULL");
    for (hipStream_t st : b->aux)
        if (st) HIP_TRY(hipStreamSynchronize(st));
    return read_stats(b->stream, b->d_stats, out, n, reset);
}

extern "C" int wolff_batch_progress(wolff_batch* b, int job, uint64_t* left, uint64_t* t)
{
    if (!b || job < 0 || (size_t)job >= b->jobs.size()) return fail(WOLFF_EINVAL, "bad job index");
    if (left) *left = b->left[job];
    if (t) *t = b->t[job];
    return WOLFF_OK;
}

extern "C" int wolff_batch_records(wolff_batch* b, int job, wolff_record* out, uint64_t cap,
                                   uint64_t* n_out)
{
    if (!b || job < 0 || (size_t)job >= b->jobs.size() || (!out && cap > 0))
        return fail(WOLFF_EINVAL, "bad argument");
    Rep r;
    HIP_TRY(copy_wait(b->stream, &r, b->d_reps + job, sizeof(Rep), hipMemcpyDeviceToHost));
    const uint64_t live = r.rec_count - b->rec_read[job];
    const uint64_t k = std::min(cap, live);
    if (k)
        HIP_TRY(copy_wait(b->stream, out, b->rec + b->rec_off[job] + b->rec_read[job],
                          k * sizeof(wolff_record), hipMemcpyDeviceToHost));
    b->rec_read[job] += k;
    if (n_out) *n_out = k;
    if (r.err) return fail(WOLFF_ESTATE, err_message(r.err));
    return WOLFF_OK;
}

extern "C" int wolff_batch_get_spins(wolff_batch* b, int job, int8_t* host, uint64_t n)
{
    if (!b || job < 0 || (size_t)job >= b->jobs.size() || !host) return fail(WOLFF_EINVAL, "bad argument");
    const Rep& r = b->reps[job];
    if (n != r.geo.N) return fail(WOLFF_EINVAL, "n must equal the number of sites");
    return copy_spins_out(b->stream, r.geo, r.dim, r.S, host, n, (int)r.q);
}

// ================================================================== server
// Continuous-batching request loop over the batched kernel.  Host-side
// state per job; device memory per job is one stream-ordered allocation
// (spins | overflow stack | records).
namespace {

struct SrvJob {
    wolff_job spec{};
    uint64_t id = 0;
    int state = WOLFF_JOB_QUEUED;
    uint64_t N = 0;
    uint64_t footprint = 0;
    void* block = nullptr;
    Rep rep{};
    bool fresh = false;                 // admitted, initial (B, M) not measured yet
    std::vector<wolff_record> results;  // records of a finished job
    uint64_t taken = 0;
};

uint64_t job_footprint(uint64_t N, uint64_t n_updates)
{
    return padded_bytes(N) + ((4 * N + 255) & ~uint64_t(255)) +
           std::max<uint64_t>(n_updates, 1) * sizeof(wolff_record) + 256;
}

}  // namespace

struct wolff_server {
    hipStream_t stream = nullptr;
    uint64_t budget = 0;
    uint64_t resident = 0;
    uint64_t slots = 0;
    int wg = 256;
    int qentries = 2048;
    uint64_t ticks_per_ms = 100000;     // wall-clock counter rate
    uint64_t next_id = 1;
    std::map<uint64_t, SrvJob> jobs;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> running;      // slot order of the last quantum
    std::vector<uint64_t> finished;     // finished since the last query
    Rep* h_reps = nullptr;              // pinned staging of the descriptors
    Rep* d_reps = nullptr;
    uint32_t* d_order = nullptr;
    uint32_t* d_next = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    uint64_t quanta = 0, updates = 0, added = 0;
    double gpu_ms = 0.0;
    // LDS classes of the batched form (as in wolff_batch): per quantum, the
    // running Ising jobs that fit one workgroup's LDS go to lds_batch_kernel
    // launches (up to each class's resident workgroups; the overflow and
    // every other job to the one-workgroup kernel), all three concurrent
    bool use_lds = true;
    wolff::LdsGeo* h_geos = nullptr;    // pinned staging, one per slot
    wolff::LdsGeo* d_geos = nullptr;
    uint32_t* h_lists = nullptr;        // pinned: three slot lists of `slots` entries
    uint32_t* d_lists = nullptr;
    uint32_t* d_next3 = nullptr;
    hipStream_t aux[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
    int lds_cap[2] = {0, 0};            // resident workgroups of each LDS class
};

static void free_server(wolff_server* v)
{
    if (!v) return;
    if (v->stream) {
        for (auto& kv : v->jobs)
            if (kv.second.block) (void)hipFreeAsync(kv.second.block, v->stream);
        (void)hipStreamSynchronize(v->stream);
    }
    for (hipStream_t st : v->aux)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    if (v->ev_fork) (void)hipEventDestroy(v->ev_fork);
    for (hipEvent_t e : v->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (v->h_geos) (void)hipHostFree(v->h_geos);
    if (v->d_geos) (void)hipFree(v->d_geos);
    if (v->h_lists) (void)hipHostFree(v->h_lists);
    if (v->d_lists) (void)hipFree(v->d_lists);
    if (v->d_next3) (void)hipFree(v->d_next3);
    if (v->h_reps) (void)hipHostFree(v->h_reps);
    if (v->d_reps) (void)hipFree(v->d_reps);
    if (v->d_order) (void)hipFree(v->d_order);
    if (v->d_next) (void)hipFree(v->d_next);
    if (v->ev_a) (void)hipEventDestroy(v->ev_a);
    if (v->ev_b) (void)hipEventDestroy(v->ev_b);
    if (v->stream) (void)hipStreamDestroy(v->stream);
    delete v;
}

extern "C" int wolff_server_create(uint64_t hbm_budget_bytes, int max_slots, wolff_server** out)
{
    if (!out || max_slots < 0) return fail(WOLFF_EINVAL, "bad argument");
    wolff_server* v = new (std::nothrow) wolff_server();
    if (!v) return fail(WOLFF_ENOMEM, "host allocation failed");
#define SRV_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            int code_ = e_ == hipErrorOutOfMemory ? WOLFF_ENOMEM : WOLFF_EDEVICE;       \
            free_server(v);                                                             \
            return fail(code_, std::string(#expr) + ": " + hipGetErrorString(e_));      \
        }                                                                               \
    } while (0)
    SRV_TRY(hipStreamCreateWithFlags(&v->stream, hipStreamNonBlocking));
    if (hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        SRV_TRY(hipMemGetInfo(&free_b, &total_b));
        hbm_budget_bytes = (uint64_t)(0.8 * (double)free_b);
    }
    v->budget = hbm_budget_bytes;
    const int cap = batch_occupancy(v->wg, 0, v->qentries);
    v->slots = (max_slots > 0) ? (uint64_t)std::min(max_slots, cap) : (uint64_t)cap;
    int dev = 0, khz = 0;
    SRV_TRY(hipGetDevice(&dev));
    SRV_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz > 0) v->ticks_per_ms = (uint64_t)khz;
    SRV_TRY(hipHostMalloc((void**)&v->h_reps, v->slots * sizeof(Rep), hipHostMallocDefault));
    SRV_TRY(hipMalloc(&v->d_reps, v->slots * sizeof(Rep)));
    SRV_TRY(hipMalloc(&v->d_order, v->slots * sizeof(uint32_t)));
    SRV_TRY(hipMalloc(&v->d_next, sizeof(uint32_t)));
    {
        std::vector<uint32_t> ident(v->slots);
        for (uint64_t i = 0; i < v->slots; ++i) ident[i] = (uint32_t)i;
        SRV_TRY(copy_wait(v->stream, v->d_order, ident.data(), v->slots * sizeof(uint32_t),
                          hipMemcpyHostToDevice));
    }
    SRV_TRY(hipEventCreate(&v->ev_a));
    SRV_TRY(hipEventCreate(&v->ev_b));
    SRV_TRY(hipHostMalloc((void**)&v->h_geos, v->slots * sizeof(wolff::LdsGeo), hipHostMallocDefault));
    SRV_TRY(hipMalloc(&v->d_geos, v->slots * sizeof(wolff::LdsGeo)));
    SRV_TRY(hipHostMalloc((void**)&v->h_lists, 3 * v->slots * sizeof(uint32_t), hipHostMallocDefault));
    SRV_TRY(hipMalloc(&v->d_lists, 3 * v->slots * sizeof(uint32_t)));
    SRV_TRY(hipMalloc(&v->d_next3, 3 * sizeof(uint32_t)));
    for (int k = 0; k < 2; ++k) {
        SRV_TRY(hipStreamCreateWithFlags(&v->aux[k], hipStreamNonBlocking));
        SRV_TRY(hipEventCreateWithFlags(&v->ev_join[k], hipEventDisableTiming));
    }
    SRV_TRY(hipEventCreateWithFlags(&v->ev_fork, hipEventDisableTiming));
    for (int c = 0; c < 2; ++c) {
        // the mixed-dimension kernels, with the LDS of each class's largest lattice
        const int wg = c == 0 ? 256 : 512;
        const size_t bytes = ((size_t)(c == 0 ? 2048u : 32768u) + BATCH_LDS_RING) * sizeof(uint32_t);
        const void* fn = reinterpret_cast<const void*>(lds_batch_fn(wg, 0));
        SRV_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, wg, bytes) != hipSuccess || per_cu < 1)
            per_cu = 1;
        v->lds_cap[c] = per_cu * device_cus();
    }
#undef SRV_TRY
    *out = v;
    return WOLFF_OK;
}

extern "C" int wolff_server_destroy(wolff_server* v)
{
    free_server(v);
    return WOLFF_OK;
}

extern "C" int wolff_server_submit(wolff_server* v, const wolff_job* job, uint64_t* job_id)
{
    if (!v || !job || !job_id) return fail(WOLFF_EINVAL, "NULL argument");
    uint64_t N = 0;
    int rc = check_params(job->dim, job->L, job->J, job->T, &N);
    if (rc) return rc;
    if (job->start < -1 || job->start > 1 || (job->flags & ~WOLFF_JOB_UPDATE_ONLY) != 0 ||
        !valid_q(job->q))
        return fail(WOLFF_EINVAL, "bad start, flags or q field");
    if (job->n_updates > T_LIMIT) return fail(WOLFF_ERANGE, "too many updates");
    SrvJob j;
    j.spec = *job;
    j.id = v->next_id++;
    j.N = N;
    j.footprint = job_footprint(N, job->n_updates);
    if (j.footprint > v->budget) return fail(WOLFF_EINVAL, "job footprint exceeds the HBM budget");
    const uint64_t id = j.id;
    v->jobs.emplace(id, std::move(j));
    v->queue.push_back(id);
    *job_id = id;
    return WOLFF_OK;
}

// Admit queued jobs in arrival order while a slot and the footprint are free.
static int server_admit(wolff_server* v)
{
    while (!v->queue.empty() && v->running.size() < v->slots) {
        SrvJob& j = v->jobs.at(v->queue.front());
        if (v->resident + j.footprint > v->budget) break;            // strict FIFO
        void* blk = nullptr;
        HIP_TRY(hipMallocAsync(&blk, j.footprint, v->stream));
        j.block = blk;
        int8_t* S = (int8_t*)blk;
        uint32_t* ov = (uint32_t*)((char*)blk + padded_bytes(j.N));
        wolff_record* rec = (wolff_record*)((char*)ov + ((4 * j.N + 255) & ~uint64_t(255)));
        HIP_TRY(hipMemsetAsync(S, 0, padded_bytes(j.N), v->stream));
        if (j.spec.start == 0) {
            hipLaunchKernelGGL(wolff::init_kernel, dim3(std::min<uint64_t>((j.N + 255) / 256, 65536)),
                               dim3(256), 0, v->stream, S, make_geo(j.spec.dim, (uint32_t)j.spec.L),
                               j.spec.dim, (uint32_t)j.spec.seed, (uint32_t)(j.spec.seed >> 32),
                               (uint32_t)j.spec.q);
            HIP_TRY(hipGetLastError());
        } else {
            HIP_TRY(hipMemsetAsync(S, start_byte(j.spec.q, j.spec.start), j.N, v->stream));
        }
        Rep& r = j.rep;
        r = Rep{};
        r.S = S;
        r.ov = ov;
        r.rec = rec;
        r.rec_count = 0;
        r.geo = make_geo(j.spec.dim, (uint32_t)j.spec.L);
        r.dim = j.spec.dim;
        r.q = (uint32_t)j.spec.q;
        r.thr = bond_threshold(j.spec.J, j.spec.T, j.spec.q);
        r.k0 = (uint32_t)j.spec.seed;
        r.k1 = (uint32_t)(j.spec.seed >> 32);
        r.t = 0;
        r.n_left = (uint32_t)j.spec.n_updates;
        r.measure = (j.spec.flags & WOLFF_JOB_UPDATE_ONLY) ? 0u : 1u;
        j.fresh = true;
        j.state = WOLFF_JOB_RUNNING;
        v->resident += j.footprint;
        v->running.push_back(j.id);
        v->queue.pop_front();
    }
    return WOLFF_OK;
}

// One quantum over the n running slots in up to three concurrent launches:
// the LDS classes (slot lists 1 and 2, at most each class's resident
// workgroups) and the one-workgroup kernel for the rest (list 0).  The slot
// descriptors are already on the device.
static int server_split_quantum(wolff_server* v, uint32_t n, uint64_t budget)
{
    uint32_t cnt[3] = {0u, 0u, 0u};
    uint32_t* lists[3] = {v->h_lists, v->h_lists + v->slots, v->h_lists + 2 * v->slots};
    for (uint32_t i = 0; i < n; ++i) {
        const SrvJob& j = v->jobs.at(v->running[i]);
        wolff::LdsGeo g{};
        int c = batch_lds_class(j.spec, &g);
        if (c >= 0 && cnt[1 + c] >= (uint32_t)v->lds_cap[c]) c = -1;   // class full: global kernel
        v->h_geos[i] = g;
        lists[1 + c][cnt[1 + c]++] = i;
    }
    HIP_TRY(hipMemcpyAsync(v->d_geos, v->h_geos, n * sizeof(wolff::LdsGeo), hipMemcpyHostToDevice, v->stream));
    HIP_TRY(hipMemcpyAsync(v->d_lists, v->h_lists, 3 * v->slots * sizeof(uint32_t), hipMemcpyHostToDevice,
                           v->stream));
    HIP_TRY(hipEventRecord(v->ev_fork, v->stream));
    int k = 0;                                                       // launches so far
    for (int part = 0; part < 3; ++part) {
        if (cnt[part] == 0) continue;
        hipStream_t st = k == 0 ? v->stream : v->aux[k - 1];
        if (k > 0) HIP_TRY(hipStreamWaitEvent(st, v->ev_fork, 0));
        const uint32_t* d_list = v->d_lists + (size_t)part * v->slots;
        uint32_t* next = v->d_next3 + part;
        if (part == 0) {
            HIP_TRY(launch_batch(v->wg, 0, cnt[0], (uint32_t)v->qentries, st, v->d_reps, d_list, cnt[0],
                                 next, 0u, budget));
        } else {
            const int c = part - 1;
            const int wg = c == 0 ? 256 : 512;
            const size_t bytes = ((size_t)(c == 0 ? 2048u : 32768u) + BATCH_LDS_RING) * sizeof(uint32_t);
            hipLaunchKernelGGL(wolff::reset_counter_kernel, dim3(1), dim3(64), 0, st, next);
            hipLaunchKernelGGL(lds_batch_fn(wg, 0), dim3(cnt[part]), dim3(wg), bytes, st, v->d_reps,
                               v->d_geos, d_list, cnt[part], next, 0u, BATCH_LDS_RING - 1u, budget);
            HIP_TRY(hipGetLastError());
        }
        if (k > 0) HIP_TRY(hipEventRecord(v->ev_join[k - 1], st));
        ++k;
    }
    for (int m = 1; m < k; ++m) HIP_TRY(hipStreamWaitEvent(v->stream, v->ev_join[m - 1], 0));
    return WOLFF_OK;
}

extern "C" int wolff_server_set_lds(wolff_server* v, int on)
{
    if (!v) return fail(WOLFF_EINVAL, "server is NULL");
    v->use_lds = on != 0;
    return WOLFF_OK;
}

extern "C" int wolff_server_step(wolff_server* v, double quantum_ms, uint64_t* n_finished)
{
    if (!v || !(quantum_ms >= 0.0)) return fail(WOLFF_EINVAL, "bad argument");
    int rc = server_admit(v);
    if (rc) return rc;
    uint64_t fin = 0;
    const uint32_t n = (uint32_t)v->running.size();
    if (n > 0) {
        for (uint32_t i = 0; i < n; ++i) v->h_reps[i] = v->jobs.at(v->running[i]).rep;
        HIP_TRY(hipMemcpyAsync(v->d_reps, v->h_reps, n * sizeof(Rep), hipMemcpyHostToDevice, v->stream));
        for (uint32_t i = 0; i < n; ++i) {
            SrvJob& j = v->jobs.at(v->running[i]);
            if (j.fresh) {
                hipLaunchKernelGGL(wolff::measure_rep_kernel<1024>, dim3(1), dim3(1024), 0, v->stream,
                                   v->d_reps + i);
                HIP_TRY(hipGetLastError());
                j.fresh = false;
            }
        }
        const uint64_t budget = (uint64_t)(quantum_ms * (double)v->ticks_per_ms);
        HIP_TRY(hipEventRecord(v->ev_a, v->stream));
        if (v->use_lds) {
            if ((rc = server_split_quantum(v, n, budget == 0 ? 1 : budget))) return rc;
        } else {
            HIP_TRY(launch_batch(v->wg, 0, n, (uint32_t)v->qentries, v->stream, v->d_reps, v->d_order, n,
                                 v->d_next, 0u, budget == 0 ? 1 : budget));
        }
        HIP_TRY(hipEventRecord(v->ev_b, v->stream));
        HIP_TRY(hipMemcpyAsync(v->h_reps, v->d_reps, n * sizeof(Rep), hipMemcpyDeviceToHost, v->stream));
        HIP_TRY(hipStreamSynchronize(v->stream));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, v->ev_a, v->ev_b));
        v->gpu_ms += ms;
        v->quanta += 1;
        std::vector<uint64_t> still;
        still.reserve(n);
        for (uint32_t i = 0; i < n; ++i) {
            SrvJob& j = v->jobs.at(v->running[i]);
            const Rep before = j.rep;
            j.rep = v->h_reps[i];
            v->updates += j.rep.t - before.t;
            if (j.rep.n_left == 0 || j.rep.err) {
                const uint64_t cnt = j.rep.rec_count;
                j.results.resize(cnt);
                if (cnt)
                    HIP_TRY(copy_wait(v->stream, j.results.data(), j.rep.rec,
                                      cnt * sizeof(wolff_record), hipMemcpyDeviceToHost));
                for (const auto& r : j.results) v->added += (uint64_t)r.csize;
                HIP_TRY(hipFreeAsync(j.block, v->stream));
                j.block = nullptr;
                v->resident -= j.footprint;
                j.state = j.rep.err ? WOLFF_JOB_FAILED : WOLFF_JOB_DONE;
                v->finished.push_back(j.id);
                ++fin;
            } else {
                still.push_back(j.id);
            }
        }
        v->running.swap(still);
    }
    if (n_finished) *n_finished = fin;
    return WOLFF_OK;
}

extern "C" int wolff_server_status(wolff_server* v, uint64_t job_id, int* state, uint64_t* updates_done)
{
    if (!v) return fail(WOLFF_EINVAL, "server is NULL");
    auto it = v->jobs.find(job_id);
    if (it == v->jobs.end()) return fail(WOLFF_EINVAL, "unknown job id");
    if (state) *state = it->second.state;
    if (updates_done) *updates_done = it->second.rep.t;
    return WOLFF_OK;
}

extern "C" int wolff_server_finished(wolff_server* v, uint64_t* ids, uint64_t cap, uint64_t* n_out)
{
    if (!v || (!ids && cap > 0)) return fail(WOLFF_EINVAL, "bad argument");
    const uint64_t k = std::min<uint64_t>(cap, v->finished.size());
    for (uint64_t i = 0; i < k; ++i) ids[i] = v->finished[i];
    v->finished.erase(v->finished.begin(), v->finished.begin() + (ptrdiff_t)k);
    if (n_out) *n_out = k;
    return WOLFF_OK;
}

extern "C" int wolff_server_take(wolff_server* v, uint64_t job_id, wolff_record* out, uint64_t cap,
                                 uint64_t* n_out)
{
    if (!v || (!out && cap > 0)) return fail(WOLFF_EINVAL, "bad argument");
    auto it = v->jobs.find(job_id);
    if (it == v->jobs.end()) return fail(WOLFF_EINVAL, "unknown job id");
    SrvJob& j = it->second;
    if (j.state != WOLFF_JOB_DONE && j.state != WOLFF_JOB_FAILED)
        return fail(WOLFF_EINVAL, "job has not finished");
    const uint64_t k = std::min<uint64_t>(cap, j.results.size() - j.taken);
    if (k) std::memcpy(out, j.results.data() + j.taken, k * sizeof(wolff_record));
    j.taken += k;
    if (n_out) *n_out = k;
    const bool failed = j.state == WOLFF_JOB_FAILED;
    const std::string msg = failed ? err_message(j.rep.err) : std::string();
    if (j.taken == j.results.size()) v->jobs.erase(it);
    if (failed) return fail(WOLFF_ESTATE, msg);
    return WOLFF_OK;
}

extern "C" int wolff_server_get_stats(wolff_server* v, wolff_server_stats* out)
{
    if (!v || !out) return fail(WOLFF_EINVAL, "NULL argument");
    out->queued = v->queue.size();
    out->running = v->running.size();
    uint64_t done = 0;
    for (const auto& kv : v->jobs)
        done += kv.second.state == WOLFF_JOB_DONE || kv.second.state == WOLFF_JOB_FAILED;
    out->done = done;
    out->slots = v->slots;
    out->resident_bytes = v->resident;
    out->budget_bytes = v->budget;
    out->quanta = v->quanta;
    out->updates = v->updates;
    out->added_spins = v->added;
    out->gpu_ms = v->gpu_ms;
    return WOLFF_OK;
}

// ============================================== no-allocation entry point
// wolff_run_noalloc keeps everything the kernels need beyond the caller's
// spins and records in `scratch`, a fixed array in device memory: the
// lattice descriptor, the replica list and work counter of the
// one-workgroup kernel, and its frontier overflow stack (4 bytes per site).
// Every device the library runs on holds its own copy for the life of the
// process, and every call on that device shares it, so calls that overlap
// on one device (different streams, different threads) race.
static constexpr size_t NOALLOC_HEADER = 1024;     // descriptor, list, counter
static constexpr size_t NOALLOC_BYTES =
    NOALLOC_HEADER + (size_t)WOLFF_NOALLOC_MAX_SITES * sizeof(uint32_t);
static_assert(sizeof(Rep) + 512 <= NOALLOC_HEADER, "descriptor does not fit the header");

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Device address of `scratch` on each device, taken once per device with
// that device current (the array's name is not a device address in host
// code).
static constexpr int NOALLOC_MAX_DEVICES = 64;
static unsigned char* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

static int scratch_address(unsigned char** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(WOLFF_EDEVICE, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(WOLFF_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_dev[dev];
    return WOLFF_OK;
}

namespace wolff {
// The descriptor, the one-entry replica list and the work counter, written
// on the stream (no host copy into device memory).
__global__ void noalloc_setup_kernel(Rep* R, Rep init, uint32_t* order, uint32_t* next)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *R = init;
        order[0] = 0u;
        next[0] = 0u;
    }
}

// The error bits and update index of the descriptor, for the host.
__global__ void noalloc_status_kernel(const Rep* R, uint32_t* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = R->err;
        out[1] = R->t;
    }
}
}  // namespace wolff

extern "C" int wolff_run_noalloc(int dim, int L, double J, double T, uint64_t seed,
                                 int8_t* spins, uint64_t t0, uint32_t flags, int measure,
                                 uint64_t n_updates, wolff_record* records, void* hip_stream)
{
    uint64_t N = 0;
    int rc = check_params(dim, L, J, T, &N);
    if (rc) return rc;
    if (N > WOLFF_NOALLOC_MAX_SITES)
        return fail(WOLFF_EINVAL, "wolff_run_noalloc: L^dim = " + std::to_string(N) +
                                      " exceeds the fixed scratch limit of " +
                                      std::to_string(WOLFF_NOALLOC_MAX_SITES) + " sites");
    if (!spins || (uintptr_t)spins % 16u)
        return fail(WOLFF_EINVAL, "wolff_run_noalloc: spins must be a 16-byte aligned device pointer");
    if (n_updates > 0 && (!records || (uintptr_t)records % 8u))
        return fail(WOLFF_EINVAL, "wolff_run_noalloc: records must be an 8-byte aligned device pointer");
    if ((flags & ~(uint32_t)WOLFF_BUFFERS_KEEP_SPINS) != 0u)
        return fail(WOLFF_EINVAL, "wolff_run_noalloc: unknown flags");
    const bool keep = (flags & WOLFF_BUFFERS_KEEP_SPINS) != 0u;
    const uint64_t t_start = keep ? t0 : 0u;
    if (t_start > T_LIMIT || n_updates > T_LIMIT - t_start)
        return fail(WOLFF_ERANGE, "wolff_run_noalloc: t0 + n_updates exceeds 2^32 - 2");
    unsigned char* base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Rep* R = reinterpret_cast<Rep*>(base);
    uint32_t* order = reinterpret_cast<uint32_t*>(base + 512);
    uint32_t* next = order + 1;
    uint32_t* status = order + 2;
    uint32_t* ov = reinterpret_cast<uint32_t*>(base + NOALLOC_HEADER);

    const Geo g = make_site_order_geo(dim, (uint32_t)L);
    if (!keep) {
        hipLaunchKernelGGL(wolff::init_kernel, dim3(std::min<uint64_t>((N + 255) / 256, 65536)),
                           dim3(256), 0, st, spins, g, dim, (uint32_t)seed, (uint32_t)(seed >> 32), 0u);
        HIP_TRY(hipGetLastError());
    }
    Rep r{};
    r.S = spins;
    r.ov = ov;
    r.rec = records;
    r.rec_count = 0;
    r.geo = g;
    r.dim = dim;
    r.thr = bond_threshold(J, T);
    r.k0 = (uint32_t)seed;
    r.k1 = (uint32_t)(seed >> 32);
    r.t = (uint32_t)t_start;
    r.t_norm = (uint32_t)t_start;
    r.n_left = (uint32_t)n_updates;
    r.measure = measure ? 1u : 0u;
    r.abort = nullptr;
    hipLaunchKernelGGL(wolff::noalloc_setup_kernel, dim3(1), dim3(64), 0, st, R, r, order, next);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(wolff::measure_rep_kernel<1024>, dim3(1), dim3(1024), 0, st, R);
    HIP_TRY(hipGetLastError());
    if (n_updates > 0) {
        // the one-workgroup path with the tiles wolff_create picks for this size
        const int wg = N <= 4096 ? 64 : N <= 16384 ? 128 : N < (1ull << 20) ? 256 : 512;
        const uint32_t qe = N < (1ull << 20) ? 2048u : 4096u;
        HIP_TRY(launch_batch(wg, dim, 1u, qe, st, R, order, 1u, next, 0u));
        // plain +-1 bytes in the caller's lattice (the incremental bond sum tags members)
        hipLaunchKernelGGL(wolff::plain_kernel, dim3(std::min<uint64_t>((N / 4 + 255) / 256 + 1, 4096)),
                           dim3(256), 0, st, spins, (uint32_t)N);
        HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(wolff::noalloc_status_kernel, dim3(1), dim3(64), 0, st, R, status);
    HIP_TRY(hipGetLastError());
    uint32_t host_status[2] = {0u, 0u};
    HIP_TRY(hipMemcpyAsync(host_status, status, sizeof(host_status), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (host_status[0] != 0u) return fail(WOLFF_ESTATE, err_message(host_status[0]));
    if ((uint64_t)host_status[1] != t_start + n_updates)
        return fail(WOLFF_ESTATE, "wolff_run_noalloc: the kernel stopped at update " +
                                      std::to_string(host_status[1]));
    return WOLFF_OK;
}
