/*
 * CPU oracle for the Wolff single-cluster update of the Ising model.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never calls it and shares no code, header or constant table with it.
 *
 * What it computes (Komura & Okabe, arXiv:1110.0899):
 *   - Hamiltonian H = -J sum_<ij> S_i S_j on the periodic square (d=2) or
 *     simple-cubic (d=3) lattice (Section 2, Eq. for H).
 *   - The Wolff single-cluster update, steps (i)-(v) of Section 2: pick a
 *     random site, add parallel nearest neighbours with probability
 *     p = 1 - exp(-2 J / T), repeat for every added spin until no new bond is
 *     made, flip the cluster.  The paper leaves the flip timing free; this
 *     oracle flips the whole cluster at the end of the update.
 *   - Energy and magnetisation after every update (Section 5, the
 *     "+ measurement" timing), recomputed from scratch over the lattice.
 *
 * Readings of points the paper leaves open (the paper uses an LCG whose
 * parameters it does not give):
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11,
 *     "Parallel random numbers: as easy as 1, 2, 3"), key = (seed low word,
 *     seed high word).
 *       initial spin of site i : word 0 of philox((i, 0, 0, 2)); +1 if < 2^31
 *       seed site of update t  : s = floor(((x1 << 32) | x0) * N / 2^64),
 *                                x = philox((0, t, 0, 1))
 *       bond (b, mu) of update t with seed site s :
 *                                r = word mu of philox((b, t, s, 0)),
 *                                where bond (b, mu) joins b and b + e_mu.
 *   - Bond test: active iff r < thr, thr = floor(p * 2^32) computed once in
 *     binary64 (p = 1 - exp(-2 J / T)), clamped to 2^32 - 1.
 *   - "Parallel" means equal to s0, the seed's spin before the update.
 *   - Site index i = x + L*y (+ L*L*z); L = 2 keeps both bonds between a pair
 *     (the bond set is always {(i, mu)}: N*d bonds).
 * With these readings the cluster is the connected component of s in the
 * graph of active bonds between sites whose spin equals s0, so every correct
 * traversal order gives the same cluster.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ---------------------------------------------------------------- Philox */

/* One Philox4x32 round: two 32x32->64 products, the high halves are mixed
 * into the other words with the round key (Salmon et al., Sec. 3.3). */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

/* Philox4x32 with 10 rounds; the key advances by the Weyl constants
 * (golden ratio, sqrt(3)-1) between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static void make_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

/* ------------------------------------------------------------ parameters */

/* floor(p * 2^32) in binary64, clamped to [0, 2^32 - 1]. */
static uint32_t scaled_threshold(double p)
{
    const double scaled = ldexp(p, 32);
    if (!(scaled > 0.0)) return 0u;
    if (scaled >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)floor(scaled);
}

/* thr = floor(p * 2^32), p = 1 - exp(-2J/T) (Section 2, step (ii)). */
uint32_t orc_threshold(double J, double T)
{
    const double p = 1.0 - exp(-2.0 * J / T);
    return scaled_threshold(p);
}

/* Step (i): the seed site of update t, uniform on [0, N). */
uint64_t orc_seed_site(uint64_t seed, uint32_t t, uint64_t N)
{
    uint32_t key[2], ctr[4] = {0u, t, 0u, 1u}, x[4];
    make_key(seed, key);
    orc_philox4x32_10(ctr, key, x);
    const unsigned __int128 u = ((unsigned __int128)(((uint64_t)x[1] << 32) | x[0])) * N;
    return (uint64_t)(u >> 64);
}

static uint64_t lattice_sites(int dim, int L)
{
    uint64_t N = 1;
    for (int a = 0; a < dim; ++a) N *= (uint64_t)L;
    return N;
}

/* Site index <-> coordinates, x fastest. */
static void site_coords(int dim, int L, uint64_t i, int c[3])
{
    c[0] = c[1] = c[2] = 0;
    for (int a = 0; a < dim; ++a) {
        c[a] = (int)(i % (uint64_t)L);
        i /= (uint64_t)L;
    }
}

static uint64_t site_index(int dim, int L, const int c[3])
{
    uint64_t i = 0;
    for (int a = dim - 1; a >= 0; --a) i = i * (uint64_t)L + (uint64_t)c[a];
    return i;
}

/* Neighbour of site i one step along axis mu in direction sgn (+1 / -1),
 * periodic boundaries (Section 2). */
static uint64_t neighbour(int dim, int L, uint64_t i, int mu, int sgn)
{
    int c[3];
    site_coords(dim, L, i, c);
    c[mu] = (c[mu] + sgn + L) % L;
    return site_index(dim, L, c);
}

/* ----------------------------------------------------------------- state */

void orc_init_spins(int dim, int L, uint64_t seed, int8_t *S)
{
    const uint64_t N = lattice_sites(dim, L);
    uint32_t key[2];
    make_key(seed, key);
    for (uint64_t i = 0; i < N; ++i) {
        uint32_t ctr[4] = {(uint32_t)i, 0u, 0u, 2u}, x[4];
        orc_philox4x32_10(ctr, key, x);
        S[i] = (x[0] < 0x80000000u) ? (int8_t)1 : (int8_t)-1;
    }
}

/* Integer bond sum B = sum_i sum_mu S_i S_{i+e_mu} (E = -J B) and
 * magnetisation M = sum_i S_i, recomputed from the whole lattice. */
void orc_observables(int dim, int L, const int8_t *S, int64_t *B, int64_t *M)
{
    const uint64_t N = lattice_sites(dim, L);
    int64_t b = 0, m = 0;
    for (uint64_t i = 0; i < N; ++i) {
        m += S[i];
        for (int mu = 0; mu < dim; ++mu)
            b += (int64_t)S[i] * (int64_t)S[neighbour(dim, L, i, mu, +1)];
    }
    *B = b;
    *M = m;
}

/* ------------------------------------------------------- one Wolff update */

/* Grow the cluster of update t from the current lattice S (not modified).
 * member[] (N bytes) is set to 1 for cluster sites and 0 elsewhere.
 * Returns |C|; *s_out / *s0_out receive the seed site and its spin.
 * Returns 0 on allocation failure. */
uint64_t orc_cluster(int dim, int L, uint32_t thr, uint64_t seed, uint32_t t,
                     const int8_t *S, uint8_t *member, uint64_t *s_out, int *s0_out)
{
    const uint64_t N = lattice_sites(dim, L);
    uint32_t key[2];
    make_key(seed, key);
    const uint64_t s = orc_seed_site(seed, t, N);
    const int8_t s0 = S[s];

    uint64_t *stack = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    if (!stack) return 0;
    memset(member, 0, (size_t)N);

    uint64_t size = 0, top = 0;
    member[s] = 1;
    stack[top++] = s;
    size = 1;
    while (top > 0) {
        const uint64_t j = stack[--top];
        for (int mu = 0; mu < dim; ++mu) {
            for (int sgn = +1; sgn >= -1; sgn -= 2) {
                const uint64_t k = neighbour(dim, L, j, mu, sgn);
                if (member[k] || S[k] != s0) continue;
                /* bond (b, mu) joins b and b + e_mu */
                const uint64_t b = (sgn > 0) ? j : k;
                uint32_t ctr[4] = {(uint32_t)b, t, (uint32_t)s, 0u}, r[4];
                orc_philox4x32_10(ctr, key, r);
                if (r[mu] < thr) {
                    member[k] = 1;
                    stack[top++] = k;
                    ++size;
                }
            }
        }
    }
    free(stack);
    if (s_out) *s_out = s;
    if (s0_out) *s0_out = s0;
    return size;
}

/* Run n updates with indices t0 .. t0+n-1 on S (modified in place).
 * rec receives (B, M, |C|) after each update (3 int64 per update).
 * Returns 0, -1 on allocation failure, -2 if the magnetisation identity
 * M_after = M_before - 2 s0 |C| fails (an internal consistency check). */
int orc_run(int dim, int L, uint32_t thr, uint64_t seed, uint32_t t0, uint64_t n,
            int8_t *S, int64_t *rec)
{
    const uint64_t N = lattice_sites(dim, L);
    uint8_t *member = (uint8_t *)malloc((size_t)N);
    if (!member) return -1;
    int64_t B, M;
    orc_observables(dim, L, S, &B, &M);
    for (uint64_t u = 0; u < n; ++u) {
        const uint32_t t = t0 + (uint32_t)u;
        uint64_t s;
        int s0;
        const uint64_t csize = orc_cluster(dim, L, thr, seed, t, S, member, &s, &s0);
        if (csize == 0) { free(member); return -1; }
        for (uint64_t i = 0; i < N; ++i)
            if (member[i]) S[i] = (int8_t)(-S[i]);
        const int64_t M_prev = M;
        orc_observables(dim, L, S, &B, &M);
        if (M != M_prev - 2 * (int64_t)s0 * (int64_t)csize) { free(member); return -2; }
        rec[3 * u + 0] = B;
        rec[3 * u + 1] = M;
        rec[3 * u + 2] = (int64_t)csize;
    }
    free(member);
    return 0;
}

/* Raw bond draw, exposed so that tests can rebuild the activated-bond graph
 * independently of the traversal above. */
uint32_t orc_bond_draw(uint64_t seed, uint32_t t, uint32_t s, uint32_t b, int mu)
{
    uint32_t key[2], ctr[4] = {b, t, s, 0u}, r[4];
    make_key(seed, key);
    orc_philox4x32_10(ctr, key, r);
    return r[mu];
}

/* ================================================================ Potts
 * The q-state Potts model, H = -J sum_<ij> delta(s_i, s_j) with colours
 * s in {0 .. q-1}, on the same lattices.  Section 6 states that the method
 * extends to it directly; the readings taken here:
 *   - bond probability p = 1 - exp(-J / T) between equal colours, the same
 *     bond keying and threshold compare as the Ising update;
 *   - the cluster takes one new colour, uniform over the q-1 others:
 *     new = (s0 + 1 + floor(x0 (q-1) / 2^32)) mod q, x = philox((0, t, 0, 3));
 *   - initial colour of site i: floor(x0 q / 2^32), x = philox((i, 0, 0, 2));
 *   - records: B = sum_i sum_mu (q delta(s_i, s_{i+e_mu}) - 1) and
 *     M = sum_i (q delta(s_i, 0) - 1), so that E = -J (B + d N) / q.
 * With q = 2 and J_Potts = 2 J_Ising these are the Ising update, spins and
 * records exactly (colour 0 = +1, colour 1 = -1), which is one of the pins.
 * The cluster itself is grown by orc_cluster: equal colours, active bonds. */

uint32_t orc_potts_threshold(double J, double T)
{
    const double p = 1.0 - exp(-J / T);
    return scaled_threshold(p);
}

void orc_potts_init(int dim, int L, int q, uint64_t seed, int8_t *S)
{
    const uint64_t N = lattice_sites(dim, L);
    uint32_t key[2];
    make_key(seed, key);
    for (uint64_t i = 0; i < N; ++i) {
        uint32_t ctr[4] = {(uint32_t)i, 0u, 0u, 2u}, x[4];
        orc_philox4x32_10(ctr, key, x);
        S[i] = (int8_t)(((uint64_t)x[0] * (uint64_t)q) >> 32);
    }
}

/* The colour that the cluster of update t (seed colour s0) takes. */
int orc_potts_new_colour(uint64_t seed, uint32_t t, int q, int s0)
{
    uint32_t key[2], ctr[4] = {0u, t, 0u, 3u}, x[4];
    make_key(seed, key);
    orc_philox4x32_10(ctr, key, x);
    const int r = (int)(((uint64_t)x[0] * (uint64_t)(q - 1)) >> 32);
    return (s0 + 1 + r) % q;
}

void orc_potts_observables(int dim, int L, int q, const int8_t *S, int64_t *B, int64_t *M)
{
    const uint64_t N = lattice_sites(dim, L);
    int64_t b = 0, m = 0;
    for (uint64_t i = 0; i < N; ++i) {
        m += (S[i] == 0) ? q - 1 : -1;
        for (int axis = 0; axis < dim; ++axis) {
            const uint64_t k = neighbour(dim, L, i, axis, +1);
            b += (S[i] == S[k]) ? q - 1 : -1;
        }
    }
    *B = b;
    *M = m;
}

/* n Potts updates t0 .. t0+n-1 on S in place; rec as orc_run.  Returns 0,
 * -1 on allocation failure, -2 if M_after = M_before + q |C| (delta(new, 0)
 * - delta(s0, 0)) fails. */
int orc_potts_run(int dim, int L, int q, uint32_t thr, uint64_t seed, uint32_t t0, uint64_t n,
                  int8_t *S, int64_t *rec)
{
    const uint64_t N = lattice_sites(dim, L);
    uint8_t *member = (uint8_t *)malloc((size_t)N);
    if (!member) return -1;
    int64_t B, M;
    orc_potts_observables(dim, L, q, S, &B, &M);
    for (uint64_t u = 0; u < n; ++u) {
        const uint32_t t = t0 + (uint32_t)u;
        uint64_t s;
        int s0;
        const uint64_t csize = orc_cluster(dim, L, thr, seed, t, S, member, &s, &s0);
        if (csize == 0) { free(member); return -1; }
        const int c = orc_potts_new_colour(seed, t, q, s0);
        for (uint64_t i = 0; i < N; ++i) S[i] = member[i] ? (int8_t)c : S[i];
        const int64_t M_prev = M;
        orc_potts_observables(dim, L, q, S, &B, &M);
        const int64_t dz = (int64_t)(c == 0) - (int64_t)(s0 == 0);
        if (M != M_prev + (int64_t)q * (int64_t)csize * dz) { free(member); return -2; }
        rec[3 * u + 0] = B;
        rec[3 * u + 1] = M;
        rec[3 * u + 2] = (int64_t)csize;
    }
    free(member);
    return 0;
}
