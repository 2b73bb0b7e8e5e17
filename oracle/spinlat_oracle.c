/*
 * spinlat_oracle.c -- plain CPU oracle for the checkerboard Metropolis sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library or its
 * Python binding) may include, link or call this file; only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
 * no code, header, table or constant generator with the GPU path.
 *
 * What it computes (paper: "Simulating lattice spin models on GPUs",
 * Levy, Cohen & Rabani, arXiv:1209.0296):
 *
 *   - Sec. 3 (lattice spin models), Eq. 1-2: nearest-neighbour Ising model on a
 *     periodic square (d=2) or cubic (d=3) lattice, H = -J sum_<ij> s_i s_j
 *     - h sum_i s_i, spins s in {-1,+1} (spin-1/2) or {-1,0,+1} (spin-1).
 *   - Sec. 3.1: Metropolis acceptance P_acc = min[1, exp(-dH/T)], T in energy
 *     units, applied in the GPU algorithm's order: all sites of one
 *     sub-lattice (checkerboard colour) are updated, then the other.  The
 *     paper's four colours per 2x2 cell form two non-interacting classes
 *     (Fig. 3), i.e. the two parity classes (x+y[+z]) & 1; colour 0 first.
 *   - Sec. 3.2, Eq. 3: North-East facilitated model with J = 0: occupation
 *     n in {0,1}; a site may change only when its north and east neighbours
 *     are both up (n = 1); then the Metropolis rule applies with equilibrium
 *     up-density c (excitation energy 1, c = 1/(1+e^{1/T})).
 *   - Sec. 3.2, the NE algorithm with random sub-lattices: square sub-lattices,
 *     lambda random sites per iteration, two launches per sweep
 *     (or_ne_tiles_launch below, with its readings), and its balanced variant
 *     that alternates the two colours (or_ne_balanced_launch).
 *
 * Readings of points the paper leaves open (all documented in the design
 * notes of the repository):
 *   - sign convention: H = -J sum s_i s_j - h sum s_i (ferromagnet for J>0);
 *   - bonds: the forward-bond sum sum_i sum_{d<dim} s_i s_{i+e_d}; for L = 2
 *     this counts each neighbouring pair twice;
 *   - acceptance as an integer compare: the 32-bit uniform u is accepted iff
 *     u < thr, thr = floor(min(1, p) * 2^32) computed in double precision;
 *   - random numbers: the paper's per-thread LCG (Sec. 4, Eq. 5-7) makes the
 *     result depend on the launch schedule; it is replaced by Philox4x32-10
 *     (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as
 *     1, 2, 3", SC'11) keyed by the seed and indexed by (sweep, colour, site);
 *   - NE directions: north = (x, y-1), east = (x+1, y), rows y = 0..L-1.
 *
 * Random-number contract (both sides implement it from its definition):
 *   R(seed, tag, t, colour, k, w, j) =
 *       Philox4x32-10(key = (seed mod 2^32, seed >> 32),
 *                     ctr = (k / G, colour, t, tag))[(k mod G) * w + j],
 *   G = 4 / w; w = 1 words per site (spin-1/2, NE), w = 2 (spin-1);
 *   tag SWEEP = 0, INIT = 1; k = (natural row-major index) >> 1 is the index of
 *   the site inside its colour (L even).
 *
 * Everything here is written to be read against the paper, not to be fast:
 * one Philox evaluation per attempt, exp() per attempt, brute-force recounts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "spinlat_oracle.h"

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 3 "Philox"): a 10-round
 * Feistel-like bijection of a 128-bit counter keyed by 64 bits.  Each round
 * multiplies counter words 0 and 2 by fixed odd constants (full 64-bit
 * products), xors the high halves with the other two words and the round key,
 * and permutes; the key is bumped by the Weyl constants between rounds. */

#define OR_PHILOX_M0 0xD2511F53u
#define OR_PHILOX_M1 0xCD9E8D57u
#define OR_PHILOX_W0 0x9E3779B9u
#define OR_PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += OR_PHILOX_W0;
            k1 += OR_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)OR_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)OR_PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint32_t or_rand(uint64_t seed, uint32_t tag, uint32_t t, uint32_t colour,
                 uint64_t k, int w, int j)
{
    const uint64_t G = (uint64_t)(4 / w);
    uint32_t ctr[4] = {(uint32_t)(k / G), colour, t, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    return out[(k % G) * (uint64_t)w + (uint64_t)j];
}

/* ---------------------------------------------------------------------- */
/* Metropolis acceptance (Sec. 3.1): P_acc = min[1, exp(-dE/T)], expressed as
 * an integer threshold on a 32-bit uniform word. */

#define OR_TWO32 4294967296.0

uint64_t or_threshold_from_prob(double p)
{
    if (!(p < 1.0)) return (uint64_t)1 << 32;   /* p >= 1 (or NaN): always */
    if (!(p > 0.0)) return 0;
    double scaled = floor(p * OR_TWO32);        /* exact: scaling by 2^32 */
    return (uint64_t)scaled;
}

uint64_t or_threshold(double dE, double T)
{
    if (dE <= 0.0) return (uint64_t)1 << 32;
    return or_threshold_from_prob(exp(-dE / T));
}

/* Energy change of the move s -> sp with neighbour sum nsum (Eq. 2 with a
 * field h): dE = -(sp - s) * (J * nsum + h).  The expression and its
 * evaluation order are part of the contract, so that both sides round the
 * same way. */
double or_delta_e(double J, double h, int s, int sp, int nsum)
{
    return -(double)(sp - s) * (J * (double)nsum + h);
}

/* ---------------------------------------------------------------------- */
/* Lattice geometry: natural row-major index i = (z*L + y)*L + x. */

static inline int64_t idx3(int L, int x, int y, int z)
{
    return ((int64_t)z * L + y) * L + x;
}

/* periodic index for a in [-L, 2L): every caller steps at most one site past an edge */
static inline int wrap(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

static int nsites_dims(const or_params* p, int64_t* N)
{
    int64_t n = (int64_t)p->L * p->L;
    if (p->dim == 3) n *= p->L;
    *N = n;
    return 0;
}

int64_t or_nsites(const or_params* p)
{
    int64_t N;
    nsites_dims(p, &N);
    return N;
}

/* Sum of the 2*dim nearest neighbours of (x,y,z) (periodic). */
static int neighbour_sum(const or_params* p, const int8_t* s, int x, int y, int z)
{
    const int L = p->L;
    int zz = (p->dim == 3) ? z : 0;
    int sum = 0;
    sum += s[idx3(L, wrap(x + 1, L), y, zz)];
    sum += s[idx3(L, wrap(x - 1, L), y, zz)];
    sum += s[idx3(L, x, wrap(y + 1, L), zz)];
    sum += s[idx3(L, x, wrap(y - 1, L), zz)];
    if (p->dim == 3) {
        sum += s[idx3(L, x, y, wrap(z + 1, L))];
        sum += s[idx3(L, x, y, wrap(z - 1, L))];
    }
    return sum;
}

/* ---------------------------------------------------------------------- */
/* Initial state (Alg. I step 1: random initialisation; Sec. 3.2: NE sites up
 * with probability c).  The 32-bit word of a site is R(seed, INIT, 0, colour,
 * k, 1, 0). */

void or_init(const or_params* p, int8_t* s)
{
    const int L = p->L;
    const int nz = (p->dim == 3) ? L : 1;
    const uint64_t bern_thr = or_threshold_from_prob(p->c);
    /* every site is independent: rows are shared out among threads */
#pragma omp parallel for schedule(static) collapse(2)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int64_t i = idx3(L, x, y, z);
                uint32_t colour = (uint32_t)((x + y + z) & 1);
                uint64_t k = (uint64_t)i >> 1;
                uint32_t u = or_rand(p->seed, OR_TAG_INIT, 0, colour, k, 1, 0);
                int8_t v;
                if (p->model != OR_ISING) {
                    v = (int8_t)(((uint64_t)u < bern_thr) ? 1 : 0);
                } else if (p->init == OR_INIT_COLD) {
                    v = 1;
                } else if (p->two_s == 1) {
                    v = (int8_t)((u < 0x80000000u) ? 1 : -1);
                } else {
                    v = (int8_t)((int)(((uint64_t)u * 3u) >> 32) - 1);
                }
                s[i] = v;
            }
}

/* ---------------------------------------------------------------------- */
/* One half-sweep: every site of one colour is visited once.  Same-colour
 * sites are never neighbours, so the visiting order inside the colour does
 * not matter (Fig. 3); rows are shared out among threads. */

static int64_t half_sweep_ising(const or_params* p, int8_t* s, uint32_t t, uint32_t colour)
{
    const int L = p->L;
    const int nz = (p->dim == 3) ? L : 1;
    const int nrows = nz * L;
    const int w = (p->two_s == 1) ? 1 : 2;
    int64_t accepted = 0;
#pragma omp parallel for schedule(static) reduction(+ : accepted)
    for (int row = 0; row < nrows; ++row) {
        int z = row / L, y = row % L;
        for (int x = 0; x < L; ++x) {
            if ((uint32_t)((x + y + z) & 1) != colour) continue;
            int64_t i = idx3(L, x, y, z);
            uint64_t k = (uint64_t)i >> 1;
            int sv = s[i];
            int nsum = neighbour_sum(p, s, x, y, z);
            int sp;
            uint32_t ua;
            if (p->two_s == 1) {
                ua = or_rand(p->seed, OR_TAG_SWEEP, t, colour, k, w, 0);
                sp = -sv;
            } else {
                ua = or_rand(p->seed, OR_TAG_SWEEP, t, colour, k, w, 0);
                uint32_t up = or_rand(p->seed, OR_TAG_SWEEP, t, colour, k, w, 1);
                /* the two values other than sv, a < b; proposal uniform */
                int a, b;
                if (sv == -1) { a = 0; b = 1; }
                else if (sv == 0) { a = -1; b = 1; }
                else { a = -1; b = 0; }
                sp = (up < 0x80000000u) ? a : b;
            }
            double dE = or_delta_e(p->J, p->h, sv, sp, nsum);
            uint64_t thr = or_threshold(dE, p->T);
            if ((uint64_t)ua < thr) {
                s[i] = (int8_t)sp;
                accepted += 1;
            }
        }
    }
    return accepted;
}

/* North-East half-sweep (Sec. 3.2): a site may change only when its north and
 * east neighbours are up.  With J = 0 (OR_NORTH_EAST) the rates follow from
 * the up-density c alone.  OR_NE_COUPLED keeps the Ising energy of Eq. 2 with
 * a field, E = -J sum s_i s_j - h sum s_i over the spins s = 2n - 1, and
 * accepts an allowed move with the Metropolis probability of that energy
 * change: the thermodynamics of the Ising model under the NE constraint.
 * (Eq. 3 writes the couplings with the opposite sign: its J and B are -J and
 * -h here; J = 0, h = -1 gives the J = 0 model at the T where
 * c = e^{-1/T} / (e^{1/T} + e^{-1/T}).) */
static int64_t half_sweep_ne(const or_params* p, int8_t* s, uint32_t t, uint32_t colour)
{
    const int L = p->L;
    const int coupled = p->model == OR_NE_COUPLED;
    /* up-flip costs energy 1 (n: 0 -> 1): probability c/(1-c) capped at 1;
     * down-flip releases it: (1-c)/c capped at 1 (always, for c <= 1/2). */
    const uint64_t thr_up = or_threshold_from_prob(p->c / (1.0 - p->c));
    const uint64_t thr_down = or_threshold_from_prob((1.0 - p->c) / p->c);
    int64_t accepted = 0;
#pragma omp parallel for schedule(static) reduction(+ : accepted)
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            if ((uint32_t)((x + y) & 1) != colour) continue;
            int64_t i = idx3(L, x, y, 0);
            uint64_t k = (uint64_t)i >> 1;
            int n = s[i] & 1;
            int north = s[idx3(L, x, wrap(y - 1, L), 0)] & 1;
            int east = s[idx3(L, wrap(x + 1, L), y, 0)] & 1;
            if (!(north && east)) continue;          /* kinetic constraint */
            /* the site's word R(seed, SWEEP, t, colour, k, 1, 0) is a pure
             * function of its indices, so it is only evaluated for a move the
             * constraint allows */
            uint32_t u = or_rand(p->seed, OR_TAG_SWEEP, t, colour, k, 1, 0);
            uint64_t thr;
            if (coupled) {
                int south = s[idx3(L, x, wrap(y + 1, L), 0)] & 1;
                int west = s[idx3(L, wrap(x - 1, L), y, 0)] & 1;
                int sv = 2 * n - 1;
                int nsum = (2 * north - 1) + (2 * east - 1) + (2 * south - 1) + (2 * west - 1);
                thr = or_threshold(or_delta_e(p->J, p->h, sv, -sv, nsum), p->T);
            } else {
                thr = n ? thr_down : thr_up;
            }
            if ((uint64_t)u < thr) {
                s[i] = (int8_t)((n ^ 1) | 2);        /* new n, flag "has flipped" */
                accepted += 1;
            }
        }
    }
    return accepted;
}

int64_t or_half_sweep(const or_params* p, int8_t* s, uint32_t t, uint32_t colour)
{
    if (p->model == OR_NORTH_EAST || p->model == OR_NE_COUPLED) return half_sweep_ne(p, s, t, colour);
    if (p->model != OR_ISING) return -1;     /* no colour half-sweeps */
    return half_sweep_ising(p, s, t, colour);
}

/* ---------------------------------------------------------------------- */
/* Observables by brute force over all sites: forward-bond sum, magnetisation
 * (sum of s, or of n for NE) and the number of NE sites never flipped since
 * the persistence origin (flag bit clear). */

void or_recount(const or_params* p, const int8_t* s, int64_t out[3])
{
    const int L = p->L;
    const int nz = (p->dim == 3) ? L : 1;
    int64_t bond = 0, mag = 0, unflipped = 0;
    /* integer sums: sharing rows out among threads cannot change them */
#pragma omp parallel for schedule(static) collapse(2) reduction(+ : bond, mag, unflipped)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int64_t i = idx3(L, x, y, z);
                int v, vx, vy, vz = 0;
                if (p->model != OR_ISING) {
                    v = s[i] & 1;
                    vx = s[idx3(L, wrap(x + 1, L), y, z)] & 1;
                    vy = s[idx3(L, x, wrap(y + 1, L), z)] & 1;
                    if ((s[i] & 2) == 0) unflipped += 1;
                } else {
                    v = s[i];
                    vx = s[idx3(L, wrap(x + 1, L), y, z)];
                    vy = s[idx3(L, x, wrap(y + 1, L), z)];
                    if (p->dim == 3) vz = s[idx3(L, x, y, wrap(z + 1, L))];
                }
                bond += (int64_t)v * (vx + vy + vz);
                mag += v;
            }
    out[0] = bond;
    out[1] = mag;
    out[2] = (p->model != OR_ISING) ? unflipped : -1;
}

void or_reset_persistence(const or_params* p, int8_t* s)
{
    if (p->model == OR_ISING) return;
    int64_t N = or_nsites(p);
    for (int64_t i = 0; i < N; ++i) s[i] = (int8_t)(s[i] & 1);
}

/* ---------------------------------------------------------------------- */
/* The paper's own North-East algorithm (Sec. 3.2, Alg. NE): the lattice is cut
 * into Q square sub-lattices of P = B*B sites.  In each launch every
 * sub-lattice is processed once: q = P/(2 lambda) times, lambda sites of the
 * sub-lattice are drawn at random and updated together, then the sub-lattice
 * is synchronised.  Two launches make one sweep (q * lambda * 2 = P attempts
 * per sub-lattice).
 *
 * Readings: a neighbour that belongs to another sub-lattice (the north row
 * and east column copied with the sub-lattice) is read as it was when the
 * launch started -- the launch reads `src` and writes `dst` -- so the order in
 * which sub-lattices are processed (the paper's random assignment of
 * sub-lattices to blocks) cannot change the result; a neighbour inside the
 * same sub-lattice (including the periodic wrap when B = L, Q = 1) is read
 * live.  The lambda updates of one iteration all read the sub-lattice as it
 * was at the start of the iteration, and an accepted move sets n to 1-n (the
 * same byte for every thread that drew the site), so sites drawn twice need no
 * tie-break.  With Q = lambda = 1 this is the serial random-site Metropolis
 * algorithm.  Random numbers: attempt
 * a = j*lambda + l (thread l of iteration j) on sub-lattice tau in launch
 * `launch` uses words 2*(a mod 2) and 2*(a mod 2)+1 of
 * Philox4x32-10(key = seed, ctr = (tau, a/2, launch, 2)): the first picks the
 * site floor(word * P / 2^32) (row-major in the sub-lattice), the second
 * decides acceptance.  Sub-lattices are numbered row-major, tau = (y0/B) *
 * (L/B) + x0/B.  `accepted` counts, per iteration, the sites whose value
 * changed.  Sweep t uses launches 2t and 2t+1. */

int64_t or_ne_tiles_launch(const or_params* p, const int8_t* src, int8_t* dst, uint32_t launch)
{
    const int L = p->L, B = p->tile, lam = p->lambda;
    if (p->dim != 2 || B < 2 || lam < 1 || L % B != 0 || (B * B) % (2 * lam) != 0) return -1;
    const int P = B * B, tiles_x = L / B, q = P / (2 * lam);
    const uint64_t thr_up = or_threshold_from_prob(p->c / (1.0 - p->c));
    const uint64_t thr_down = or_threshold_from_prob((1.0 - p->c) / p->c);
    memcpy(dst, src, (size_t)L * L);
    int64_t accepted = 0;
#pragma omp parallel for schedule(static) reduction(+ : accepted)
    for (int tau = 0; tau < tiles_x * tiles_x; ++tau) {
        const int x0 = (tau % tiles_x) * B, y0 = (tau / tiles_x) * B;
        int8_t* tile = (int8_t*)malloc((size_t)P);
        int8_t* next = (int8_t*)malloc((size_t)P);
        for (int r = 0; r < B; ++r)
            for (int cc = 0; cc < B; ++cc) tile[r * B + cc] = src[idx3(L, x0 + cc, y0 + r, 0)];
        for (int j = 0; j < q; ++j) {
            memcpy(next, tile, (size_t)P);
            for (int l = 0; l < lam; ++l) {
                const uint32_t a = (uint32_t)(j * lam + l);
                uint32_t ctr[4] = {(uint32_t)tau, a / 2, launch, OR_TAG_NE_TILES};
                uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
                uint32_t w[4];
                or_philox4x32_10(ctr, key, w);
                const uint32_t site_word = w[(a % 2) * 2];
                const uint32_t acc_word = w[(a % 2) * 2 + 1];
                const int s = (int)(((uint64_t)site_word * (uint64_t)P) >> 32);
                const int r = s / B, cc = s % B;
                const int n = tile[s] & 1;
                int north, east;
                if (r > 0) north = tile[(r - 1) * B + cc] & 1;
                else if (tiles_x == 1) north = tile[(B - 1) * B + cc] & 1;
                else north = src[idx3(L, x0 + cc, wrap(y0 - 1, L), 0)] & 1;
                if (cc < B - 1) east = tile[r * B + cc + 1] & 1;
                else if (tiles_x == 1) east = tile[r * B] & 1;
                else east = src[idx3(L, wrap(x0 + B, L), y0 + r, 0)] & 1;
                if (!(north && east)) continue;
                const uint64_t thr = n ? thr_down : thr_up;
                if ((uint64_t)acc_word < thr) next[s] = (int8_t)((n ^ 1) | 2);
            }
            for (int i = 0; i < P; ++i)
                if (next[i] != tile[i]) accepted += 1;
            memcpy(tile, next, (size_t)P);
        }
        for (int r = 0; r < B; ++r)
            for (int cc = 0; cc < B; ++cc) dst[idx3(L, x0 + cc, y0 + r, 0)] = tile[r * B + cc];
        free(tile);
        free(next);
    }
    return accepted;
}

/* ---------------------------------------------------------------------- */
/* The balanced variant of the sub-lattice NE algorithm (end of Sec. 3.2): an
 * iteration updates lambda random sites of colour 0 ("red") of the
 * sub-lattice, then lambda random sites of colour 1 ("white"); four launches
 * make a sweep, each with q' = P/(8 lambda) iterations, so a sub-lattice gets P
 * attempts per sweep.
 *
 * Readings: boundaries as in or_ne_tiles_launch (other sub-lattices as at the
 * start of the launch, the own sub-lattice live).  Sites of one colour are
 * never neighbours, so the lambda updates of a half-iteration see frozen
 * neighbours.  When several attempts of a half-iteration draw the same site,
 * only the lowest-numbered one is applied: each site then gets at most one
 * Metropolis move per half-iteration, a composition of moves that each keep
 * the product measure stationary.  Random numbers: attempt
 * a = (2 j + h) lambda + l (thread l, iteration j, half h = 0 red, 1 white)
 * uses words 2 (a mod 2) and 2 (a mod 2) + 1 of Philox4x32-10(key = seed,
 * ctr = (tau, a/2, launch, 3)); the first picks the site
 * floor(word (P/2) / 2^32) among the P/2 sites of colour h, numbered row by
 * row (row r holds the columns 2i + ((r + h) mod 2)); the second decides
 * acceptance.  `accepted` counts flips.  Sweep t uses launches 4t .. 4t+3. */

int64_t or_ne_balanced_launch(const or_params* p, const int8_t* src, int8_t* dst, uint32_t launch)
{
    const int L = p->L, B = p->tile, lam = p->lambda;
    if (p->dim != 2 || B < 2 || (B & 1) || lam < 1 || L % B != 0 || (B * B) % (8 * lam) != 0)
        return -1;
    const int P = B * B, half_sites = P / 2, tiles_x = L / B, q = P / (8 * lam);
    const uint64_t thr_up = or_threshold_from_prob(p->c / (1.0 - p->c));
    const uint64_t thr_down = or_threshold_from_prob((1.0 - p->c) / p->c);
    memcpy(dst, src, (size_t)L * L);
    int64_t accepted = 0;
#pragma omp parallel for schedule(static) reduction(+ : accepted)
    for (int tau = 0; tau < tiles_x * tiles_x; ++tau) {
        const int x0 = (tau % tiles_x) * B, y0 = (tau / tiles_x) * B;
        int8_t* tile = (int8_t*)malloc((size_t)P);
        char* claimed = (char*)malloc((size_t)half_sites);
        for (int r = 0; r < B; ++r)
            for (int cc = 0; cc < B; ++cc) tile[r * B + cc] = src[idx3(L, x0 + cc, y0 + r, 0)];
        for (int j = 0; j < q; ++j)
            for (int h = 0; h < 2; ++h) {
                memset(claimed, 0, (size_t)half_sites);
                for (int l = 0; l < lam; ++l) {
                    const uint32_t a = (uint32_t)((2 * j + h) * lam + l);
                    uint32_t ctr[4] = {(uint32_t)tau, a / 2, launch, OR_TAG_NE_BALANCED};
                    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
                    uint32_t w[4];
                    or_philox4x32_10(ctr, key, w);
                    const int i = (int)(((uint64_t)w[(a % 2) * 2] * (uint64_t)half_sites) >> 32);
                    if (claimed[i]) continue;       /* a lower-numbered attempt has it */
                    claimed[i] = 1;
                    const int r = i / (B / 2);
                    const int cc = 2 * (i % (B / 2)) + ((r + h) & 1);
                    const int s = r * B + cc;
                    const int n = tile[s] & 1;
                    int north, east;
                    if (r > 0) north = tile[(r - 1) * B + cc] & 1;
                    else if (tiles_x == 1) north = tile[(B - 1) * B + cc] & 1;
                    else north = src[idx3(L, x0 + cc, wrap(y0 - 1, L), 0)] & 1;
                    if (cc < B - 1) east = tile[r * B + cc + 1] & 1;
                    else if (tiles_x == 1) east = tile[r * B] & 1;
                    else east = src[idx3(L, wrap(x0 + B, L), y0 + r, 0)] & 1;
                    if (!(north && east)) continue;
                    const uint64_t thr = n ? thr_down : thr_up;
                    if ((uint64_t)w[(a % 2) * 2 + 1] < thr) {
                        tile[s] = (int8_t)((n ^ 1) | 2);
                        accepted += 1;
                    }
                }
            }
        for (int r = 0; r < B; ++r)
            for (int cc = 0; cc < B; ++cc) dst[idx3(L, x0 + cc, y0 + r, 0)] = tile[r * B + cc];
        free(tile);
        free(claimed);
    }
    return accepted;
}

/* ---------------------------------------------------------------------- */
/* A run of n sweeps starting at sweep index t0.  Sweep t updates colour 0
 * then colour 1 (Alg. I steps 5-7: two launches per Monte Carlo step).  After
 * sweep t the record r = {t+1, bond_sum, mag, accepted, unflipped} is
 * appended (record r_0 describes the state before the first sweep). */

int or_run(const or_params* p, int8_t* s, uint32_t t0, uint32_t nsweeps,
           int64_t* records, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int8_t* tmp = NULL;
    if (p->model == OR_NE_TILES || p->model == OR_NE_BALANCED) {
        tmp = (int8_t*)malloc((size_t)p->L * p->L);
        if (!tmp) return -1;
    }
    for (uint32_t n = 0; n < nsweeps; ++n) {
        uint32_t t = t0 + n;
        int64_t acc = 0;
        if (p->model == OR_NE_BALANCED) {
            int64_t a4 = 0;
            for (uint32_t i = 0; i < 4; ++i) {
                const int64_t ai = or_ne_balanced_launch(p, (i & 1) ? tmp : s, (i & 1) ? s : tmp,
                                                         4 * t + i);
                if (ai < 0) {
                    free(tmp);
                    return -1;
                }
                a4 += ai;
            }
            acc = a4;
        } else if (p->model == OR_NE_TILES) {
            const int64_t a0 = or_ne_tiles_launch(p, s, tmp, 2 * t);
            const int64_t a1 = a0 < 0 ? -1 : or_ne_tiles_launch(p, tmp, s, 2 * t + 1);
            if (a1 < 0) {
                free(tmp);
                return -1;
            }
            acc = a0 + a1;
        } else {
            acc += or_half_sweep(p, s, t, 0);
            acc += or_half_sweep(p, s, t, 1);
        }
        if (records) {
            int64_t obs[3];
            or_recount(p, s, obs);
            int64_t* r = records + (int64_t)n * OR_RECORD_WORDS;
            r[0] = (int64_t)t + 1;
            r[1] = obs[0];
            r[2] = obs[1];
            r[3] = acc;
            r[4] = obs[2];
        }
    }
    free(tmp);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* The acceptance thresholds as a table, for comparison with the table the
 * GPU library exposes.  Ising layout: entry [di][nsum + z] for the spin change
 * ds = sp - s in {-2,-1,+1,+2} (di = 0..3) and nsum in [-z, z], z = 2*dim;
 * OR_NE_COUPLED uses the Ising layout (dim 2); the J = 0 NE layout is
 * {up-flip, down-flip}.  Returns the number of entries. */

int64_t or_threshold_table(const or_params* p, uint64_t* out, int64_t cap)
{
    if (p->model != OR_ISING && p->model != OR_NE_COUPLED) {
        if (cap < 2) return -1;
        out[0] = or_threshold_from_prob(p->c / (1.0 - p->c));
        out[1] = or_threshold_from_prob((1.0 - p->c) / p->c);
        return 2;
    }
    const int z = 2 * p->dim;
    const int ds_list[4] = {-2, -1, 1, 2};
    int64_t n = 4 * (int64_t)(2 * z + 1);
    if (cap < n) return -1;
    for (int di = 0; di < 4; ++di)
        for (int nsum = -z; nsum <= z; ++nsum) {
            /* express the move as s -> s + ds with s = 0 (dE depends on ds) */
            double dE = or_delta_e(p->J, p->h, 0, ds_list[di], nsum);
            out[di * (2 * z + 1) + (nsum + z)] = or_threshold(dE, p->T);
        }
    return n;
}

int or_abi(void) { return OR_ABI; }
