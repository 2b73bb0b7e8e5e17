/*
 * spinlat.h -- C ABI of the MI355X (gfx950) checkerboard Metropolis library.
 *
 * The library runs the sub-lattice-parallel ("checkerboard") Metropolis sweep
 * of "Simulating lattice spin models on GPUs" (Levy, Cohen & Rabani,
 * arXiv:1209.0296):
 *   - Ising model, Sec. 3 Eq. 1-2 with the reading H = -J sum_<ij> s_i s_j
 *     - h sum_i s_i over forward nearest-neighbour bonds of a periodic
 *     L^2 or L^3 lattice, spin-1/2 (s = +-1) or spin-1 (s in {-1,0,+1});
 *   - North-East facilitated model, Sec. 3.2 Eq. 3 with J = 0: occupation
 *     n in {0,1}, a site may change only when its north and east neighbours
 *     are up; equilibrium up-density c;
 *   - the same constraint on the Ising energy (Sec. 3.2, J != 0; model
 *     SL_NE_COUPLED): an allowed move n -> 1-n is accepted with the Metropolis
 *     probability of E = -J sum s_i s_j - h sum s_i over s = 2n - 1 (Eq. 3
 *     writes the couplings with the opposite sign: its J and B are -J and -h
 *     here), checkerboard half-sweeps, c only sets the initial density;
 *   - Metropolis acceptance min[1, exp(-dE/T)] (Sec. 3.1), evaluated as an
 *     integer compare of a 32-bit Philox4x32-10 word against a threshold
 *     table computed on the host in double precision;
 *   - one sweep = colour 0 (sites with (x+y[+z]) even) then colour 1
 *     (Alg. I steps 5-7, Fig. 3: two non-interacting sub-lattices);
 *   - the North-East model also by the paper's random sub-lattice algorithm
 *     (Sec. 3.2, model SL_NE_SUBLATTICE): square sub-lattices of B x B sites,
 *     each launch makes q = B^2 / (2 lambda) iterations per sub-lattice in
 *     which lambda random sites are updated together, two launches per sweep.
 *     Neighbours in another sub-lattice are read as at the start of the launch,
 *     neighbours in the same sub-lattice as at the start of the iteration; an
 *     accepted move sets n to 1-n, so a site drawn twice in one iteration
 *     flips once.  With B = L and lambda = 1 (not offered by the kernels) this
 *     would be the serial random-site algorithm.  The balanced variant
 *     (SL_NE_SUBLATTICE_BALANCED, end of Sec. 3.2) draws lambda sites of colour
 *     0, then lambda of colour 1 per iteration, P/(8 lambda) iterations per
 *     launch, four launches per sweep; when attempts of a half draw the same
 *     site only the lowest-numbered one is applied.
 *
 * Random-number contract (result is a pure function of seed, sweep and site,
 * so any launch schedule gives the same lattice bit for bit):
 *   word(seed, tag, t, colour, k, w, j) =
 *     Philox4x32-10(key = (seed mod 2^32, seed >> 32),
 *                   ctr = (k / G, colour, t, tag))[(k mod G)*w + j],  G = 4/w,
 *   w = 1 (spin-1/2, NE) or 2 (spin-1); tag 0 = sweep, 1 = initial state;
 *   k = (natural row-major site index) >> 1 (L even).
 *   Spin-1/2: accept s -> -s iff word < thr.  Spin-1: word j=0 accepts,
 *   word j=1 picks the proposal (lower of the two other values iff < 2^31).
 *   NE: word decides up-flips (thr = floor(min(1, c/(1-c)) 2^32)) and
 *   down-flips (floor(min(1, (1-c)/c) 2^32)).  SL_NE_COUPLED: the spin-1/2
 *   Ising threshold of the move s -> -s, s = 2n - 1, nsum over the four
 *   neighbours' 2n - 1; the move needs the north and east neighbours up.
 *   NE sub-lattices: attempt a = j*lambda + l (thread l, iteration j) on
 *   sub-lattice tau = (y0/B)*(L/B) + x0/B in launch m (m = 2t, then 2t+1) uses
 *   words 2(a mod 2) and 2(a mod 2)+1 of Philox4x32-10(key = seed,
 *   ctr = (tau, a/2, m, 2)): the first picks the site floor(word B^2 / 2^32)
 *   (row-major in the sub-lattice), the second is compared with the threshold.
 *   Balanced variant: attempt a = (2j + h)*lambda + l (half h: colour h) in
 *   launch m (4t .. 4t+3) uses words 2(a mod 2), 2(a mod 2)+1 of
 *   Philox4x32-10(key = seed, ctr = (tau, a/2, m, 3)): the first picks the site
 *   floor(word (B^2/2) / 2^32) among the sites of colour h, row by row (row r
 *   holds columns 2i + ((r + h) mod 2)), the second decides acceptance.
 *   Initial state: word(seed, 1, 0, colour, k, 1, 0): spin-1/2 +1 iff
 *   < 2^31; spin-1 floor(3 word / 2^32) - 1; NE up iff < floor(c 2^32).
 *   Threshold: thr(dE) = 2^32 if dE <= 0, else floor(exp(-dE/T) 2^32), with
 *   dE = -(double)(s'-s) * (J * (double)nsum + h) and nsum the sum of the
 *   2*dim neighbours.
 *
 * Records: record r_0 describes the state at creation; r_{i+1} the state after
 * sweep t0+i: {t, bond_sum = sum_i sum_{d<dim} s_i s_{i+e_d}, mag = sum_i s_i
 * (NE: sum_i n_i, bond_sum over n), accepted = moves accepted in that sweep
 * (NE sub-lattices: per iteration, the number of sites that changed),
 * unflipped = NE sites not flipped since the persistence origin (-1 for
 * Ising)}.  Energy: Ising E = -J bond_sum - h mag; SL_NE_COUPLED the same over
 * s = 2n - 1, i.e. E = -J (4 bond_sum - 8 mag + 2N) - h (2 mag - N).
 *
 * Ownership: the caller owns the device buffer (sl_query_bytes bytes, 256-byte
 * aligned) and the HIP stream; the handle borrows both and must be destroyed
 * before either goes away.  All device work is enqueued on that stream.
 * Errors: every function returns a status; nothing is thrown across the ABI;
 * sl_last_error() gives a thread-local message for the last failure.
 * Thread safety: one handle must not be used from two threads at once.
 */
#ifndef SPINLAT_H
#define SPINLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SL_ABI_VERSION 3u

typedef struct sl_lattice sl_lattice; /* opaque, owned by the library */

typedef enum sl_status {
    SL_OK = 0,
    SL_E_INVALID = 1,     /* a parameter is out of its domain */
    SL_E_UNSUPPORTED = 2, /* valid model, but no kernel for it (e.g. L % 8 != 0) */
    SL_E_BUFFER = 3,      /* caller buffer too small, misaligned or NULL */
    SL_E_HIP = 4,         /* a HIP runtime call failed (message has its text) */
    SL_E_STATE = 5,       /* call not allowed now (record ring full, ...) */
    SL_E_OVERFLOW = 6     /* sweep index would reach 2^32 (NE sub-lattices: 2^31,
                             balanced: 2^30) */
} sl_status;

typedef enum sl_model {
    SL_ISING = 0,
    SL_NORTH_EAST = 1,    /* NE model, checkerboard half-sweeps */
    SL_NE_SUBLATTICE = 2, /* NE model, random sub-lattice algorithm (Sec. 3.2) */
    SL_NE_SUBLATTICE_BALANCED = 3, /* its balanced variant: colour 0 then colour 1 sites
                                      per iteration, four launches per sweep */
    SL_NE_COUPLED = 4 /* NE constraint with the Ising rates of (J, h, T), checkerboard
                         half-sweeps; SL_MODE_SIMPLE, SL_MODE_RESIDENT, and SL_MODE_HALF /
                         SL_MODE_FUSED when every threshold is >= 1 */
} sl_model;

typedef enum sl_init {
    SL_INIT_COLD = 0,   /* Ising: every spin +1 */
    SL_INIT_RANDOM = 1, /* Ising: uniform over the spin values; NE: up w.p. c */
    SL_INIT_BUFFER = 2  /* copy init_spins (device, natural order) */
} sl_init;

typedef struct sl_params {
    uint32_t abi_version;     /* must be SL_ABI_VERSION */
    int32_t model;            /* sl_model; NE requires dim == 2 and two_s == 1 */
    int32_t dim;              /* 2 or 3 */
    int32_t L;                /* linear size, even, >= 2; kernels need L % 8 == 0 */
    int32_t two_s;            /* 1: s in {-1,+1}; 2: s in {-1,0,+1} */
    int32_t init;             /* sl_init */
    double J, h, T;           /* Ising (and SL_NE_COUPLED) coupling, field, temperature
                                 (T > 0, may be +inf) */
    double c;                 /* NE up-density, 0 < c < 1 (SL_NE_COUPLED: initial only) */
    uint64_t seed;            /* Philox key */
    uint64_t t0;              /* index of the first sweep (resume), < 2^32 */
    uint64_t record_capacity; /* records held on the device between sl_measure calls, >= 1 */
    const int8_t* init_spins; /* SL_INIT_BUFFER: device pointer to L^dim bytes in natural
                                 row-major order [z][y][x] (Ising: s; NE: n | flag<<1) */
    int32_t ne_side;          /* SL_NE_SUBLATTICE[_BALANCED]: sub-lattice side B in
                                 {8,16,32,64}, L % B == 0 (ignored by the other models) */
    int32_t ne_lambda;        /* SL_NE_SUBLATTICE[_BALANCED]: sites updated together, a power
                                 of two in [2, 128] with 2 lambda <= B^2 (balanced:
                                 8 lambda <= B^2); ignored otherwise */
} sl_params;

typedef struct sl_record {
    uint64_t t;
    int64_t bond_sum;
    int64_t mag;
    int64_t accepted;
    int64_t unflipped;
} sl_record;

/* Launch schedule.  Every schedule produces the same lattice and records. */
typedef enum sl_mode {
    SL_MODE_AUTO = 0,         /* library's choice for the shape */
    SL_MODE_SIMPLE = 1,       /* one thread per 4 same-colour sites, direct global loads,
                                 two launches per sweep */
    SL_MODE_HALF = 2,         /* row-group streaming, one colour in place per launch,
                                 two launches per sweep (2D and 3D) */
    SL_MODE_FUSED = 3,        /* row-group streaming, both colours in one launch per sweep
                                 with the colour-0 halo rows recomputed (2D only) */
    SL_MODE_HALF_WINDOW = 4,  /* as HALF with 64-lane column windows (any shape) */
    SL_MODE_FUSED_WINDOW = 5, /* as FUSED with 64-lane column windows and halo lanes */
    SL_MODE_RESIDENT = 6,     /* small lattices (both colours <= 48 KiB): one workgroup keeps
                                 the lattice in LDS and runs up to 4096 whole sweeps per
                                 launch; the default for lattices of at most 16 KiB */
    SL_MODE_HALF_ROWS = 7     /* one colour per launch, two launches per sweep; every colour
                                 row is updated by its own row group from vector loads of
                                 its neighbour rows, no walk; tile_rows = waves per
                                 workgroup, 1..16 (0: 4), tile_words D in {1, 2, 4} (0:
                                 widest that fits); the colour row must fit one wave:
                                 ceil(L / (8 D)) <= 64.  Ising lattices may have rows that
                                 D does not divide (then at least two lanes per row; the
                                 last lane holds the row's last D words); NE lattices need
                                 L / 8 divisible by D.  The default for 3D lattices that
                                 fit */
} sl_mode;

typedef struct sl_launch {
    int32_t mode;        /* sl_mode */
    int32_t tile_rows;   /* streaming modes: rows per strip; HALF_ROWS: waves per
                            workgroup (0: default) */
    int32_t tile_words;  /* HALF/FUSED/HALF_ROWS: 4-byte words per lane, 1, 2 or 4 (0:
                            default); must be 0 for the window modes */
    int32_t reserved;
} sl_launch;

/* Bytes of device memory the lattice needs (Alg. I steps 1-2: the lattice
 * lives in GPU memory; here two copies of both colour arrays, the per-sweep
 * record ring and the threshold table).  Host-only, pure; the caller then
 * allocates that many bytes, 256-byte aligned.  SL_E_INVALID /
 * SL_E_UNSUPPORTED / SL_E_OVERFLOW as sl_create_lattice. */
sl_status sl_query_bytes(const sl_params* params, size_t* device_bytes);

/* Threshold table the kernels use (Sec. 3.1: P_acc = min[1, exp(-dH/T)] with
 * the energy of Eq. 2 and a field; Sec. 3.2: the NE rates at up-density c),
 * as floor(P_acc 2^32) in double precision.  Host-only, pure: it takes the
 * parameters, not a lattice, so it can be read before any device work.
 * Ising and SL_NE_COUPLED: 4*(4*dim+1) entries, [di][nsum + 2*dim] for
 * s'-s = {-2,-1,+1,+2}[di]; the J = 0 NE models: {up, down}.  Each entry is in
 * [0, 2^32].  out (host, cap entries) receives them, *n_out the count;
 * SL_E_BUFFER (and *n_out set) if cap is too small. */
sl_status sl_threshold_table(const sl_params* params, uint64_t* out, size_t cap,
                             size_t* n_out);

/* Bind the caller's device buffer and stream, initialise the lattice and
 * record r_0 (Alg. I step 1: random initialisation -- done here on the GPU
 * from the counter-based words of tag 1 rather than on the CPU; Sec. 3.2: NE
 * sites up with probability c; or a copy of init_spins).  device_buf
 * (device, >= sl_query_bytes bytes, 256-byte aligned) is borrowed, never
 * freed; hip_stream is a hipStream_t (NULL: the default stream).  Work is
 * enqueued on the stream; the call synchronises once, after the table upload.
 * Errors: SL_E_INVALID (parameters), SL_E_UNSUPPORTED (no kernel for the
 * shape), SL_E_OVERFLOW (t0), SL_E_BUFFER (buffer NULL, small or misaligned),
 * SL_E_HIP. */
sl_status sl_create_lattice(const sl_params* params, void* device_buf, size_t bytes,
                            void* hip_stream, sl_lattice** out);

/* Choose the launch schedule for later sweeps (validated; SL_E_UNSUPPORTED if
 * the schedule does not fit the shape: HALF/FUSED need the colour row to split
 * into row groups of <= 64 lanes or a multiple of 64 lanes up to 1024, and for
 * spin-1/2 every threshold >= 1; the window modes take any shape).  NE
 * sub-lattice lattices have one schedule and accept only SL_MODE_AUTO;
 * SL_NE_COUPLED lattices take SL_MODE_SIMPLE, SL_MODE_RESIDENT, and the
 * whole-row modes when every threshold is >= 1.  The schedule changes speed
 * only, never a result (the random numbers are keyed by sweep and site; the
 * paper's kernel boundary between colours, Alg. I steps 6-7, is one choice of
 * barrier among several here). */
sl_status sl_set_launch(sl_lattice* lat, const sl_launch* launch);
sl_status sl_get_launch(const sl_lattice* lat, sl_launch* launch);

/* Enqueue n sweeps on the stream; asynchronous (Alg. I steps 5-7: colour 0,
 * then colour 1, a kernel end or a workgroup barrier between them; one sweep is
 * one Monte Carlo step, an attempt per site, as defined after Alg. I).  Each
 * sweep adds one record to the ring.  Fails with SL_E_STATE (nothing
 * enqueued) if the unread records would exceed record_capacity, SL_E_OVERFLOW
 * if a sweep index would reach 2^32 (NE sub-lattices 2^31, balanced 2^30);
 * both checks hold for any n, including 2^64 - 1. */
sl_status sl_sweep(sl_lattice* lat, uint64_t n);

/* Synchronise the stream and move all unread records to out[0..n) (host
 * memory, cap records).  Sec. 3.1 averages observables from lattice copies
 * the GPU sends to the host from time to time; here the sweep reduces bond
 * sum, magnetisation, accepted moves and persistence on the device every sweep
 * and this call copies only those records.  SL_E_BUFFER (nothing drained) if
 * cap is smaller than the count. */
sl_status sl_measure(sl_lattice* lat, sl_record* out, size_t cap, size_t* n_out);

/* Number of unread records and the index of the next sweep (host state, no
 * device work; either pointer may be NULL). */
sl_status sl_status_counts(const sl_lattice* lat, uint64_t* pending, uint64_t* next_t);

/* Enqueue a copy of the lattice into device_out (device, n >= L^dim bytes,
 * natural row-major order [z][y][x], NE bytes n | flag << 1).  Asynchronous;
 * the caller copies to the host if it wants one (Alg. I step 8 and Sec. 3.1:
 * the lattice is copied out from time to time; also the checkpoint that
 * SL_INIT_BUFFER with t0 resumes from).  SL_E_BUFFER if device_out is NULL or
 * n too small. */
sl_status sl_copy_spins(sl_lattice* lat, int8_t* device_out, size_t n);

/* NE (every NE model): clear every "has flipped" flag; the persistence
 * origin becomes the current sweep (the time origin of Phi(t), Eq. 4, and of
 * the persistence function the NE workloads record; the paper does not define
 * persistence, the flag is this library's reading).  Asynchronous.
 * SL_E_STATE for Ising. */
sl_status sl_reset_persistence(sl_lattice* lat);

/* Release the handle (never frees the borrowed buffer or the stream).
 * Synchronises the stream first; unread records are lost. */
sl_status sl_destroy(sl_lattice* lat);

/* Observables of n records (host-only, pure, double precision): Ising
 * E = -J bond_sum - h mag (Eq. 2 with a field), M = mag, P = NaN; NE (J = 0,
 * one unit of energy per up site, Eq. 3 read with n in {0,1}): E = mag,
 * M = mag, P = unflipped / L^dim (persistence); SL_NE_COUPLED: E the Ising
 * energy over s = 2n - 1 (see Records), M = mag, P as NE.  Any output may be
 * NULL. */
sl_status sl_record_observables(const sl_params* params, const sl_record* records, size_t n,
                                double* E, double* M, double* P);

/* ---------------------------------------------------------------------------
 * Batches: many independent lattices ("jobs") of uneven size, model,
 * temperature and seed advanced by shared launches.  Each job follows exactly
 * the sweep of a lattice created alone with the same parameters: its lattice
 * and records are identical alone and in any mix, because its random numbers
 * depend only on its seed, sweep index and site.
 *
 * The caller owns one device arena; the batch keeps its job table and work
 * lists at the start of it and places every job's lattice and record ring in
 * the rest.  A job is admitted only if its footprint (sl_batch_job_bytes) fits
 * in the free arena space; removing a job returns its space.
 * Batched jobs need L % 8 == 0 and a checkerboard model (SL_ISING,
 * SL_NORTH_EAST or SL_NE_COUPLED).  Each job gets a kernel class when it is
 * admitted:
 *   - resident: both colours fit 48 KiB; one workgroup per job runs the
 *     call's sweeps in LDS, in one launch per call for all such jobs, on a
 *     stream of the library's own that overlaps the other launches;
 *   - 2D jobs whose colour row fits one wave (and, for spin-1/2 and coupled
 *     NE, every threshold >= 1): fused sweeps (both colours in one pass, two
 *     copies of the lattice, so twice the lattice bytes);
 *   - 3D jobs that fit one wave likewise: half-sweeps by row groups;
 *   - the rest: half-sweep column windows (coupled NE jobs must fit a row
 *     class or LDS, SL_E_UNSUPPORTED otherwise).
 * The non-resident jobs of a call share launches by kernel family: one per
 * sweep for the fused jobs, one per colour for the row groups and for the
 * other half-sweep classes.  They are captured once per shape into HIP graphs
 * and replayed; the row-group family runs on another stream of the library's
 * own, beside the other families.  Every stream the library uses is joined
 * back into the caller's stream within each sl_batch_sweep call.
 * ------------------------------------------------------------------------- */
typedef struct sl_batch sl_batch;

#define SL_BATCH_NO_GRAPH 1u    /* launch the per-sweep kernels directly, no graph replay */
#define SL_BATCH_NO_FUSED 2u    /* 2D jobs take half-sweep walks instead of fused sweeps */
#define SL_BATCH_NO_RESIDENT 4u /* no resident class: small jobs run with the others */

typedef struct sl_batch_config {
    uint32_t abi_version;     /* SL_ABI_VERSION */
    uint32_t max_jobs;        /* size of the job table */
    uint32_t record_capacity; /* records each job holds between measurements (>= 2) */
    int32_t tile_rows;        /* rows per strip of the walk and fused classes (0: default) */
    uint64_t max_workgroups;  /* size of the work list (0: default 1 << 20) */
    uint32_t flags;           /* SL_BATCH_* (0: every class, graph replay) */
    uint32_t reserved;        /* 0 */
} sl_batch_config;

/* Arena bytes a job with these parameters occupies (host-only, pure). */
sl_status sl_batch_job_bytes(const sl_params* params, const sl_batch_config* cfg, size_t* bytes);

/* Arena bytes the batch itself needs before any job (host-only, pure). */
sl_status sl_batch_base_bytes(const sl_batch_config* cfg, size_t* bytes);

/* Bind the caller's device arena (256-byte aligned) and stream. */
sl_status sl_batch_create(const sl_batch_config* cfg, void* device_arena, size_t arena_bytes,
                          void* hip_stream, sl_batch** out);

/* Admit a job (params as for sl_create_lattice, record_capacity ignored) that
 * is to run `sweeps` sweeps in total.  Initialises its lattice and record r_0
 * on the stream, asynchronously (SL_INIT_BUFFER: init_spins must stay valid
 * until the stream has run the copy).  SL_E_BUFFER: not enough free arena
 * (nothing changed); SL_E_STATE: job table full; SL_E_UNSUPPORTED: no class
 * fits (e.g. L % 8 != 0); SL_E_OVERFLOW: t0 + sweeps would pass 2^32. */
sl_status sl_batch_add(sl_batch* b, const sl_params* params, uint64_t sweeps, uint32_t* job_id);

/* Enqueue up to n sweeps of every job that has sweeps left and room in its
 * record ring; jobs stop individually.  Asynchronous: the per-call counters and
 * work lists go up from double-buffered pinned staging (the host waits only if
 * the upload of the call before the previous one has not run yet).  The first
 * call of a shape captures its launches into a graph (SL_E_HIP if that
 * fails). */
sl_status sl_batch_sweep(sl_batch* b, uint64_t n);

/* Per-job counters: sweeps done, sweeps left, unread records. */
sl_status sl_batch_job_status(const sl_batch* b, uint32_t job_id, uint64_t* done,
                              uint64_t* remaining, uint64_t* pending);

/* Synchronise and move the job's unread records to out (host memory). */
sl_status sl_batch_measure(sl_batch* b, uint32_t job_id, sl_record* out, size_t cap,
                           size_t* n_out);

/* Synchronise and move the unread records of every job to out (host memory)
 * with one fold launch and one copy: the records of a job are contiguous and
 * in sweep order, job_of[i] names the job of out[i].  SL_E_BUFFER (nothing
 * drained) if cap is smaller than the total. */
sl_status sl_batch_drain(sl_batch* b, sl_record* out, uint32_t* job_of, size_t cap, size_t* n_out);

/* Enqueue a copy of a job's lattice, natural order, into device_out. */
sl_status sl_batch_copy_spins(sl_batch* b, uint32_t job_id, int8_t* device_out, size_t n);

/* Retire a job: synchronises, frees its arena space; unread records are lost. */
sl_status sl_batch_remove(sl_batch* b, uint32_t job_id);

/* Release the batch (never frees the arena).  Synchronises. */
sl_status sl_batch_destroy(sl_batch* b);

/* ---------------------------------------------------------------------------
 * Observables of a run (paper Sec. 5: magnetisation, energy and heat capacity
 * against temperature, Fig. 6; Eq. 4: the NE spin autocorrelation).
 * ------------------------------------------------------------------------- */
typedef struct sl_stats {
    uint64_t n;            /* records averaged */
    double e;              /* <e>, e = (-J bond_sum - h mag) / N, energy per site */
    double e_var;          /* <(e - <e>)^2> */
    double m;              /* <m>, m = mag / N */
    double m_abs;          /* <|m|> */
    double m2;             /* <m^2> */
    double m4;             /* <m^4> */
    double heat_capacity;  /* per site, N <(e - <e>)^2> / T^2 (k_B = 1) */
    double susceptibility; /* per site, N (<m^2> - <|m|>^2) / T */
    double binder;         /* 1 - <m^4> / (3 <m^2>^2); NaN if <m^2> = 0 */
} sl_stats;

/* Means over records[0..n) of an Ising run, or of an SL_NE_COUPLED run in its
 * spin variables s = 2n - 1 (host-only, pure, double precision; the caller
 * leaves out the records before equilibrium).  SL_E_INVALID for n == 0 or the
 * J = 0 NE models. */
sl_status sl_record_statistics(const sl_params* params, const sl_record* records, size_t n,
                               sl_stats* out);

/* Overlap sum_i v_i(t) v_i^ref of the current lattice with a reference lattice
 * (device pointer, L^dim bytes in natural order as sl_copy_spins writes them,
 * e.g. the state at the time origin): v = s for Ising, v = 2n - 1 for an NE
 * occupation n (flag bits ignored).  Synchronises the stream; the result is
 * written to *overlap on the host. */
sl_status sl_overlap(sl_lattice* lat, const int8_t* reference, int64_t* overlap);

/* NE spin autocorrelation of Eq. 4 from an overlap: Phi = (overlap / N -
 * <s>^2) / (1 - <s>^2) with <s> = 2c - 1 (host-only, pure); for SL_NE_COUPLED
 * c is the initial density, which the caller sets to the equilibrium one when
 * Phi should decay to 0.  SL_E_INVALID for Ising parameters. */
sl_status sl_autocorrelation(const sl_params* params, int64_t overlap, double* phi);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): sl_create_lattice +
 * sl_sweep(n) + sl_measure + sl_copy_spins of one lattice in one call that
 * calls no allocator, host or device.  The working memory (two copies of the
 * colour arrays, the record accumulators and the threshold table) is a
 * static device array of 33 MiB that each GPU the library runs on holds until
 * the process ends; lattices of up to 2^24 sites fit (e.g. 2D 4096^2, 3D 256^3),
 * larger ones return SL_E_UNSUPPORTED.  params as for sl_create_lattice
 * (record_capacity is ignored; SL_INIT_BUFFER reads init_spins, which may be
 * spins_out).  On the stream (a hipStream_t, NULL: the default stream) it
 * initialises the lattice, runs sweeps t0 .. t0 + n - 1 in the default
 * schedule, writes the final lattice to spins_out (device, L^dim bytes,
 * natural order as sl_copy_spins) and the records r_0 .. r_n to records_out
 * (device, n + 1 records).  Asynchronous: the outputs are valid once the
 * stream has reached this work.  Calls on one GPU share its working memory:
 * calls that overlap on one GPU (other streams, other threads) race.
 * Errors as sl_create_lattice and sl_sweep; SL_E_BUFFER if an output is NULL. */
sl_status sl_sweep_static(const sl_params* params, uint64_t n, int8_t* spins_out,
                          sl_record* records_out, void* hip_stream);

const char* sl_status_str(sl_status status);
const char* sl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPINLAT_H */
