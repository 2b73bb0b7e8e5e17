// batch.cpp -- host side of the batch ABI (include/spinlat.h, "Batches").
//
// The caller's arena holds, in order: the device job table, two sets of
// per-call upload areas (per-job counters {t, record slot, sweeps in this call,
// current copy}, the work list in one segment per kernel family, the count and
// offset of each segment and the list of resident jobs; calls alternate
// between the two sets), the fold table and
// buffer for record readback, and a heap from which each job's lattice (two
// colour arrays, or two copies of them for fused jobs) and record ring are
// carved first-fit.  Admission by footprint is the heap allocation succeeding.
//
// A call (sl_batch_sweep) uploads the counters and work lists from pinned
// staging (double-buffered, so the host never waits for the previous call),
// runs the resident jobs' launch on a second stream of the library's own
// while the per-sweep launches of the other jobs run on the caller's stream,
// and joins the two.  The per-sweep launches of the kernel families are
// captured once per (sweeps, grid buckets) shape into HIP graphs, each on one
// stream, and replayed; the kernels read the true segment counts from device
// memory.  The two row-group families run on a third stream of the library's,
// beside the other families (they touch disjoint jobs), so that one family's
// waves fill the issue slots another leaves idle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/spinlat.h"
#include "batch_internal.h"
#include "host_common.h"
#include "spinlat_internal.h"

using namespace spinlat;
using namespace spinlat::host;

namespace {

constexpr uint64_t kDefaultMaxWG = 1ull << 20;
constexpr size_t kGraphCache = 16;

uint64_t max_wg(const sl_batch_config* c) { return c->max_workgroups ? c->max_workgroups : kDefaultMaxWG; }

// One set of per-call device upload areas.
struct UploadLayout {
    size_t dyn, wgs, counts, res;  // offsets from the set's start
    size_t bytes;
};

UploadLayout upload_layout(const sl_batch_config* c)
{
    UploadLayout u{};
    size_t off = 0;
    u.dyn = off;
    off += round_up((size_t)c->max_jobs * kDynWords * sizeof(uint32_t), kAlign);
    u.wgs = off;
    off += round_up((size_t)max_wg(c) * sizeof(BatchWG), kAlign);
    u.counts = off;
    off += kAlign;
    u.res = off;
    off += round_up((size_t)c->max_jobs * sizeof(uint32_t), kAlign);
    u.bytes = off;
    return u;
}

struct BaseLayout {
    size_t jobs, up[2], foldtab, fold, heap;
    UploadLayout u;
};

BaseLayout base_layout(const sl_batch_config* c)
{
    BaseLayout b{};
    b.u = upload_layout(c);
    size_t off = 0;
    b.jobs = off;
    off += round_up((size_t)c->max_jobs * sizeof(BatchJob), kAlign);
    for (int k = 0; k < 2; ++k) {
        b.up[k] = off;
        off += b.u.bytes;
    }
    b.foldtab = off;
    off += round_up((size_t)c->max_jobs * sizeof(BatchFold), kAlign);
    b.fold = off;  // every job's unread records at once
    off += round_up((size_t)c->max_jobs * c->record_capacity * kRecordWords * sizeof(int64_t), kAlign);
    b.heap = off;
    return b;
}

sl_status check_config(const sl_batch_config* c)
{
    if (!c) return fail(SL_E_INVALID, "config is NULL");
    if (c->abi_version != SL_ABI_VERSION)
        return fail(SL_E_INVALID, "abi_version %u != %u", c->abi_version, SL_ABI_VERSION);
    if (c->max_jobs < 1 || c->max_jobs > (1u << 24)) return fail(SL_E_INVALID, "max_jobs out of range");
    if (c->record_capacity < 2) return fail(SL_E_INVALID, "record_capacity must be >= 2");
    if (c->tile_rows < 0) return fail(SL_E_INVALID, "tile_rows must be >= 0");
    if (c->flags & ~(uint32_t)(SL_BATCH_NO_GRAPH | SL_BATCH_NO_FUSED | SL_BATCH_NO_RESIDENT))
        return fail(SL_E_INVALID, "unknown batch flags 0x%x", c->flags);
    return SL_OK;
}

struct JobFoot {
    uint64_t nh;
    size_t col_bytes, ring_bytes, total;
};

JobFoot job_foot(const sl_params* p, uint32_t cap, uint32_t copies)
{
    JobFoot f{};
    const uint64_t nsites = p->dim == 2 ? (uint64_t)p->L * p->L : (uint64_t)p->L * p->L * p->L;
    f.nh = nsites / 2;
    f.col_bytes = round_up(f.nh, kAlign);
    f.ring_bytes = round_up((size_t)cap * kSlotWords * sizeof(int64_t), kAlign);
    f.total = 2 * copies * f.col_bytes + f.ring_bytes;
    return f;
}

int default_rows(int dim, bool fused) { return fused ? 4 : dim == 3 ? 4 : 8; }

struct JobHost {
    bool used = false;
    sl_params params{};
    int kind = 0;
    size_t off = 0;
    JobFoot foot{};
    RowGeomHost geom{};
    uint32_t cur = 0;  // copy holding the current state (fused jobs alternate)
    uint64_t t = 0, remaining = 0, pending = 0, first_t = 0, done = 0;
    uint64_t table[kMaxLut] = {};
    size_t table_n = 0;
};

bool resident_job(const JobHost& J) { return J.geom.variant == kBvResident; }
bool fused_job(const JobHost& J) { return J.geom.variant >= kBvFusedD4 && J.geom.variant <= kBvFusedD1; }

// Kernel kind of a job's class: the model kind, with coupled NE jobs apart.
int class_kind(const JobHost& J)
{
    return J.params.model == SL_NE_COUPLED ? kBatchKindNeCoupled : J.kind;
}

struct GraphEntry {
    uint64_t key;  // sweeps * 2 + upload set
    uint32_t grid[kBatchFamilies];
    hipGraphExec_t exec;
};

uint32_t bucket(uint64_t n)
{
    if (n == 0) return 0;
    uint32_t b = 64;
    while (b < n) b <<= 1;
    return b;
}

}  // namespace

struct sl_batch {
    sl_batch_config cfg;
    uint8_t* arena;
    size_t arena_bytes;
    hipStream_t stream;  // the caller's
    hipStream_t side;    // resident jobs run here, concurrently
    hipStream_t par;     // the row-group families run here, beside the others
    hipStream_t cap;     // graph capture only
    hipEvent_t ev_up[2];   // per upload set: its uploads were consumed by the launches
    hipEvent_t ev_fork, ev_join, ev_par;
    BaseLayout base;
    std::vector<JobHost> jobs;
    FreeList heap;       // free ranges of the job heap
    BatchJob* h_jobs;    // pinned [max_jobs]: one staging entry per job slot
    uint8_t* h_up[2];    // pinned upload staging, one per upload set
    sl_record* h_stage;  // pinned [max_jobs * record_capacity]
    BatchFold* h_fold;   // pinned [max_jobs]
    uint64_t calls;
    std::vector<GraphEntry> graphs;
};

namespace {

BatchJob* d_jobs(const sl_batch* b) { return reinterpret_cast<BatchJob*>(b->arena + b->base.jobs); }
uint8_t* d_up(const sl_batch* b, int k) { return b->arena + b->base.up[k]; }

Geom geom_of(const sl_params* p, uint64_t nh)
{
    Geom g;
    g.L = (uint32_t)p->L;
    g.Lh = (uint32_t)(p->L / 2);
    g.dim = (uint32_t)p->dim;
    g.rows = p->dim == 2 ? g.L : g.L * g.L;
    g.nh = nh;
    return g;
}

uint8_t* col_of(const sl_batch* b, const JobHost& J, uint32_t copy, uint32_t colour)
{
    return b->arena + J.off + (2 * copy + colour) * J.foot.col_bytes;
}

unsigned long long* ring_of(const sl_batch* b, uint32_t j)
{
    const JobHost& J = b->jobs[j];
    return reinterpret_cast<unsigned long long*>(b->arena + J.off + 2 * J.geom.copies * J.foot.col_bytes);
}

SweepArgs job_args(const sl_batch* b, uint32_t j)
{
    const JobHost& J = b->jobs[j];
    SweepArgs a{};
    a.col[0] = col_of(b, J, J.cur, 0);
    a.col[1] = col_of(b, J, J.cur, 1);
    a.g = geom_of(&J.params, J.foot.nh);
    a.key0 = (uint32_t)J.params.seed;
    a.key1 = (uint32_t)(J.params.seed >> 32);
    a.lut = d_jobs(b)[j].table;
    a.lut_n = (int32_t)J.table_n;
    a.update = 1;
    return a;
}

sl_status check_job(const sl_batch* b, uint32_t j)
{
    if (!b) return fail(SL_E_INVALID, "NULL batch");
    if (j >= b->jobs.size() || !b->jobs[j].used) return fail(SL_E_INVALID, "no job %u", j);
    return SL_OK;
}

// Parameters of a job (record capacity from the batch), its class and footprint.
sl_status prepare_job(const sl_batch_config* cfg, const sl_params* params, sl_params* p, JobFoot* foot,
                      RowGeomHost* geom, uint64_t* table, size_t* table_n)
{
    if (!params) return fail(SL_E_INVALID, "params is NULL");
    *p = *params;
    p->record_capacity = cfg->record_capacity;
    sl_status st = validate(p);
    if (st != SL_OK) return st;
    if (is_sub_lattice(p->model))
        return fail(SL_E_UNSUPPORTED, "batched jobs use the checkerboard sweep; the NE "
                                      "sub-lattice algorithm runs as a single lattice");
    *table_n = build_table(p, table);
    bool lut32 = true;
    for (size_t i = 0; i < *table_n; ++i)
        if (table[i] == 0) lut32 = false;
    const bool coupled = p->model == SL_NE_COUPLED;
    const bool spin_half_table = kind_of(p) == KIND_ISING_HALF || coupled;
    const uint64_t nh = (p->dim == 2 ? (uint64_t)p->L * p->L : (uint64_t)p->L * p->L * p->L) / 2;
    const Geom g = geom_of(p, nh);
    const bool fused = p->dim == 2 && !(cfg->flags & SL_BATCH_NO_FUSED);
    const int H = cfg->tile_rows > 0 ? cfg->tile_rows : default_rows(p->dim, fused);
    if (!(cfg->flags & SL_BATCH_NO_RESIDENT) && batch_resident_geom(g, *geom)) {
        // resident jobs run the direct update in LDS: any table
    } else if (!batch_geom(g, H, lut32 || !spin_half_table, fused, *geom)) {
        return fail(SL_E_UNSUPPORTED, "L = %d does not fit the batched kernels", p->L);
    }
    if (coupled && geom->variant == kBvWindow)
        return fail(SL_E_UNSUPPORTED, "batched coupled NE jobs need a colour row that fits one wave "
                                      "and every threshold >= 1 (L = %d), or a lattice that fits LDS", p->L);
    *foot = job_foot(p, cfg->record_capacity, geom->copies);
    return SL_OK;
}

// Per-sweep launches of one kernel family: the fused family once per sweep,
// the others once per colour.
hipError_t enqueue_family(sl_batch* b, int k, int f, uint64_t n, uint32_t grid, hipStream_t s)
{
    const UploadLayout& u = b->base.u;
    const uint32_t* dyn = reinterpret_cast<const uint32_t*>(d_up(b, k) + u.dyn);
    const BatchWG* wgs = reinterpret_cast<const BatchWG*>(d_up(b, k) + u.wgs);
    const uint32_t* meta = reinterpret_cast<const uint32_t*>(d_up(b, k) + u.counts);
    hipError_t e = hipSuccess;
    for (uint64_t s2 = 0; s2 < n && e == hipSuccess && grid; ++s2)
        for (uint32_t c = 0; c < (f == 2 ? 1u : 2u) && e == hipSuccess; ++c)
            e = launch_batch_family(f, d_jobs(b), dyn, wgs, meta, grid, c, (uint32_t)s2, s);
    return e;
}

// The per-sweep launches of the shape (n, grids) on upload set k as a graph,
// captured on first use.
sl_status graph_for(sl_batch* b, int k, uint64_t n, const uint32_t (&grid)[kBatchFamilies], hipGraphExec_t* out)
{
    const uint64_t key = n * 2 + (uint64_t)k;
    for (size_t i = 0; i < b->graphs.size(); ++i)
        if (b->graphs[i].key == key && std::equal(grid, grid + kBatchFamilies, b->graphs[i].grid)) {
            // most recently used last: eviction takes the front
            const GraphEntry g = b->graphs[i];
            b->graphs.erase(b->graphs.begin() + (long)i);
            b->graphs.push_back(g);
            *out = g.exec;
            return SL_OK;
        }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "batch: begin graph capture");
    hipError_t le = hipSuccess;
    for (int f = 0; f < kBatchFamilies && le == hipSuccess; ++f) le = enqueue_family(b, k, f, n, grid[f], b->cap);
    e = hipStreamEndCapture(b->cap, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le != hipSuccess ? le : e, "batch: graph capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "batch: graph instantiate");
    if (b->graphs.size() >= kGraphCache) {
        // the least recently used graph may still run: wait before destroying
        // it (graphs of earlier calls run on the caller's stream or on par,
        // which the caller's stream joins at the end of every call)
        e = hipStreamSynchronize(b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->par);
        if (e != hipSuccess) return hip_fail(e, "batch: synchronise before graph eviction");
        (void)hipGraphExecDestroy(b->graphs.front().exec);
        b->graphs.erase(b->graphs.begin());
    }
    GraphEntry ge{key, {}, exec};
    std::copy(grid, grid + kBatchFamilies, ge.grid);
    b->graphs.push_back(ge);
    *out = exec;
    return SL_OK;
}

}  // namespace

extern "C" {

sl_status sl_batch_base_bytes(const sl_batch_config* cfg, size_t* bytes)
{
    sl_status st = check_config(cfg);
    if (st != SL_OK) return st;
    if (!bytes) return fail(SL_E_INVALID, "bytes is NULL");
    *bytes = base_layout(cfg).heap;
    return SL_OK;
}

sl_status sl_batch_job_bytes(const sl_params* params, const sl_batch_config* cfg, size_t* bytes)
{
    sl_status st = check_config(cfg);
    if (st != SL_OK) return st;
    if (!bytes) return fail(SL_E_INVALID, "bytes is NULL");
    sl_params p;
    JobFoot foot;
    RowGeomHost geom;
    uint64_t table[kMaxLut];
    size_t tn;
    st = prepare_job(cfg, params, &p, &foot, &geom, table, &tn);
    if (st != SL_OK) return st;
    *bytes = foot.total;
    return SL_OK;
}

sl_status sl_batch_create(const sl_batch_config* cfg, void* device_arena, size_t arena_bytes,
                          void* hip_stream, sl_batch** out)
{
    sl_status st = check_config(cfg);
    if (st != SL_OK) return st;
    if (!out) return fail(SL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!device_arena || reinterpret_cast<uintptr_t>(device_arena) % kAlign)
        return fail(SL_E_BUFFER, "arena must be non-NULL and %zu-byte aligned", kAlign);
    const BaseLayout base = base_layout(cfg);
    if (arena_bytes < base.heap)
        return fail(SL_E_BUFFER, "arena has %zu bytes, the batch needs %zu before any job", arena_bytes,
                    base.heap);
    sl_batch* b = new (std::nothrow) sl_batch();
    if (!b) return fail(SL_E_STATE, "out of host memory");
    b->cfg = *cfg;
    b->arena = static_cast<uint8_t*>(device_arena);
    b->arena_bytes = arena_bytes;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->side = nullptr;
    b->par = nullptr;
    b->cap = nullptr;
    b->ev_up[0] = b->ev_up[1] = nullptr;
    b->ev_fork = b->ev_join = b->ev_par = nullptr;
    b->base = base;
    b->jobs.resize(cfg->max_jobs);
    const size_t heap = round_up(base.heap, kAlign);
    b->heap.reset(heap, arena_bytes > heap ? (arena_bytes - heap) / kAlign * kAlign : 0);
    b->h_jobs = nullptr;
    b->h_up[0] = b->h_up[1] = nullptr;
    b->h_stage = nullptr;
    b->h_fold = nullptr;
    b->calls = 0;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->h_jobs), (size_t)cfg->max_jobs * sizeof(BatchJob),
                                 hipHostMallocDefault);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_up[k]), base.u.bytes, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_stage),
                          (size_t)cfg->max_jobs * cfg->record_capacity * sizeof(sl_record), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_fold), (size_t)cfg->max_jobs * sizeof(BatchFold),
                          hipHostMallocDefault);
    // the library's own streams keep the default priority
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->par, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&b->ev_up[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_par, hipEventDisableTiming);
    if (e != hipSuccess) {
        sl_batch_destroy(b);
        return hip_fail(e, "batch: pinned staging, streams and events");
    }
    *out = b;
    return SL_OK;
}

sl_status sl_batch_add(sl_batch* b, const sl_params* params, uint64_t sweeps, uint32_t* job_id)
{
    if (!b) return fail(SL_E_INVALID, "NULL batch");
    if (!job_id) return fail(SL_E_INVALID, "job_id is NULL");
    JobHost J;
    sl_status st = prepare_job(&b->cfg, params, &J.params, &J.foot, &J.geom, J.table, &J.table_n);
    if (st != SL_OK) return st;
    if (sweeps > (1ull << 32) - J.params.t0)  // validate() keeps t0 < 2^32
        return fail(SL_E_OVERFLOW, "t0 + sweeps would pass 2^32");
    uint32_t j = 0;
    while (j < b->jobs.size() && b->jobs[j].used) ++j;
    if (j == b->jobs.size()) return fail(SL_E_STATE, "job table full (%u jobs)", b->cfg.max_jobs);
    if (!b->heap.alloc(J.foot.total, &J.off))
        return fail(SL_E_BUFFER, "arena has no free block of %zu bytes for this job", J.foot.total);
    J.used = true;
    J.kind = kind_of(&J.params);
    J.t = J.params.t0;
    J.first_t = J.params.t0;
    J.remaining = sweeps;
    J.cur = 0;
    b->jobs[j] = J;

    // device job-table entry, staged in this slot's own pinned entry: the
    // slot is rewritten only after sl_batch_remove, which synchronises
    BatchJob* hj = b->h_jobs + j;
    std::memset(hj, 0, sizeof(BatchJob));
    for (uint32_t cp = 0; cp < J.geom.copies; ++cp)
        for (uint32_t c = 0; c < 2; ++c) hj->col[cp][c] = col_of(b, J, cp, c);
    hj->acc = ring_of(b, j);
    hj->key0 = (uint32_t)J.params.seed;
    hj->key1 = (uint32_t)(J.params.seed >> 32);
    hj->cls = batch_class(class_kind(J), J.params.dim, J.geom.variant);
    hj->copies = J.geom.copies;
    hj->dim = (uint32_t)J.params.dim;
    hj->table_n = (uint32_t)J.table_n;
    std::memcpy(hj->rg_words, J.geom.bytes, sizeof(hj->rg_words));
    std::memcpy(hj->table, J.table, J.table_n * sizeof(uint64_t));
    hipError_t e = hipMemcpyAsync(d_jobs(b) + j, hj, sizeof(BatchJob), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = launch_fill_u64(ring_of(b, j), (uint64_t)b->cfg.record_capacity * kSlotWords, b->stream);
    SweepArgs a = job_args(b, j);
    if (e == hipSuccess) {
        if (J.params.init == SL_INIT_BUFFER) {
            e = launch_from_natural(a, J.params.init_spins, b->stream);
        } else {
            const uint64_t bern = thr_from_prob(J.params.c);
            e = launch_init(a, J.kind, J.params.init == SL_INIT_COLD ? 0 : 1, (uint32_t)bern,
                            (uint32_t)(bern >> 32), b->stream);
        }
    }
    // record r_0: observables of the initial state
    a.update = 0;
    a.acc = ring_of(b, j);
    for (uint32_t c = 0; c < 2 && e == hipSuccess; ++c) {
        a.colour = c;
        e = launch_simple_half(a, J.kind, b->stream);
    }
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(b->stream);
        b->heap.release(J.off, J.foot.total);
        b->jobs[j] = JobHost();
        return hip_fail(e, "batch add");
    }
    b->jobs[j].pending = 1;
    *job_id = j;
    return SL_OK;
}

sl_status sl_batch_sweep(sl_batch* b, uint64_t n)
{
    const TraceRange range("sl_batch_sweep");
    if (!b) return fail(SL_E_INVALID, "NULL batch");
    if (n == 0) return SL_OK;
    const uint32_t cap = b->cfg.record_capacity;
    uint32_t top = 0;  // one past the highest used job index
    uint64_t n_eff = 0;
    std::vector<uint64_t> budget(b->jobs.size(), 0);
    for (uint32_t j = 0; j < b->jobs.size(); ++j) {
        const JobHost& J = b->jobs[j];
        if (!J.used) continue;
        top = j + 1;
        const uint64_t room = cap > J.pending ? cap - J.pending : 0;
        budget[j] = std::min<uint64_t>(std::min<uint64_t>(n, J.remaining), room);
        n_eff = std::max(n_eff, budget[j]);
    }
    if (n_eff == 0) return SL_OK;

    // this call's upload set; wait until the launches that read it last (two
    // calls ago) have been enqueued past its upload
    const int k = (int)(b->calls & 1u);
    hipError_t e = hipEventSynchronize(b->ev_up[k]);
    if (e != hipSuccess) return hip_fail(e, "batch: wait for staging");
    const UploadLayout& u = b->base.u;
    uint8_t* hu = b->h_up[k];
    uint32_t* h_dyn = reinterpret_cast<uint32_t*>(hu + u.dyn);
    BatchWG* h_wgs = reinterpret_cast<BatchWG*>(hu + u.wgs);
    uint32_t* h_counts = reinterpret_cast<uint32_t*>(hu + u.counts);
    uint32_t* h_res = reinterpret_cast<uint32_t*>(hu + u.res);

    // work list: one segment per kernel family, each grouped by class so
    // neighbouring workgroups run the same code; resident jobs in their own list
    uint64_t nwg = 0, nres = 0;
    uint32_t count[kBatchFamilies] = {}, offset[kBatchFamilies] = {};
    for (int fam = 0; fam < kBatchFamilies; ++fam) {
        offset[fam] = (uint32_t)nwg;
        for (uint32_t kind : {(uint32_t)KIND_ISING_HALF, (uint32_t)KIND_ISING_ONE, (uint32_t)KIND_NE,
                              (uint32_t)kBatchKindNeCoupled})
            for (int dim : {2, 3})
                for (uint32_t v = 0; v < 16; ++v) {
                    if (v == kBvResident || batch_family(v, kind) != fam) continue;
                    for (uint32_t j = 0; j < top; ++j) {
                        const JobHost& J = b->jobs[j];
                        if (!J.used || !budget[j] || (uint32_t)class_kind(J) != kind || J.params.dim != dim ||
                            J.geom.variant != v)
                            continue;
                        const uint32_t per = J.geom.items_per_wg;
                        const uint32_t kwg = (J.geom.nitems + per - 1) / per;
                        if (nwg + kwg > max_wg(&b->cfg))
                            return fail(SL_E_STATE, "work list full (%llu workgroups); raise max_workgroups",
                                        (unsigned long long)max_wg(&b->cfg));
                        for (uint32_t w = 0; w < kwg; ++w) h_wgs[nwg + w] = BatchWG{j, w * per};
                        nwg += kwg;
                    }
                }
        count[fam] = (uint32_t)nwg - offset[fam];
    }
    for (uint32_t j = 0; j < top; ++j) {
        const JobHost& J = b->jobs[j];
        uint32_t* d = h_dyn + kDynWords * j;
        d[0] = (uint32_t)J.t;
        d[1] = (uint32_t)J.pending;
        d[2] = J.used ? (uint32_t)budget[j] : 0u;
        d[3] = J.cur;
        if (J.used && budget[j] && resident_job(J)) h_res[nres++] = j;
    }
    for (int f = 0; f < kBatchFamilies; ++f) {
        h_counts[2 * f] = count[f];
        h_counts[2 * f + 1] = offset[f];
    }
    uint8_t* du = d_up(b, k);
    e = hipMemcpyAsync(du + u.dyn, h_dyn, (size_t)top * kDynWords * sizeof(uint32_t), hipMemcpyHostToDevice,
                       b->stream);
    if (e == hipSuccess && nwg)
        e = hipMemcpyAsync(du + u.wgs, h_wgs, nwg * sizeof(BatchWG), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(du + u.counts, h_counts, 2 * kBatchFamilies * sizeof(uint32_t), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess && nres)
        e = hipMemcpyAsync(du + u.res, h_res, nres * sizeof(uint32_t), hipMemcpyHostToDevice, b->stream);
    // the staging of set k may be rewritten once these copies have run
    if (e == hipSuccess) e = hipEventRecord(b->ev_up[k], b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch: upload");
    ++b->calls;

    // the row-group families get a stream of their own when another family runs
    bool par_work = false, main_work = false;
    for (int f = 0; f < kBatchFamilies; ++f) (row_family(f) ? par_work : main_work) |= count[f] != 0;
    const bool split = par_work && main_work;
    if (nres || split) {
        e = hipEventRecord(b->ev_fork, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch: fork");
    }
    // resident jobs: one launch on the side stream, overlapping the rest
    if (nres) {
        e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
        if (e == hipSuccess)
            e = launch_batch_resident(d_jobs(b), reinterpret_cast<const uint32_t*>(du + u.dyn),
                                      reinterpret_cast<const uint32_t*>(du + u.res), (uint32_t)nres, b->side);
        if (e == hipSuccess) e = hipEventRecord(b->ev_join, b->side);
        if (e != hipSuccess) return hip_fail(e, "batch: resident launch");
    }
    // the other jobs: n_eff sweeps of per-family launches, replayed from a graph
    if (nwg) {
        // grids per stream: a family with grid 0 is not launched
        uint32_t g_main[kBatchFamilies], g_par[kBatchFamilies] = {};
        for (int f = 0; f < kBatchFamilies; ++f) g_main[f] = bucket(count[f]);
        if (split) {
            for (int f = 0; f < kBatchFamilies; ++f)
                if (row_family(f)) {
                    g_par[f] = g_main[f];
                    g_main[f] = 0;
                }
            e = hipStreamWaitEvent(b->par, b->ev_fork, 0);
            if (e != hipSuccess) return hip_fail(e, "batch: fork");
        }
        if (b->cfg.flags & SL_BATCH_NO_GRAPH) {
            for (int f = 0; f < kBatchFamilies && e == hipSuccess; ++f) {
                if (g_par[f]) e = enqueue_family(b, k, f, n_eff, g_par[f], b->par);
                if (e == hipSuccess && g_main[f]) e = enqueue_family(b, k, f, n_eff, g_main[f], b->stream);
            }
            if (e != hipSuccess) return hip_fail(e, "batch sweep");
        } else {
            // both graphs first (a lookup never evicts the graph it returns or
            // one used since), then the launches
            hipGraphExec_t x_par = nullptr, x_main = nullptr;
            sl_status gs = split ? graph_for(b, k, n_eff, g_par, &x_par) : SL_OK;
            if (gs == SL_OK && std::any_of(g_main, g_main + kBatchFamilies, [](uint32_t g) { return g != 0; }))
                gs = graph_for(b, k, n_eff, g_main, &x_main);
            if (gs != SL_OK) return gs;
            if (x_par) e = hipGraphLaunch(x_par, b->par);
            if (e == hipSuccess && x_main) e = hipGraphLaunch(x_main, b->stream);
            if (e != hipSuccess) return hip_fail(e, "batch: graph launch");
        }
        if (split) {
            e = hipEventRecord(b->ev_par, b->par);
            if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_par, 0);
            if (e != hipSuccess) return hip_fail(e, "batch: join the row-group stream");
        }
    }
    if (nres) {
        e = hipStreamWaitEvent(b->stream, b->ev_join, 0);
        if (e != hipSuccess) return hip_fail(e, "batch: join resident launch");
    }
    for (uint32_t j = 0; j < top; ++j) {
        JobHost& J = b->jobs[j];
        if (!J.used || !budget[j]) continue;
        J.t += budget[j];
        J.pending += budget[j];
        J.remaining -= budget[j];
        J.done += budget[j];
        if (fused_job(J)) J.cur ^= (uint32_t)(budget[j] & 1u);
    }
    return SL_OK;
}

sl_status sl_batch_job_status(const sl_batch* b, uint32_t job_id, uint64_t* done, uint64_t* remaining,
                              uint64_t* pending)
{
    sl_status st = check_job(b, job_id);
    if (st != SL_OK) return st;
    const JobHost& J = b->jobs[job_id];
    if (done) *done = J.done;
    if (remaining) *remaining = J.remaining;
    if (pending) *pending = J.pending;
    return SL_OK;
}

sl_status sl_batch_measure(sl_batch* b, uint32_t job_id, sl_record* out, size_t cap, size_t* n_out)
{
    sl_status st = check_job(b, job_id);
    if (st != SL_OK) return st;
    if (n_out) *n_out = 0;
    JobHost& J = b->jobs[job_id];
    const uint64_t n = J.pending;
    if (n == 0) return SL_OK;
    if (!out || cap < n)
        return fail(SL_E_BUFFER, "%llu records pending, buffer holds %zu", (unsigned long long)n, cap);
    int64_t* fold = reinterpret_cast<int64_t*>(b->arena + b->base.fold);
    hipError_t e = launch_fold(ring_of(b, job_id), fold, n, J.first_t, J.params.model == SL_ISING ? 1 : 0,
                               b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_stage, fold, n * sizeof(sl_record), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch measure");
    std::memcpy(out, b->h_stage, n * sizeof(sl_record));
    J.first_t += n;
    J.pending = 0;
    if (n_out) *n_out = n;
    return SL_OK;
}

sl_status sl_batch_drain(sl_batch* b, sl_record* out, uint32_t* job_of, size_t cap, size_t* n_out)
{
    const TraceRange range("sl_batch_drain");
    if (!b) return fail(SL_E_INVALID, "NULL batch");
    if (n_out) *n_out = 0;
    uint64_t total = 0;
    uint32_t ne = 0;
    for (uint32_t j = 0; j < b->jobs.size(); ++j) {
        const JobHost& J = b->jobs[j];
        if (!J.used || J.pending == 0) continue;
        total += J.pending;
    }
    if (total == 0) return SL_OK;
    if (!out || !job_of || cap < total)
        return fail(SL_E_BUFFER, "%llu records pending, buffer holds %zu", (unsigned long long)total, cap);
    // the fold table's staging is reused by every drain: the previous drain
    // synchronised before returning, so its copy has run
    total = 0;
    for (uint32_t j = 0; j < b->jobs.size(); ++j) {
        const JobHost& J = b->jobs[j];
        if (!J.used || J.pending == 0) continue;
        b->h_fold[ne++] = BatchFold{ring_of(b, j), total, J.first_t, (uint32_t)J.pending,
                                    J.params.model == SL_ISING ? 1u : 0u};
        total += J.pending;
    }
    BatchFold* dtab = reinterpret_cast<BatchFold*>(b->arena + b->base.foldtab);
    int64_t* fold = reinterpret_cast<int64_t*>(b->arena + b->base.fold);
    hipError_t e = hipMemcpyAsync(dtab, b->h_fold, ne * sizeof(BatchFold), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = launch_batch_fold(dtab, ne, fold, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_stage, fold, total * sizeof(sl_record), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch drain");
    std::memcpy(out, b->h_stage, total * sizeof(sl_record));
    uint64_t k = 0;
    for (uint32_t j = 0; j < b->jobs.size(); ++j) {
        JobHost& J = b->jobs[j];
        if (!J.used || J.pending == 0) continue;
        for (uint64_t i = 0; i < J.pending; ++i) job_of[k++] = j;
        J.first_t += J.pending;
        J.pending = 0;
    }
    if (n_out) *n_out = total;
    return SL_OK;
}

sl_status sl_batch_copy_spins(sl_batch* b, uint32_t job_id, int8_t* device_out, size_t n)
{
    sl_status st = check_job(b, job_id);
    if (st != SL_OK) return st;
    const JobHost& J = b->jobs[job_id];
    if (!device_out || n < 2 * J.foot.nh)
        return fail(SL_E_BUFFER, "copy_spins needs %llu bytes", (unsigned long long)(2 * J.foot.nh));
    hipError_t e = launch_to_natural(job_args(b, job_id), device_out, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch copy_spins");
    return SL_OK;
}

sl_status sl_batch_remove(sl_batch* b, uint32_t job_id)
{
    sl_status st = check_job(b, job_id);
    if (st != SL_OK) return st;
    // no queued launch may still use its memory (resident launches join the
    // caller's stream)
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch remove");
    JobHost& J = b->jobs[job_id];
    b->heap.release(J.off, J.foot.total);
    J = JobHost();
    return SL_OK;
}

sl_status sl_batch_destroy(sl_batch* b)
{
    if (!b) return fail(SL_E_INVALID, "NULL batch");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    if (b->par) (void)hipStreamSynchronize(b->par);
    for (GraphEntry& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    for (int k = 0; k < 2; ++k)
        if (b->ev_up[k]) (void)hipEventDestroy(b->ev_up[k]);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->ev_par) (void)hipEventDestroy(b->ev_par);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->par) (void)hipStreamDestroy(b->par);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->h_jobs) (void)hipHostFree(b->h_jobs);
    for (int k = 0; k < 2; ++k)
        if (b->h_up[k]) (void)hipHostFree(b->h_up[k]);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->h_fold) (void)hipHostFree(b->h_fold);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "batch destroy");
    return SL_OK;
}

}  // extern "C"
