// batch.cpp -- host side of the batch ABI (include/spinlat.h, "Batches").
//
// The caller's arena holds, in order: the device job table, the per-job
// counters {t, record slot, sweeps in this call}, the work list of the batched
// kernels, a fold buffer for record readback, and a heap from which each
// job's lattice (two colour arrays) and record ring are carved first-fit.
// Admission by footprint is the heap allocation succeeding.
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

uint64_t max_wg(const sl_batch_config* c) { return c->max_workgroups ? c->max_workgroups : kDefaultMaxWG; }

struct BaseLayout {
    size_t jobs, dyn, wgs, foldtab, fold, heap;
};

BaseLayout base_layout(const sl_batch_config* c)
{
    BaseLayout b{};
    size_t off = 0;
    b.jobs = off;
    off += round_up((size_t)c->max_jobs * sizeof(BatchJob), kAlign);
    b.dyn = off;
    off += round_up((size_t)c->max_jobs * kDynWords * sizeof(uint32_t), kAlign);
    b.wgs = off;
    off += round_up((size_t)max_wg(c) * sizeof(BatchWG), kAlign);
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
    return SL_OK;
}

struct JobFoot {
    uint64_t nh;
    size_t col_bytes, ring_bytes, total;
};

JobFoot job_foot(const sl_params* p, uint32_t cap)
{
    JobFoot f{};
    const uint64_t nsites = p->dim == 2 ? (uint64_t)p->L * p->L : (uint64_t)p->L * p->L * p->L;
    f.nh = nsites / 2;
    f.col_bytes = round_up(f.nh, kAlign);
    f.ring_bytes = round_up((size_t)cap * kSlotWords * sizeof(int64_t), kAlign);
    f.total = 2 * f.col_bytes + f.ring_bytes;
    return f;
}

int default_rows(int dim) { return dim == 3 ? 4 : 8; }

struct JobHost {
    bool used = false;
    sl_params params{};
    int kind = 0;
    size_t off = 0;
    JobFoot foot{};
    RowGeomHost geom{};
    uint64_t t = 0, remaining = 0, pending = 0, first_t = 0, done = 0;
    uint64_t table[kMaxLut] = {};
    size_t table_n = 0;
};

// Kernel kind of a job's class: the model kind, with coupled NE jobs apart.
int class_kind(const JobHost& J)
{
    return J.params.model == SL_NE_COUPLED ? kBatchKindNeCoupled : J.kind;
}

}  // namespace

struct sl_batch {
    sl_batch_config cfg;
    uint8_t* arena;
    size_t arena_bytes;
    hipStream_t stream;
    BaseLayout base;
    std::vector<JobHost> jobs;
    FreeList heap;  // free ranges of the job heap
    BatchJob* h_job;     // pinned staging of one job-table entry
    uint32_t* h_dyn;     // pinned [max_jobs][kDynWords]
    BatchWG* h_wgs;      // pinned [max_wg]
    sl_record* h_stage;  // pinned [max_jobs * record_capacity]
    BatchFold* h_fold;   // pinned [max_jobs]
};

namespace {

BatchJob* d_jobs(const sl_batch* b) { return reinterpret_cast<BatchJob*>(b->arena + b->base.jobs); }
uint32_t* d_dyn(const sl_batch* b) { return reinterpret_cast<uint32_t*>(b->arena + b->base.dyn); }
BatchWG* d_wgs(const sl_batch* b) { return reinterpret_cast<BatchWG*>(b->arena + b->base.wgs); }

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

SweepArgs job_args(const sl_batch* b, uint32_t j)
{
    const JobHost& J = b->jobs[j];
    SweepArgs a{};
    a.col[0] = b->arena + J.off;
    a.col[1] = b->arena + J.off + J.foot.col_bytes;
    a.g = geom_of(&J.params, J.foot.nh);
    a.key0 = (uint32_t)J.params.seed;
    a.key1 = (uint32_t)(J.params.seed >> 32);
    a.lut = d_jobs(b)[j].table;
    a.lut_n = (int32_t)J.table_n;
    a.update = 1;
    return a;
}

unsigned long long* ring_of(const sl_batch* b, uint32_t j)
{
    const JobHost& J = b->jobs[j];
    return reinterpret_cast<unsigned long long*>(b->arena + J.off + 2 * J.foot.col_bytes);
}

sl_status check_job(const sl_batch* b, uint32_t j)
{
    if (!b) return fail(SL_E_INVALID, "NULL batch");
    if (j >= b->jobs.size() || !b->jobs[j].used) return fail(SL_E_INVALID, "no job %u", j);
    return SL_OK;
}

// Parameters of a job (record capacity from the batch) and its geometry.
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
    *foot = job_foot(p, cfg->record_capacity);
    *table_n = build_table(p, table);
    bool lut32 = true;
    for (size_t i = 0; i < *table_n; ++i)
        if (table[i] == 0) lut32 = false;
    const int H = cfg->tile_rows > 0 ? cfg->tile_rows : default_rows(p->dim);
    const bool coupled = p->model == SL_NE_COUPLED;
    const bool spin_half_table = kind_of(p) == KIND_ISING_HALF || coupled;
    if (!batch_geom(geom_of(p, foot->nh), H, lut32 || !spin_half_table, *geom))
        return fail(SL_E_UNSUPPORTED, "L = %d does not fit the batched kernels", p->L);
    if (coupled && geom->D == 0)
        return fail(SL_E_UNSUPPORTED, "batched coupled NE jobs need a colour row that fits one wave "
                                      "and every threshold >= 1 (L = %d)", p->L);
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
    b->base = base;
    b->jobs.resize(cfg->max_jobs);
    const size_t heap = round_up(base.heap, kAlign);
    b->heap.reset(heap, arena_bytes > heap ? (arena_bytes - heap) / kAlign * kAlign : 0);
    b->h_job = nullptr;
    b->h_dyn = nullptr;
    b->h_wgs = nullptr;
    b->h_stage = nullptr;
    b->h_fold = nullptr;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->h_job), sizeof(BatchJob), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_dyn),
                          (size_t)cfg->max_jobs * kDynWords * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_wgs), (size_t)max_wg(cfg) * sizeof(BatchWG),
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_stage),
                          (size_t)cfg->max_jobs * cfg->record_capacity * sizeof(sl_record), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_fold), (size_t)cfg->max_jobs * sizeof(BatchFold),
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        sl_batch_destroy(b);
        return hip_fail(e, "batch: pinned staging");
    }
    std::memset(b->h_dyn, 0, (size_t)cfg->max_jobs * kDynWords * sizeof(uint32_t));
    e = hipMemcpyAsync(d_dyn(b), b->h_dyn, (size_t)cfg->max_jobs * kDynWords * sizeof(uint32_t),
                       hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        sl_batch_destroy(b);
        return hip_fail(e, "batch: clear counters");
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
    b->jobs[j] = J;

    // device job-table entry
    BatchJob* hj = b->h_job;
    std::memset(hj, 0, sizeof(BatchJob));
    hj->col[0] = b->arena + J.off;
    hj->col[1] = b->arena + J.off + J.foot.col_bytes;
    hj->acc = ring_of(b, j);
    hj->key0 = (uint32_t)J.params.seed;
    hj->key1 = (uint32_t)(J.params.seed >> 32);
    hj->cls = batch_class(class_kind(J), J.params.dim, J.geom.D);
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
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // h_job is reused by the next add
    if (e != hipSuccess) {
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
    if (!b) return fail(SL_E_INVALID, "NULL batch");
    if (n == 0) return SL_OK;
    const uint32_t cap = b->cfg.record_capacity;
    uint32_t top = 0;       // one past the highest used job index
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

    // the work list grouped by kernel variant (kind, dim, words per lane), so
    // neighbouring workgroups of the one launch run the same code
    uint64_t nwg = 0;
    for (int kind : {(int)KIND_ISING_HALF, (int)KIND_ISING_ONE, (int)KIND_NE, kBatchKindNeCoupled})
        for (int dim : {2, 3})
            for (int D : {4, 2, 1, 0}) {
                for (uint32_t j = 0; j < top; ++j) {
                    const JobHost& J = b->jobs[j];
                    if (!J.used || !budget[j] || class_kind(J) != kind || J.params.dim != dim ||
                        J.geom.D != D)
                        continue;
                    const uint32_t per = J.geom.items_per_wg;
                    const uint32_t k = (J.geom.nitems + per - 1) / per;
                    if (nwg + k > max_wg(&b->cfg))
                        return fail(SL_E_STATE, "work list full (%llu workgroups); raise max_workgroups",
                                    (unsigned long long)max_wg(&b->cfg));
                    for (uint32_t w = 0; w < k; ++w) b->h_wgs[nwg + w] = BatchWG{j, w * per};
                    nwg += k;
                }
            }
    for (uint32_t j = 0; j < top; ++j) {
        uint32_t* d = b->h_dyn + kDynWords * j;
        const JobHost& J = b->jobs[j];
        d[0] = (uint32_t)J.t;
        d[1] = (uint32_t)J.pending;
        d[2] = J.used ? (uint32_t)budget[j] : 0u;
        d[3] = 0u;
    }
    hipError_t e = hipMemcpyAsync(d_dyn(b), b->h_dyn, (size_t)top * kDynWords * sizeof(uint32_t),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_wgs(b), b->h_wgs, nwg * sizeof(BatchWG), hipMemcpyHostToDevice, b->stream);
    // the staging buffers are rewritten by the next call: wait for the copies
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    // one launch per colour for every job (the work list is grouped by
    // variant); sweep s of the call runs sweep t + s of the jobs with more
    // than s sweeps in this call
    for (uint64_t s = 0; s < n_eff && e == hipSuccess; ++s)
        for (uint32_t colour = 0; colour < 2 && e == hipSuccess; ++colour)
            e = launch_batch_all(d_jobs(b), d_dyn(b), d_wgs(b), (uint32_t)nwg, colour, (uint32_t)s,
                                 b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch sweep");
    for (uint32_t j = 0; j < top; ++j) {
        JobHost& J = b->jobs[j];
        if (!J.used || !budget[j]) continue;
        J.t += budget[j];
        J.pending += budget[j];
        J.remaining -= budget[j];
        J.done += budget[j];
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
    if (!b) return fail(SL_E_INVALID, "NULL batch");
    if (n_out) *n_out = 0;
    uint64_t total = 0;
    uint32_t ne = 0;
    for (uint32_t j = 0; j < b->jobs.size(); ++j) {
        const JobHost& J = b->jobs[j];
        if (!J.used || J.pending == 0) continue;
        b->h_fold[ne++] = BatchFold{ring_of(b, j), total, J.first_t, (uint32_t)J.pending,
                                    J.params.model == SL_ISING ? 1u : 0u};
        total += J.pending;
    }
    if (total == 0) return SL_OK;
    if (!out || !job_of || cap < total)
        return fail(SL_E_BUFFER, "%llu records pending, buffer holds %zu", (unsigned long long)total, cap);
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
    hipError_t e = hipStreamSynchronize(b->stream);  // no queued launch may still use its memory
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
    if (b->h_job) (void)hipHostFree(b->h_job);
    if (b->h_dyn) (void)hipHostFree(b->h_dyn);
    if (b->h_wgs) (void)hipHostFree(b->h_wgs);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->h_fold) (void)hipHostFree(b->h_fold);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "batch destroy");
    return SL_OK;
}

}  // extern "C"
