// kernels_batch.hip -- launches that advance many independent lattices (jobs)
// of uneven size, model, temperature and seed together.
//
// Every job keeps its own lattice, threshold table, Philox key, sweep index
// and record ring; the launches read them from a device job table.  Because
// the random numbers depend on (seed, sweep, site) only, a job's lattice and
// records are the same alone and in any mix.
//
// Job classes (chosen by the host when a job is admitted):
//   - resident: the lattice (both colours) fits 48 KiB of LDS.  One launch per
//     call runs every resident job's sweeps of the call, one workgroup per job,
//     the whole chunk of sweeps in LDS (k_batch_resident).
//   - fused (2D): both colours of a sweep in the colour-0 launch, strips of
//     whole rows with the colour-0 halo rows recomputed, reading one copy of
//     the job's lattice and writing the other.
//   - rows (3D): one colour per launch, each colour row updated by its own
//     row group (no walk).
//   - walk / window: one colour per launch, whole-row walks down strips, or
//     64-lane column windows for rows that fit no wave.
// The non-resident classes form four kernel families, each with its own
// kernel so that its register budget is its own: half (walks and windows),
// rows of spin-1/2 jobs and rows of spin-1 jobs launch once per colour, fused
// once per sweep (all colour work of the fused jobs).  A work list names the workgroups as (job, first item) pairs in
// one segment per family, sorted by class, so a workgroup touches one job and
// its reduction goes to that job's record.  The number of valid entries and
// the offset of each segment are read from device memory, so a grid rounded
// up to a bucket size can be captured once in a graph and replayed for any
// mix whose counts fit the bucket.
//
// Per-job counters {t, record slot, sweeps in this call, current copy} live in
// a device array the host uploads once per call; the launches of the call's
// s-th sweep take s as an argument, so a job runs sweep t + s into record slot
// + s while s is below its count, and nothing runs between the sweeps to move
// the counters.
#include "batch_internal.h"
#include "row_device.hpp"
#include "rows_device.hpp"
#include "simple_device.hpp"
#include "stream_device.hpp"

namespace spinlat {

using namespace rowk;

namespace {

__device__ __forceinline__ SweepArgs job_sweep_args(const BatchJob& J, const uint32_t* dj, uint32_t colour,
                                                    uint32_t step)
{
    SweepArgs a{};
    const bool second = J.copies == 2 && ((dj[3] + step) & 1u);
    a.col[0] = second ? J.col[1][0] : J.col[0][0];
    a.col[1] = second ? J.col[1][1] : J.col[0][1];
    a.key0 = J.key0;
    a.key1 = J.key1;
    a.t = dj[0] + step;
    a.colour = colour;
    return a;
}

template <int KIND, int DIM, int D>
__device__ __forceinline__ void batch_walk_body(const BatchJob& J, const uint32_t* dj, const BatchWG w, uint32_t colour,
                                                uint32_t step, RowLuts& lut, uint32_t (&xch)[2][16][2])
{
    uint64_t thr_up, thr_down;
    build_row_luts<KIND, DIM>(lut, J.table, thr_up, thr_down);
    __syncthreads();
    const SweepArgs a = job_sweep_args(J, dj, colour, step);
    const RowGeom rg = *reinterpret_cast<const RowGeom*>(J.rg_words);
    Obs o = {0, 0, 0, 0, 0};
    const Lanes ln = lanes_of(rg, false);
    const uint32_t item = ln.slot < rg.slots ? w.item_base + ln.wave * rg.slots + ln.slot : 0xFFFFFFFFu;
    half_item<KIND, DIM, D, false>(a, rg, item, ln, lut, xch, thr_up, thr_down, o);
    int32_t bond, mag, acc, unfl;
    finish_obs<KIND, DIM>(o, bond, mag, acc, unfl);
    block_accumulate(bond, mag, acc, unfl, J.acc + (uint64_t)(dj[1] + step) * kSlotWords);
}

template <int KIND, int DIM, int D>
__device__ __forceinline__ void batch_rows_body(const BatchJob& J, const uint32_t* dj, const BatchWG w, uint32_t colour,
                                                uint32_t step, RowLuts& lut)
{
    const SweepArgs a = job_sweep_args(J, dj, colour, step);
    const RowGeom rg = *reinterpret_cast<const RowGeom*>(J.rg_words);
    Obs o = {0, 0, 0, 0, 0};
    const Lanes ln = lanes_of(rg, false);
    rows_run<KIND, DIM, D, kRagNone>(a, rg, w.item_base + ln.wave * rg.K, ln, J.table, lut, o);
    int32_t bond, mag, acc, unfl;
    finish_obs<KIND, DIM>(o, bond, mag, acc, unfl);
    block_accumulate(bond, mag, acc, unfl, J.acc + (uint64_t)(dj[1] + step) * kSlotWords);
}

// 2D jobs with two copies: the whole sweep, reading copy cur and writing the
// other.
template <int KIND, int D>
__device__ __forceinline__ void batch_fused_body(const BatchJob& J, const uint32_t* dj, const BatchWG w, uint32_t step,
                                                 RowLuts& lut, uint32_t (&xch)[2][16][4])
{
    uint64_t thr_up, thr_down;
    build_row_luts<KIND, 2>(lut, J.table, thr_up, thr_down);
    __syncthreads();
    const SweepArgs a = job_sweep_args(J, dj, 0u, step);  // the current copy
    const bool second = (dj[3] + step) & 1u;
    uint8_t* const N0 = second ? J.col[0][0] : J.col[1][0];  // the other copy
    uint8_t* const N1 = second ? J.col[0][1] : J.col[1][1];
    const RowGeom rg = *reinterpret_cast<const RowGeom*>(J.rg_words);
    Obs o = {0, 0, 0, 0, 0};
    const Lanes ln = lanes_of(rg, false);
    const uint32_t item = ln.slot < rg.slots ? w.item_base + ln.wave * rg.slots + ln.slot : 0xFFFFFFFFu;
    fused_item<KIND, D, false, 0>(a, rg, item, ln, lut, xch, thr_up, thr_down, a.col[0], a.col[1], N0, N1, o);
    int32_t bond, mag, acc, unfl;
    finish_obs<KIND, 2>(o, bond, mag, acc, unfl);
    block_accumulate(bond, mag, acc, unfl, J.acc + (uint64_t)(dj[1] + step) * kSlotWords);
}

template <int KIND, int DIM>
__device__ __forceinline__ void batch_window_body(const BatchJob& J, const uint32_t* dj, const BatchWG w,
                                                  uint32_t colour, uint32_t step, streamk::Luts& lut)
{
    uint64_t thr_up, thr_down;
    streamk::build_luts<KIND, DIM>(lut, J.table, thr_up, thr_down);
    __syncthreads();
    const SweepArgs a = job_sweep_args(J, dj, colour, step);
    const streamk::StreamGeom sg = *reinterpret_cast<const streamk::StreamGeom*>(J.rg_words);
    streamk::Obs o = {0, 0, 0, 0};
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t item = w.item_base + (threadIdx.x >> 6) * sg.G + lane / sg.W;
    streamk::stream_half_item<KIND, DIM>(a, sg, item, lut, thr_up, thr_down, o);
    block_accumulate(o.bond, o.mag, o.acc, o.unfl, J.acc + (uint64_t)(dj[1] + step) * kSlotWords);
}

union BatchLds {
    RowLuts row;
    streamk::Luts win;
};

// Kernel families: each launch runs one family's variants only, so its
// register budget is that of its own bodies.
constexpr int kFamHalf = 0, kFamRows = 1, kFamFused = 2, kFamRowsOne = 3;

template <int FAM, int KIND, int DIM>
__device__ __forceinline__ void dispatch(uint32_t v, const BatchJob& J, const uint32_t* dj, const BatchWG w,
                                         uint32_t colour, uint32_t step, BatchLds& lds, uint32_t (&xch)[2][16][4])
{
    if constexpr (FAM == kFamHalf) {
        uint32_t(&xch2)[2][16][2] = *reinterpret_cast<uint32_t(*)[2][16][2]>(&xch);
        if (v == kBvWalkD4) batch_walk_body<KIND, DIM, 4>(J, dj, w, colour, step, lds.row, xch2);
        else if (v == kBvWalkD2) batch_walk_body<KIND, DIM, 2>(J, dj, w, colour, step, lds.row, xch2);
        else if (v == kBvWalkD1) batch_walk_body<KIND, DIM, 1>(J, dj, w, colour, step, lds.row, xch2);
        else if constexpr (KIND != KIND_NE_COUPLED) {
            if (v == kBvWindow) batch_window_body<KIND, DIM>(J, dj, w, colour, step, lds.win);
        }
    } else if constexpr (FAM == kFamRows || FAM == kFamRowsOne) {
        if (v == kBvRowsD4) batch_rows_body<KIND, DIM, 4>(J, dj, w, colour, step, lds.row);
        else if (v == kBvRowsD2) batch_rows_body<KIND, DIM, 2>(J, dj, w, colour, step, lds.row);
        else if (v == kBvRowsD1) batch_rows_body<KIND, DIM, 1>(J, dj, w, colour, step, lds.row);
    } else if constexpr (DIM == 2) {
        if (v == kBvFusedD2) batch_fused_body<KIND, 2>(J, dj, w, step, lds.row, xch);
        else if (v == kBvFusedD1) batch_fused_body<KIND, 1>(J, dj, w, step, lds.row, xch);
    }
}

static_assert(kBatchKindNeCoupled == KIND_NE_COUPLED, "batch class kind of coupled NE jobs");

// One family's launch: meta = {count, offset} of the family's work-list
// segment (valid entries; the grid may be larger: a bucket size).
template <int FAM>
__global__ void __launch_bounds__(256) k_batch_family(const BatchJob* __restrict__ jobs,
                                                      const uint32_t* __restrict__ dyn,
                                                      const BatchWG* __restrict__ wgs,
                                                      const uint32_t* __restrict__ meta, uint32_t colour, uint32_t step)
{
    __shared__ BatchLds lds;
    __shared__ uint32_t xch[2][16][4];
    if (blockIdx.x >= meta[2 * FAM]) return;  // whole workgroup
    const BatchWG w = wgs[meta[2 * FAM + 1] + blockIdx.x];
    const uint32_t* dj = dyn + kDynWords * w.job;
    if (step >= dj[2]) return;  // whole workgroup: no sweep left for this job in this call
    const BatchJob& J = jobs[w.job];
    const uint32_t kind = J.cls >> 5, dim3d = (J.cls >> 4) & 1u, v = J.cls & 15u;
    if constexpr (FAM == kFamRowsOne) {
        // row groups of spin-1 jobs only (the row class is 3D)
        dispatch<FAM, KIND_ISING_ONE, 3>(v, J, dj, w, colour, step, lds, xch);
    } else if (kind == KIND_ISING_HALF) {
        if (dim3d) dispatch<FAM, KIND_ISING_HALF, 3>(v, J, dj, w, colour, step, lds, xch);
        else dispatch<FAM, KIND_ISING_HALF, 2>(v, J, dj, w, colour, step, lds, xch);
    } else if (kind == KIND_ISING_ONE) {
        if constexpr (FAM != kFamRows) {  // spin-1 row groups are family kFamRowsOne
            if (dim3d) dispatch<FAM, KIND_ISING_ONE, 3>(v, J, dj, w, colour, step, lds, xch);
            else dispatch<FAM, KIND_ISING_ONE, 2>(v, J, dj, w, colour, step, lds, xch);
        }
    } else if (kind == KIND_NE) {
        dispatch<FAM, KIND_NE, 2>(v, J, dj, w, colour, step, lds, xch);
    } else {
        dispatch<FAM, KIND_NE_COUPLED, 2>(v, J, dj, w, colour, step, lds, xch);
    }
}

// One workgroup per resident job: all of the job's sweeps of this call in LDS.
__global__ void __launch_bounds__(simplek::kResidentBlock) k_batch_resident(const BatchJob* __restrict__ jobs,
                                                                           const uint32_t* __restrict__ dyn,
                                                                           const uint32_t* __restrict__ list)
{
    extern __shared__ __align__(16) uint8_t sm[];
    __shared__ uint64_t lut[kMaxLut];
    const uint32_t j = list[blockIdx.x];
    const uint32_t* dj = dyn + kDynWords * j;
    const uint32_t n = dj[2];
    if (n == 0) return;
    const BatchJob& J = jobs[j];
    SweepArgs a = job_sweep_args(J, dj, 0u, 0u);
    const RowGeom rg = *reinterpret_cast<const RowGeom*>(J.rg_words);
    a.g.L = rg.L;
    a.g.Lh = rg.Lh;
    a.g.dim = J.dim;
    a.g.rows = J.dim == 2 ? rg.L : rg.L * rg.L;
    a.g.nh = (uint64_t)a.g.rows * rg.Lh;  // the resident geometry keeps only L and Lh
    a.lut = J.table;
    a.lut_n = (int32_t)J.table_n;
    a.acc = J.acc + (uint64_t)dj[1] * kSlotWords;
    const uint32_t kind = J.cls >> 5;
    if (kind == KIND_ISING_HALF) {
        if (J.dim == 3) simplek::resident_run<KIND_ISING_HALF, 3>(a, n, sm, lut);
        else simplek::resident_run<KIND_ISING_HALF, 2>(a, n, sm, lut);
    } else if (kind == KIND_ISING_ONE) {
        if (J.dim == 3) simplek::resident_run<KIND_ISING_ONE, 3>(a, n, sm, lut);
        else simplek::resident_run<KIND_ISING_ONE, 2>(a, n, sm, lut);
    } else {
        simplek::resident_run<KIND_NE, 2>(a, n, sm, lut);  // J = 0 or coupled (lut_n > 2)
    }
}

// One workgroup per job: sum the sub-slots of each unread record, write
// {t, bond_sum, mag, accepted, unflipped} and clear the accumulators.
__global__ void __launch_bounds__(256) k_batch_fold(const BatchFold* __restrict__ tab, int64_t* out)
{
    const BatchFold f = tab[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < f.n; i += 256) {
        unsigned long long* slot = f.ring + (uint64_t)i * kSlotWords;
        int64_t sum[kQ] = {0, 0, 0, 0};
        for (int s = 0; s < kSub; ++s)
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                sum[q] += (int64_t)slot[s * kSubStride + q];
                slot[s * kSubStride + q] = 0ull;
            }
        int64_t* o = out + (f.out_off + i) * kRecordWords;
        o[0] = (int64_t)(f.first_t + i);
        o[1] = sum[0];
        o[2] = sum[1];
        o[3] = sum[2];
        o[4] = f.ising ? -1 : sum[3];
    }
}

}  // namespace

bool batch_geom(const Geom& g, int H, bool lut32_ok, bool allow_fused, RowGeomHost& out)
{
    out = RowGeomHost{};
    static_assert(sizeof(RowGeom) <= sizeof(out.bytes), "RowGeom storage");
    static_assert(sizeof(streamk::StreamGeom) <= sizeof(out.bytes), "StreamGeom storage");
    if (lut32_ok) {
        RowGeom rg;
        if (g.dim == 3) {
            // row groups without a walk, widest D that divides the row.
            // Measured and dropped: ragged rows for batched jobs (the served
            // stream lost 6% on one box, 439 against 467 jobs/s: the rows
            // kernels then branch per job between the two updates, which
            // single lattices measured at 8%)
            for (int D : {4, 2, 1}) {
                if (!make_rows_geom(g, D, 4, rg, false)) continue;
                __builtin_memcpy(out.bytes, &rg, sizeof(RowGeom));
                out.variant = D == 4 ? kBvRowsD4 : D == 2 ? kBvRowsD2 : kBvRowsD1;
                out.nitems = rg.nitems;
                out.items_per_wg = 4 * rg.K;
                return true;
            }
        } else if (allow_fused) {
            // two or one words per lane (colour rows up to L = 1024).  Measured
            // and dropped: two ragged words per lane for Ising rows of an odd
            // word count above 64 (the served stream lost 5% against the
            // column windows)
            for (int D : {2, 1}) {
                if (!make_row_geom(g, H, D, true, rg) || rg.R > 64) continue;
                __builtin_memcpy(out.bytes, &rg, sizeof(RowGeom));
                out.variant = D == 2 ? kBvFusedD2 : kBvFusedD1;
                out.nitems = rg.nitems;
                out.items_per_wg = 4 * rg.slots;
                out.copies = 2;
                return true;
            }
        }
        // whole-row walks within one wave
        for (int D : {4, 2, 1}) {
            if (!make_row_geom(g, H, D, false, rg) || rg.R > 64) continue;
            __builtin_memcpy(out.bytes, &rg, sizeof(RowGeom));
            out.variant = D == 4 ? kBvWalkD4 : D == 2 ? kBvWalkD2 : kBvWalkD1;
            out.nitems = rg.nitems;
            out.items_per_wg = 4 * rg.slots;
            return true;
        }
    }
    // column windows
    if (g.Lh % 4) return false;
    const streamk::StreamGeom sg = streamk::make_geom(g, H, false);
    __builtin_memcpy(out.bytes, &sg, sizeof(sg));
    out.variant = kBvWindow;
    out.nitems = sg.nitems;
    out.items_per_wg = 4 * sg.G;
    return true;
}

bool batch_resident_geom(const Geom& g, RowGeomHost& out)
{
    out = RowGeomHost{};
    if (2 * g.nh > (uint64_t)kResidentLds) return false;
    RowGeom rg{};
    rg.L = g.L;
    rg.Lh = g.Lh;
    __builtin_memcpy(out.bytes, &rg, sizeof(RowGeom));
    out.variant = kBvResident;
    out.nitems = 1;
    out.items_per_wg = 1;
    return true;
}

hipError_t launch_batch_fold(const BatchFold* tab, uint32_t nentries, int64_t* out, hipStream_t s)
{
    if (nentries == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_fold, dim3(nentries), dim3(256), 0, s, tab, out);
    return hipGetLastError();
}

hipError_t launch_batch_family(int family, const BatchJob* jobs, const uint32_t* dyn, const BatchWG* wgs,
                               const uint32_t* meta, uint32_t grid, uint32_t colour, uint32_t step, hipStream_t s)
{
    if (grid == 0) return hipSuccess;
    if (family == kFamHalf)
        hipLaunchKernelGGL(k_batch_family<kFamHalf>, dim3(grid), dim3(256), 0, s, jobs, dyn, wgs, meta, colour, step);
    else if (family == kFamRows)
        hipLaunchKernelGGL(k_batch_family<kFamRows>, dim3(grid), dim3(256), 0, s, jobs, dyn, wgs, meta, colour, step);
    else if (family == kFamRowsOne)
        hipLaunchKernelGGL(k_batch_family<kFamRowsOne>, dim3(grid), dim3(256), 0, s, jobs, dyn, wgs, meta, colour,
                           step);
    else
        hipLaunchKernelGGL(k_batch_family<kFamFused>, dim3(grid), dim3(256), 0, s, jobs, dyn, wgs, meta, colour,
                           step);
    return hipGetLastError();
}

hipError_t launch_batch_resident(const BatchJob* jobs, const uint32_t* dyn, const uint32_t* list, uint32_t njobs,
                                 hipStream_t s)
{
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_resident, dim3(njobs), dim3(simplek::kResidentBlock), kResidentLds, s, jobs, dyn,
                       list);
    return hipGetLastError();
}

}  // namespace spinlat
