// kernels_batch.hip -- one launch advances a half-sweep of many independent
// lattices (jobs) of uneven size, model, temperature and seed.
//
// Every job keeps its own lattice, threshold table, Philox key, sweep index
// and record ring; the launch reads them from a device job table.  A work
// list names the workgroups to run as (job, first item) pairs, sorted by the
// job's kernel variant (model kind, dimension, words per lane), so a
// workgroup only ever touches one job and its reduction goes to that job's
// record.  Because the random numbers depend on (seed, sweep, site) only, a
// job's lattice and records are the same alone and in any mix.
//
// Per-job counters {t, record slot, sweeps in this call} live in a small
// device array that the host uploads once per call; the launches of the
// call's s-th sweep take s as an argument, so a job runs sweep t + s into
// record slot + s while s is below its count, and nothing runs between the
// sweeps to move the counters.
#include "row_device.hpp"
#include "stream_device.hpp"
#include "batch_internal.h"

namespace spinlat {

using namespace rowk;

namespace {

template <int KIND, int DIM, int D>
__device__ __forceinline__ void batch_half_body(const BatchJob* __restrict__ jobs, const uint32_t* __restrict__ dyn,
                                                const BatchWG w, uint32_t colour, uint32_t step,
                                                RowLuts& lut, uint32_t (&xch)[2][16][2])
{
    const uint32_t* dj = dyn + kDynWords * w.job;
    if (step >= dj[2]) return;  // whole workgroup: this job has no sweep left in this call
    const BatchJob& J = jobs[w.job];
    uint64_t thr_up, thr_down;
    build_row_luts<KIND, DIM>(lut, J.table, thr_up, thr_down);
    __syncthreads();

    SweepArgs a{};
    a.col[0] = J.col[0];
    a.col[1] = J.col[1];
    a.key0 = J.key0;
    a.key1 = J.key1;
    a.t = dj[0] + step;
    a.colour = colour;
    const RowGeom rg = *reinterpret_cast<const RowGeom*>(J.rg_words);
    Obs o = {0, 0, 0, 0, 0};
    const Lanes ln = lanes_of(rg, false);
    const uint32_t slot_in_wave = ln.lane / rg.R;
    const uint32_t item = slot_in_wave < rg.slots
                              ? w.item_base + ln.wave * rg.slots + slot_in_wave
                              : 0xFFFFFFFFu;
    half_item<KIND, DIM, D, false>(a, rg, item, ln, lut, xch, thr_up, thr_down, o);
    int32_t bond, mag, acc, unfl;
    finish_obs<KIND, DIM>(o, bond, mag, acc, unfl);
    block_accumulate(bond, mag, acc, unfl, J.acc + (uint64_t)(dj[1] + step) * kSlotWords);
}

// Jobs whose colour row does not fit one wave (or whose spin-1/2 table has a
// zero threshold): 64-lane column windows with edge loads (any L % 8 == 0).
template <int KIND, int DIM>
__device__ __forceinline__ void batch_window_body(const BatchJob* __restrict__ jobs,
                                                  const uint32_t* __restrict__ dyn, const BatchWG w,
                                                  uint32_t colour, uint32_t step, streamk::Luts& lut)
{
    const uint32_t* dj = dyn + kDynWords * w.job;
    if (step >= dj[2]) return;  // whole workgroup: no sweep left for this job
    const BatchJob& J = jobs[w.job];
    uint64_t thr_up, thr_down;
    streamk::build_luts<KIND, DIM>(lut, J.table, thr_up, thr_down);
    __syncthreads();

    SweepArgs a{};
    a.col[0] = J.col[0];
    a.col[1] = J.col[1];
    a.key0 = J.key0;
    a.key1 = J.key1;
    a.t = dj[0] + step;
    a.colour = colour;
    const streamk::StreamGeom sg = *reinterpret_cast<const streamk::StreamGeom*>(J.rg_words);
    streamk::Obs o = {0, 0, 0, 0};
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t item = w.item_base + (threadIdx.x >> 6) * sg.G + lane / sg.W;
    streamk::stream_half_item<KIND, DIM>(a, sg, item, lut, thr_up, thr_down, o);
    block_accumulate(o.bond, o.mag, o.acc, o.unfl, J.acc + (uint64_t)(dj[1] + step) * kSlotWords);
}

// Every job of a half-sweep in one launch: each workgroup runs the variant of
// its job (the work list is sorted by variant, so neighbouring workgroups run
// the same code).
union BatchLds {
    RowLuts row;
    streamk::Luts win;
};

template <int KIND, int DIM>
__device__ __forceinline__ void dispatch_d(uint32_t d, const BatchJob* jobs, const uint32_t* dyn, const BatchWG w,
                                           uint32_t colour, uint32_t step, BatchLds& lds,
                                           uint32_t (&xch)[2][16][2])
{
    if (d == 0) batch_half_body<KIND, DIM, 4>(jobs, dyn, w, colour, step, lds.row, xch);
    else if (d == 1) batch_half_body<KIND, DIM, 2>(jobs, dyn, w, colour, step, lds.row, xch);
    else if (d == 2) batch_half_body<KIND, DIM, 1>(jobs, dyn, w, colour, step, lds.row, xch);
    else batch_window_body<KIND, DIM>(jobs, dyn, w, colour, step, lds.win);
}

// Coupled NE jobs run only the whole-row bodies (the host admits no other).
template <int KIND, int DIM>
__device__ __forceinline__ void dispatch_rows(uint32_t d, const BatchJob* jobs, const uint32_t* dyn,
                                              const BatchWG w, uint32_t colour, uint32_t step, BatchLds& lds,
                                              uint32_t (&xch)[2][16][2])
{
    if (d == 0) batch_half_body<KIND, DIM, 4>(jobs, dyn, w, colour, step, lds.row, xch);
    else if (d == 1) batch_half_body<KIND, DIM, 2>(jobs, dyn, w, colour, step, lds.row, xch);
    else if (d == 2) batch_half_body<KIND, DIM, 1>(jobs, dyn, w, colour, step, lds.row, xch);
}

static_assert(kBatchKindNeCoupled == KIND_NE_COUPLED, "batch class kind of coupled NE jobs");

__global__ void __launch_bounds__(256) k_batch_all(const BatchJob* __restrict__ jobs,
                                                   const uint32_t* __restrict__ dyn,
                                                   const BatchWG* __restrict__ wgs, uint32_t colour,
                                                   uint32_t step)
{
    __shared__ BatchLds lds;
    __shared__ uint32_t xch[2][16][2];
    const BatchWG w = wgs[blockIdx.x];
    const uint32_t cls = jobs[w.job].cls;
    const uint32_t kind = cls >> 3, dim3d = (cls >> 2) & 1u, d = cls & 3u;
    if (kind == KIND_ISING_HALF) {
        if (dim3d) dispatch_d<KIND_ISING_HALF, 3>(d, jobs, dyn, w, colour, step, lds, xch);
        else dispatch_d<KIND_ISING_HALF, 2>(d, jobs, dyn, w, colour, step, lds, xch);
    } else if (kind == KIND_ISING_ONE) {
        if (dim3d) dispatch_d<KIND_ISING_ONE, 3>(d, jobs, dyn, w, colour, step, lds, xch);
        else dispatch_d<KIND_ISING_ONE, 2>(d, jobs, dyn, w, colour, step, lds, xch);
    } else if (kind == KIND_NE) {
        dispatch_d<KIND_NE, 2>(d, jobs, dyn, w, colour, step, lds, xch);
    } else {
        dispatch_rows<KIND_NE_COUPLED, 2>(d, jobs, dyn, w, colour, step, lds, xch);
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

bool batch_geom(const Geom& g, int H, bool lut32_ok, RowGeomHost& out)
{
    // widest D whose row group fits one wave (the whole-row batched kernel
    // has no cross-wave exchange) ...
    for (int D : {4, 2, 1}) {
        if (!lut32_ok) break;
        RowGeom rg;
        if (!make_row_geom(g, H, D, false, rg)) continue;
        if (rg.R > 64) continue;
        static_assert(sizeof(RowGeom) <= sizeof(out.bytes), "RowGeom storage");
        __builtin_memcpy(out.bytes, &rg, sizeof(RowGeom));
        out.D = D;
        out.nitems = rg.nitems;
        out.items_per_wg = 4 * rg.slots;
        return true;
    }
    // ... else column windows (D = 0)
    if (g.Lh % 4) return false;
    const streamk::StreamGeom sg = streamk::make_geom(g, H, false);
    static_assert(sizeof(streamk::StreamGeom) <= sizeof(out.bytes), "StreamGeom storage");
    __builtin_memcpy(out.bytes, &sg, sizeof(sg));
    out.D = 0;
    out.nitems = sg.nitems;
    out.items_per_wg = 4 * sg.G;
    return true;
}

hipError_t launch_batch_fold(const BatchFold* tab, uint32_t nentries, int64_t* out, hipStream_t s)
{
    if (nentries == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_fold, dim3(nentries), dim3(256), 0, s, tab, out);
    return hipGetLastError();
}

hipError_t launch_batch_all(const BatchJob* jobs, const uint32_t* dyn, const BatchWG* wgs, uint32_t nwg,
                            uint32_t colour, uint32_t step, hipStream_t s)
{
    if (nwg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_all, dim3(nwg), dim3(256), 0, s, jobs, dyn, wgs, colour, step);
    return hipGetLastError();
}

}  // namespace spinlat
