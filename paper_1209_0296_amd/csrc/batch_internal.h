// batch_internal.h -- device job table shared by the batch runtime and the
// batched kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spinlat_internal.h"

namespace spinlat {

constexpr int kDynWords = 4;  // per job: {t, record slot, sweeps in this call, unused}
constexpr int kTableMax = 52; // Ising threshold table entries (3D: 4 x 13)

struct BatchJob {
    uint8_t* col[2];           // colour arrays
    unsigned long long* acc;   // record ring [capacity][kSub][kQ]
    uint32_t key0, key1;       // Philox key = seed
    uint32_t cls;              // kernel variant: batch_class(kind, dim, D)
    uint32_t pad;
    uint32_t rg_words[16];     // whole-row geometry of the job (RowGeom)
    uint64_t table[kTableMax]; // threshold table (NE: up, down)
};

struct BatchWG {
    uint32_t job;        // index into the job table
    uint32_t item_base;  // first item (strip, plane) of this workgroup
};

struct BatchFold {
    unsigned long long* ring;  // job's accumulators
    uint64_t out_off;          // first output record
    uint64_t first_t;          // t of the job's oldest unread record
    uint32_t n;                // records to fold
    uint32_t ising;            // 1: unflipped is reported as -1
};

struct RowGeomHost {
    uint32_t bytes[16];      // RowGeom as the kernels see it
    int D;                   // words per lane (0: column-window kernel)
    uint32_t nitems;         // items of one half-sweep
    uint32_t items_per_wg;   // items one workgroup of 256 lanes covers
};

// Geometry of a job for the batched kernels: whole-row groups within one wave
// (D = 1, 2, 4) when the row fits and the 32-bit spin-1/2 table applies, else
// 64-lane column windows (D = 0).
bool batch_geom(const Geom& g, int H, bool lut32_ok, RowGeomHost& out);

// Class kind of coupled NE jobs (SL_NE_COUPLED): the whole-row kernels'
// coupled instantiation; such jobs need a row class (D != 0).
constexpr int kBatchKindNeCoupled = 3;

// Variant index of a job for the one-launch kernel: kind, dimension and D.
inline uint32_t batch_class(int kind, int dim, int D)
{
    const uint32_t d = D == 4 ? 0u : D == 2 ? 1u : D == 1 ? 2u : 3u;
    return (uint32_t)kind * 8u + (uint32_t)(dim - 2) * 4u + d;
}

// All jobs of a half-sweep in one launch (work list sorted by variant): the
// call's sweep number `step` runs sweep t + step of every job whose count in
// this call exceeds step.
hipError_t launch_batch_all(const BatchJob* jobs, const uint32_t* dyn, const BatchWG* wgs, uint32_t nwg,
                            uint32_t colour, uint32_t step, hipStream_t s);
hipError_t launch_batch_fold(const BatchFold* tab, uint32_t nentries, int64_t* out, hipStream_t s);

}  // namespace spinlat
