// batch_internal.h -- device job table shared by the batch runtime and the
// batched kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spinlat_internal.h"

namespace spinlat {

constexpr int kDynWords = 4;  // per job: {t, record slot, sweeps in this call, current copy}
constexpr int kTableMax = 52; // Ising threshold table entries (3D: 4 x 13)

// Kernel variant of a job (low 4 bits of BatchJob::cls).
constexpr uint32_t kBvWalkD4 = 0, kBvWalkD2 = 1, kBvWalkD1 = 2;    // whole-row walk, one colour per launch
constexpr uint32_t kBvWindow = 3;                                  // column windows, one colour per launch
constexpr uint32_t kBvRowsD4 = 4, kBvRowsD2 = 5, kBvRowsD1 = 6;    // row groups without a walk (3D)
constexpr uint32_t kBvFusedD4 = 8, kBvFusedD2 = 9, kBvFusedD1 = 10; // both colours in the colour-0 launch (2D)
constexpr uint32_t kBvResident = 12;                               // whole chunk in LDS, own launch

struct BatchJob {
    uint8_t* col[2][2];        // [copy][colour] colour arrays (copy 1 only for fused jobs)
    unsigned long long* acc;   // record ring [capacity][kSub][kQ]
    uint32_t key0, key1;       // Philox key = seed
    uint32_t cls;              // kind * 32 + (dim - 2) * 16 + variant
    uint32_t copies;           // 1, or 2 for fused jobs
    uint32_t dim, table_n;
    uint32_t rg_words[16];     // geometry of the job's kernel (RowGeom or StreamGeom)
    uint64_t table[kTableMax]; // threshold table (NE: up, down)
};

struct BatchWG {
    uint32_t job;        // index into the job table
    uint32_t item_base;  // first item (strip, plane or row set) of this workgroup
};

struct BatchFold {
    unsigned long long* ring;  // job's accumulators
    uint64_t out_off;          // first output record
    uint64_t first_t;          // t of the job's oldest unread record
    uint32_t n;                // records to fold
    uint32_t ising;            // 1: unflipped is reported as -1
};

struct RowGeomHost {
    uint32_t bytes[16];      // geometry as the kernels see it
    uint32_t variant;        // kBv*
    uint32_t copies = 1;     // lattice copies the job needs
    uint32_t nitems;         // items of one launch
    uint32_t items_per_wg;   // items one workgroup of 256 lanes covers
};

// Geometry of a non-resident job: 3D row groups without a walk, 2D fused
// strips (if allow_fused) or whole-row walks when the colour row fits one
// wave and the 32-bit spin-1/2 table applies; else 64-lane column windows.
bool batch_geom(const Geom& g, int H, bool lut32_ok, bool allow_fused, RowGeomHost& out);
// Resident class: both colours in at most kResidentLds bytes.
bool batch_resident_geom(const Geom& g, RowGeomHost& out);

// Class kind of coupled NE jobs (SL_NE_COUPLED): the whole-row kernels'
// coupled instantiation; such jobs need a row class.
constexpr int kBatchKindNeCoupled = 3;

inline uint32_t batch_class(int kind, int dim, uint32_t variant)
{
    return (uint32_t)kind * 32u + (uint32_t)(dim - 2) * 16u + variant;
}

// Kernel families of the non-resident classes and their work-list segments:
// 0 walks and windows, 1 row groups of spin-1/2 jobs, 2 fused, 3 row groups of
// spin-1 jobs (two Philox calls per word need more registers; apart, the
// spin-1/2 row groups keep more waves per SIMD).
constexpr int kBatchFamilies = 4;
inline int batch_family(uint32_t variant, uint32_t kind)
{
    if (variant >= kBvFusedD4 && variant <= kBvFusedD1) return 2;
    if (variant >= kBvRowsD4 && variant <= kBvRowsD1) return kind == (uint32_t)KIND_ISING_ONE ? 3 : 1;
    return 0;
}
// Families that run on the row-group stream.
inline bool row_family(int f) { return f == 1 || f == 3; }

// One family's launch: meta holds {count, offset} of each family's segment of
// `wgs` (valid entries out of `grid` workgroups); the call's sweep number
// `step` runs sweep t + step of every job whose count in this call exceeds
// step.  Half and row families take a colour; fused jobs do both colours.
hipError_t launch_batch_family(int family, const BatchJob* jobs, const uint32_t* dyn, const BatchWG* wgs,
                               const uint32_t* meta, uint32_t grid, uint32_t colour, uint32_t step, hipStream_t s);
// Every resident job of `list` runs its sweeps of the call in LDS.
hipError_t launch_batch_resident(const BatchJob* jobs, const uint32_t* dyn, const uint32_t* list, uint32_t njobs,
                                 hipStream_t s);
hipError_t launch_batch_fold(const BatchFold* tab, uint32_t nentries, int64_t* out, hipStream_t s);

}  // namespace spinlat
