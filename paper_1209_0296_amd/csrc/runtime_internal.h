// runtime_internal.h -- the lattice handle and the enqueue steps of the
// single-lattice runtime (runtime.cpp), shared with the other host entry
// points of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spinlat.h"
#include "host_common.h"
#include "spinlat_internal.h"

// Handle of one lattice: its parameters, the layout of the borrowed device
// buffer, the stream, sweep and record counters, and the schedule.
struct sl_lattice {
    sl_params params;
    spinlat::host::Layout lay;
    uint8_t* base;
    hipStream_t stream;
    int kind;
    uint64_t next_t;   // index of the next sweep
    uint64_t pending;  // unread records
    uint64_t first_t;  // t of the oldest unread record
    int cur;           // copy of the lattice holding the current state
    sl_launch launch;
    uint64_t table[spinlat::kMaxLut];
    size_t table_n;
    sl_record* stage;  // pinned host staging for record readback (record_capacity)
};

namespace spinlat {
namespace rt {

constexpr uint64_t kResidentChunk = 4096;  // sweeps per resident launch at most

SweepArgs args_of(const sl_lattice* h);
unsigned long long* slot_ptr(const sl_lattice* h, uint64_t idx);  // record ring slot
sl_launch auto_launch(const sl_lattice* h);                         // default schedule
sl_status enqueue_observe(sl_lattice* h, uint64_t slot);            // record of the state
sl_status enqueue_sweeps(sl_lattice* h, uint64_t n);                // n sweeps, unchecked

}  // namespace rt
}  // namespace spinlat
