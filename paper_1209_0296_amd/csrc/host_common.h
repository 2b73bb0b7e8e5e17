// host_common.h -- host helpers shared by the lattice and batch runtimes: the
// pure host logic of host_logic.h plus the mapping of HIP errors to statuses.
#pragma once
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stddef.h>
#include <stdint.h>

#include "host_logic.h"

namespace spinlat {
namespace host {

sl_status hip_fail(hipError_t e, const char* what);  // SL_E_HIP with the HIP message

// A named roctx range over the enclosing scope: the host-side enqueue of a
// call shows up as one range in a rocprofv3 trace taken with --marker-trace.
class TraceRange {
public:
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace host
}  // namespace spinlat
