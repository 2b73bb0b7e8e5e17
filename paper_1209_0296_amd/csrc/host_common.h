// host_common.h -- host helpers shared by the lattice and batch runtimes: the
// pure host logic of host_logic.h plus the mapping of HIP errors to statuses.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "host_logic.h"

namespace spinlat {
namespace host {

sl_status hip_fail(hipError_t e, const char* what);  // SL_E_HIP with the HIP message

}  // namespace host
}  // namespace spinlat
