// kernels_tiled.hip -- LDS-tiled half-sweep and fused sweep kernels (gfx950).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"
#include "site_update.hpp"
#include "spinlat_internal.h"

namespace spinlat {

bool tiled_supported(const Geom&, int, int, int, bool) { return false; }

hipError_t launch_tiled_half(const SweepArgs&, int, hipStream_t) { return hipErrorNotSupported; }

hipError_t launch_fused_sweep(const SweepArgs&, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace spinlat
