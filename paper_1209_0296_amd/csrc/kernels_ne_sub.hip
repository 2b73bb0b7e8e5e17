// kernels_ne_sub.hip -- launch of the North-East model by the paper's random
// sub-lattice algorithm (Sec. 3.2): picks the instantiation for the
// sub-lattice side (device code in ne_sub_device.hpp, one translation unit per
// side).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spinlat_internal.h"

namespace spinlat {

hipError_t launch_ne_sub_b8(const NeSubArgs& a, int lambda, bool balanced, hipStream_t s);
hipError_t launch_ne_sub_b16(const NeSubArgs& a, int lambda, bool balanced, hipStream_t s);
hipError_t launch_ne_sub_b32(const NeSubArgs& a, int lambda, bool balanced, hipStream_t s);
hipError_t launch_ne_sub_b64(const NeSubArgs& a, int lambda, bool balanced, hipStream_t s);

hipError_t launch_ne_sub(const NeSubArgs& a, int B, int lambda, bool balanced, hipStream_t s)
{
    switch (B) {
        case 8: return launch_ne_sub_b8(a, lambda, balanced, s);
        case 16: return launch_ne_sub_b16(a, lambda, balanced, s);
        case 32: return launch_ne_sub_b32(a, lambda, balanced, s);
        case 64: return launch_ne_sub_b64(a, lambda, balanced, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace spinlat
