// kernels_ne_sub_b64.hip -- NE sub-lattice kernels for sub-lattices of side 64
// (device code in ne_sub_device.hpp).
#include "ne_sub_device.hpp"

namespace spinlat {

hipError_t launch_ne_sub_b64(const NeSubArgs& a, int lambda, bool balanced, hipStream_t s)
{
    return nesub::launch_side<64>(a, lambda, balanced, s);
}

}  // namespace spinlat
