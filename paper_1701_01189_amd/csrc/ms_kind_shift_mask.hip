// Kernel instantiations for one bucket kind (compiled on its own so that the
// kinds build in parallel).
#include "ms_dispatch.hpp"

namespace ms {
hipError_t pre_shift_mask(const PreArgs& a, int bits) { return pre_dispatch<kShiftMask>(a, bits); }
hipError_t post_shift_mask(const PostArgs& a, int bits) { return post_dispatch<kShiftMask>(a, bits); }
}  // namespace ms
