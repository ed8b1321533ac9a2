// Kernel instantiations for one bucket kind (compiled on its own so that the
// kinds build in parallel).
#include "ms_dispatch.hpp"

namespace ms {
hipError_t pre_learned(const PreArgs& a, int bits) { return pre_dispatch<kLearned>(a, bits); }
hipError_t post_learned(const PostArgs& a, int bits) { return post_dispatch<kLearned>(a, bits); }
}  // namespace ms
