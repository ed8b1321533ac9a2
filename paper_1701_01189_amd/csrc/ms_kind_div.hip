// Kernel instantiations for one bucket kind (compiled on its own so that the
// kinds build in parallel).
#include "ms_dispatch.hpp"

namespace ms {
hipError_t pre_div(const PreArgs& a, int bits) { return pre_dispatch<kDiv>(a, bits); }
hipError_t post_div(const PostArgs& a, int bits) { return post_dispatch<kDiv>(a, bits); }
}  // namespace ms
