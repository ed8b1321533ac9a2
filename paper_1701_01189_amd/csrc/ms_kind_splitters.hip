// Kernel instantiations for one bucket kind (compiled on its own so that the
// kinds build in parallel).
#include "ms_dispatch.hpp"

namespace ms {
hipError_t pre_splitters(const PreArgs& a, int bits) { return pre_dispatch<kSplitters>(a, bits); }
hipError_t post_splitters(const PostArgs& a, int bits) { return post_dispatch<kSplitters>(a, bits); }
}  // namespace ms
