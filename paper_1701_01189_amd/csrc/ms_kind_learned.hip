// Kernel instantiations for one bucket kind (compiled on its own so that the
// kinds build in parallel).
#include "ms_dispatch.hpp"

namespace ms {
hipError_t pre_learned(const PreArgs& a, int bits) { return pre_dispatch<kLearned>(a, bits); }
hipError_t post_learned(const PostArgs& a, int bits) { return post_dispatch<kLearned>(a, bits); }
hipError_t batched_learned(const BatchedArgs& a, int bits, bool kv, int wpb, int nw, hipStream_t st) {
  return batched_dispatch<kLearned>(a, bits, kv, wpb, nw, st);
}
}  // namespace ms
