// Kernel instantiations for one bucket kind (compiled on its own so that the
// kinds build in parallel).
#include "ms_dispatch.hpp"

namespace ms {
hipError_t pre_div(const PreArgs& a, int bits) { return pre_dispatch<kDiv>(a, bits); }
hipError_t post_div(const PostArgs& a, int bits) { return post_dispatch<kDiv>(a, bits); }
hipError_t batched_div(const BatchedArgs& a, int bits, bool kv, int wpb, int nw, hipStream_t st) {
  return batched_dispatch<kDiv>(a, bits, kv, wpb, nw, st);
}
}  // namespace ms
