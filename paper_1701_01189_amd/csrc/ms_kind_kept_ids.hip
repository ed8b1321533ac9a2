// Post-scan instantiations for table-search buckets whose ids the pre-scan
// kept (compiled on its own so that the kinds build in parallel).
#include "ms_dispatch.hpp"

namespace ms {
hipError_t post_kept_ids(const PostArgs& a, int bits) { return post_dispatch<kKeptIds>(a, bits); }
}  // namespace ms
