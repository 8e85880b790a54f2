// Rank-k Woodbury update (placeholder until the matrix-core path lands).
#include "gfo_internal.hpp"

namespace gfo {
hipError_t launch_rank_k(const Geo&, gfo_state*, const Layout&, const gfo_pick*, int, int,
                         hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace gfo
