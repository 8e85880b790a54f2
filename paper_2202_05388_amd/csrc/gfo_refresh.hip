// FP64 refresh of G from G0 and the flipped set (placeholder until the FP64
// matrix-core path lands).
#include "gfo_internal.hpp"

namespace gfo {
int launch_refresh(const Geo&, gfo_state*, const Layout&, hipStream_t) { return GFO_EINVAL; }
}  // namespace gfo
