// Render kernel instantiations for C = 16 feature channels (one file per C so
// the variants compile in parallel).
#include "render_impl.h"

namespace art {

template <>
hipError_t launch_render_c<16>(const RenderLaunch& r, const RArgs& a, unsigned grid, hipStream_t st) {
    return launch_render_dispatch<16>(r, a, grid, st);
}

}  // namespace art
