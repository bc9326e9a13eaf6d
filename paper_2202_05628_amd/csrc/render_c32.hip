// Render kernel instantiations for C = 32 feature channels.
#include "render_impl.h"

namespace art {

template <>
hipError_t launch_render_c<32>(const RenderLaunch& r, const RArgs& a, unsigned grid, hipStream_t st) {
#define ART_LAUNCH(ST, R, MODE) \
    hipLaunchKernelGGL((k_render<32, ST, R, MODE>), dim3(grid), dim3(64), 0, st, a)
    const int st_ = r.storage == ART_BF16 ? 1 : 0;
    if (r.fp32) {
        if (st_ == 0) {
            if (r.mode == 0) ART_LAUNCH(0, float, 0);
            else if (r.mode == 1) ART_LAUNCH(0, float, 1);
            else ART_LAUNCH(0, float, 2);
        } else {
            if (r.mode == 0) ART_LAUNCH(1, float, 0);
            else if (r.mode == 1) ART_LAUNCH(1, float, 1);
            else ART_LAUNCH(1, float, 2);
        }
    } else {
        if (st_ == 0) {
            if (r.mode == 0) ART_LAUNCH(0, double, 0);
            else if (r.mode == 1) ART_LAUNCH(0, double, 1);
            else ART_LAUNCH(0, double, 2);
        } else {
            if (r.mode == 0) ART_LAUNCH(1, double, 0);
            else if (r.mode == 1) ART_LAUNCH(1, double, 1);
            else ART_LAUNCH(1, double, 2);
        }
    }
#undef ART_LAUNCH
    return hipGetLastError();
}

}  // namespace art
