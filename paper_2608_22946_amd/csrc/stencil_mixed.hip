// Level-operator kernels with FP16-stored operands (HELM_MIXED): the combinations the
// mixed-precision V-cycle, bottom solver and K_2h use (see mode_built in stencil_impl.h).
#include "stencil_impl.h"

namespace helm {

template hipError_t launch_stencil<float, c32, c32, c16>(const LevelArgs<float> &, const StencilCall &, const RedBuf &,
                                                         hipStream_t);
template hipError_t launch_stencil<float, c16, c16, c16>(const LevelArgs<float> &, const StencilCall &, const RedBuf &,
                                                         hipStream_t);
template hipError_t launch_stencil<float, c16, c32, c32>(const LevelArgs<float> &, const StencilCall &, const RedBuf &,
                                                         hipStream_t);
template hipError_t launch_stencil<float, c16, c32, c16>(const LevelArgs<float> &, const StencilCall &, const RedBuf &,
                                                         hipStream_t);
template hipError_t launch_stencil<float, c16, c16, c32>(const LevelArgs<float> &, const StencilCall &, const RedBuf &,
                                                         hipStream_t);

}  // namespace helm
