// Instantiation of the stencil kernels for LinkBF16 links and the Wilson operator.
#include "stencil_kernels.hpp"

namespace bri {

hipError_t launch_bf16_wil(const StencilArgs &a, bool dag, int mode, const StencilConfig &cfg, hipStream_t st) {
    return dag ? launch_cfg<LinkBF16, true, KERN_WIL>(a, mode, cfg, st) : launch_cfg<LinkBF16, false, KERN_WIL>(a, mode, cfg, st);
}

}  // namespace bri
