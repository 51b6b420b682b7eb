// Instantiation of the stencil kernels for LinkF32 links and the Brillouin operator.
#include "stencil_kernels.hpp"

namespace bri {

hipError_t launch_f32_bri(const StencilArgs &a, bool dag, int mode, const StencilConfig &cfg, hipStream_t st) {
    return dag ? launch_cfg<LinkF32, true, KERN_BRI>(a, mode, cfg, st) : launch_cfg<LinkF32, false, KERN_BRI>(a, mode, cfg, st);
}

}  // namespace bri
