// Instantiation of the stencil kernels for LinkF64 links and the Wilson operator.
#include "stencil_kernels.hpp"

namespace bri {

hipError_t launch_f64_wil(const StencilArgs &a, bool dag, int mode, const StencilConfig &cfg, hipStream_t st) {
    return dag ? launch_cfg<LinkF64, true, KERN_WIL>(a, mode, cfg, st) : launch_cfg<LinkF64, false, KERN_WIL>(a, mode, cfg, st);
}

}  // namespace bri
