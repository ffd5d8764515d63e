// Batched-launch kernels for stencil operators (see batch_kernel.h).
#include "batch_kernel.h"

namespace phc {

BatchKernel batch_kernel_stencil(bool mix) {
    return mix ? solve_batch_kernel<kStencil, true> : solve_batch_kernel<kStencil, false>;
}

}  // namespace phc
