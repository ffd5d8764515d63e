// Batched-launch kernels for csr operators (see batch_kernel.h).
#include "batch_kernel.h"

namespace phc {

BatchKernel batch_kernel_csr(bool mix) {
    return mix ? solve_batch_kernel<kCsr, true> : solve_batch_kernel<kCsr, false>;
}

}  // namespace phc
