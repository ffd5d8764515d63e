// Solve-kernel variants for dense operators (FP64 MFMA products, E in memory;
// small operators with everything in LDS).
#include "solve_body.h"

namespace phc {

KernelFn pick_dense(int r) {
    switch (r) {
    case 1: return solve_kernel<kDense, 1, 1, true, false>;
    case 2: return solve_kernel<kDense, 2, 1, true, false>;
    case 3: return solve_kernel<kDense, 3, 1, true, false>;
    case 4: return solve_kernel<kDense, 4, 1, true, false>;
    default: return nullptr;
    }
}

KernelFn pick_dense_lds(int r) {
    switch (r) {
    case 1: return solve_kernel_dense_lds<1>;
    case 2: return solve_kernel_dense_lds<2>;
    case 3: return solve_kernel_dense_lds<3>;
    case 4: return solve_kernel_dense_lds<4>;
    default: return nullptr;
    }
}

}  // namespace phc
