// Solve-kernel variants for dense operators (FP64 MFMA products, E in memory).
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

}  // namespace phc
