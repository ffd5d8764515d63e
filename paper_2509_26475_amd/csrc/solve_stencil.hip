// Solve-kernel variants for stencil operators (Al-Mohy, Sec. 4, Algorithm 3).
#include "solve_body.h"

namespace phc {

KernelFn pick_stencil(int r, int rpt, bool emem, bool mix) {
    return pick_r<kStencil>(r, rpt, emem, mix);
}

KernelFn pick_stencil_wide(int r, bool mix) {
    switch (r) {
    case 1: return mix ? solve_kernel<kStencil, 1, 1, true, true, kWideNT>
                       : solve_kernel<kStencil, 1, 1, true, false, kWideNT>;
    case 2: return mix ? solve_kernel<kStencil, 2, 1, true, true, kWideNT>
                       : solve_kernel<kStencil, 2, 1, true, false, kWideNT>;
    default: return nullptr;
    }
}

}  // namespace phc
