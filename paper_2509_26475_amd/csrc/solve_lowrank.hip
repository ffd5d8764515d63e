// Solve-kernel variants for low-rank operators A = U W^T (Al-Mohy, Sec. 5,
// third experiment), compiled apart from the other kinds.
#include "solve_body.h"

namespace phc {

KernelFn pick_lowrank(int r, int rpt, bool emem, bool mix) {
    return pick_r<kLowRank>(r, rpt, emem, mix);
}

}  // namespace phc
