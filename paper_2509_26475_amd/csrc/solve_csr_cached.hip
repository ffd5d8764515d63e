// Solve-kernel variants for CSR operators with rows of at most kCacheNnz
// entries, held in registers for the whole solve.
#include "solve_body.h"

namespace phc {

KernelFn pick_csr_cached(int r, int rpt, bool mix) {
    return pick_r<kCsrCached>(r, rpt, false, mix);
}

}  // namespace phc
