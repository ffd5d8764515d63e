// Solve-kernel variants for CSR operators whose rows are read per product.
#include "solve_body.h"

namespace phc {

KernelFn pick_csr(int r, int rpt, bool emem, bool mix) {
    return pick_r<kCsr>(r, rpt, emem, mix);
}

}  // namespace phc
