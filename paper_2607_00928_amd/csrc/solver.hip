#include "hss.h"
#include "solver.h"

namespace nd {

void factor(Plan* P) { throw Error(NUDFT2_E_INTERNAL, "factor: not built yet"); }
void solve(Plan* P, const double2* f, double2* c, int nrhs, nudft2_solve_info* info,
           bool adjoint) {
  throw Error(NUDFT2_E_INTERNAL, "solve: not built yet");
}

}  // namespace nd
