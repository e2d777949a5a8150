// Factorization and solution drivers.
#pragma once

#include "plan.h"

namespace nd {

void factor(Plan* P);
void solve(Plan* P, const double2* f, double2* c, int nrhs, nudft2_solve_info* info,
           bool adjoint);

}  // namespace nd
