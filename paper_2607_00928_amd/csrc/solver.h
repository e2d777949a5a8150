// Factorization and solution drivers.
#pragma once

#include "plan.h"

namespace nd {

void factor(Plan* P);
// adjoint == false: c = A^+ f (refined as opts say); adjoint == true:
// c (length M per right-hand side) = (A^+)^H f (f of length N).
void solve(Plan* P, const double2* f, double2* c, int nrhs, nudft2_solve_info* info,
           bool adjoint);
// Backward pass of c = A^+ f: grad_f = (A^+)^H g; grad_pts (M x 2, may be
// null) = dL/d(x_j, y_j) summed over the right-hand sides.
void lsq_backward(Plan* P, const double2* f, const double2* c, const double2* g, double2* grad_f,
                  double* grad_pts, int nrhs, nudft2_solve_info* info);

}  // namespace nd
