// Device least-squares solve of the reduced interface system.
#pragma once

#include "ap_solver.h"

namespace mdp {

struct LSResult {
    double rel_residual = 0.0;  // ||A x - F|| / ||F||
    double cond = 0.0;          // estimate of cond_2 of the column-equilibrated A (0 if not requested)
    bool shifted = false;       // the shifted first pass was needed
    int passes = 0;
};

// min ||A x - F||_2 for A (m x nc, column-major, ld m, device; overwritten) and
// F (m, device); x_out (nc, device).
LSResult ls_solve(Workspace& ws, double2* A, const double2* F, int m, int nc, double2* x_out, bool want_cond,
                  hipStream_t st);

}  // namespace mdp
