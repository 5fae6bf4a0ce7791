// Device-resident state of one Krylov solve (GMRES cycle or PCG pass),
// shared by the kernels and the host drivers.
#pragma once

namespace adj {

struct GmresState {
  int j;          // completed iterations of this cycle (PCG: of this pass)
  int active;     // 1 while the cycle runs
  int restart;    // GMRES restart length (PCG: iteration limit of the pass)
  int done;       // batched solves: 1 once the scene has converged
  double tol;     // absolute tolerance on the residual estimate
  double res;     // current residual estimate
  double rnorm;   // true residual norm (restart checks)
};

}  // namespace adj
