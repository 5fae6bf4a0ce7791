// Device-resident state of one Krylov solve (GMRES cycle or PCG pass),
// shared by the kernels and the host drivers.
#pragma once

namespace adj {

// Rows per 256-thread block of the Woodbury gather (capacitance rows) and
// correction (vertex rows), four per wavefront: 4 while that gives at least
// ~2048 blocks, up to 16 for large batches (each block first stages a
// per-scene vector in LDS, which the extra rows amortise).
inline int wb_rows_per_block(long long total_rows) {
  const long long q = (total_rows + 4 * 2048 - 1) / (4 * 2048);
  return 4 * (int)(q < 1 ? 1 : (q > 4 ? 4 : q));
}

// Where one scene's contact arrays live (caller's device memory) and where
// they go in the union arrays; shared by the gather kernel and the host.
struct ContactSrc {
  const int* vid;
  const int* fric;
  const double* frame;
  const double* delta;
  const double* lam;
  int n;     // contacts of the scene
  int off;   // first union contact
  int voff;  // first union vertex
  int pad;
};

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
