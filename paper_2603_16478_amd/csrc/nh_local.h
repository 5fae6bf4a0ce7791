// Per-element local projection (Neo-Hookean, as-rigid-as-possible,
// co-rotational) and its SVD quantities, in registers (Sec. 5.3;
// App. B.0-B.4).  Used by the Jacobian/assembly kernel,
// the gradient kernel and the forward residual kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace adj {

// F = D_s B_m with D_s = [x1-x0, x2-x0, x3-x0]: F[r][c] = sum_k x_k[r] Bt[k][c].
__device__ __forceinline__ void deformation_gradient(const double x[4][3], const double Bt[4][3],
                                                     double F[3][3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      F[r][c] = x[0][r] * Bt[0][c] + x[1][r] * Bt[1][c] + x[2][r] * Bt[2][c] + x[3][r] * Bt[3][c];
}

__device__ __forceinline__ double det3(const double A[3][3]) {
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// One-sided (Hestenes) Jacobi SVD: rotate column pairs of A = F until they
// are orthogonal; then sigma_i = |a_i|, U_i = a_i / sigma_i, F = U diag(s) V^T.
// Any orthogonal U, V are acceptable: P, J and the gradients are invariant
// under the gauge freedom of the SVD (App. B.4).
__device__ __forceinline__ void svd3(const double F[3][3], double U[3][3], double s[3],
                                     double V[3][3]) {
  double A[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      A[r][c] = F[r][c];
      V[r][c] = (r == c) ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 12; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int pp = 0; pp < 3; ++pp) {
      const int p = (pp == 2) ? 1 : 0;
      const int q = (pp == 0) ? 1 : 2;
      double al = A[0][p] * A[0][p] + A[1][p] * A[1][p] + A[2][p] * A[2][p];
      double be = A[0][q] * A[0][q] + A[1][q] * A[1][q] + A[2][q] * A[2][q];
      double ga = A[0][p] * A[0][q] + A[1][p] * A[1][q] + A[2][p] * A[2][q];
      if (fabs(ga) > 1e-16 * sqrt(al * be)) {
        rotated = true;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t);
        double sn = c * t;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          double ap = A[r][p], aq = A[r][q];
          A[r][p] = c * ap - sn * aq;
          A[r][q] = sn * ap + c * aq;
          double vp = V[r][p], vq = V[r][q];
          V[r][p] = c * vp - sn * vq;
          V[r][q] = sn * vp + c * vq;
        }
      }
    }
    if (!rotated) break;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double n = sqrt(A[0][c] * A[0][c] + A[1][c] * A[1][c] + A[2][c] * A[2][c]);
    s[c] = n;
    double in = 1.0 / n;
#pragma unroll
    for (int r = 0; r < 3; ++r) U[r][c] = A[r][c] * in;
  }
}

// Optimality of the Neo-Hookean prox (App. B.3):
//   g(theta) = mu (3 theta - 2 sigma - 1/theta) + lam log(J) / theta = 0.
// Newton from theta = sigma; dg/dtheta = Diag(Dd) + lam u u^T with
// Dd_i = 3 mu + (mu - lam log J)/theta_i^2 and u = 1/theta (App. B.2), solved
// by Sherman-Morrison.
struct NHLocal {
  double th[3];
  double Dd[3];   // diagonal part of dg/dtheta at the root
  double u[3];    // 1/theta
  double den;     // 1 + lam u^T Dd^{-1} u
  double logJ;
};

// x = (Diag(Dd) + lam u u^T)^{-1} b
__device__ __forceinline__ void sm_solve(const double Dd[3], const double u[3], double lam,
                                         const double b[3], double x[3]) {
  double dib[3], diu[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    dib[i] = b[i] / Dd[i];
    diu[i] = u[i] / Dd[i];
  }
  double num = lam * (u[0] * dib[0] + u[1] * dib[1] + u[2] * dib[2]);
  double den = 1.0 + lam * (u[0] * diu[0] + u[1] * diu[1] + u[2] * diu[2]);
  double f = num / den;
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i] = dib[i] - diu[i] * f;
}

__device__ __forceinline__ void nh_theta(const double s[3], double mu, double lam, NHLocal& L) {
  double t[3] = {s[0], s[1], s[2]};
  for (int it = 0; it < 61; ++it) {
    double lj = log(t[0]) + log(t[1]) + log(t[2]);
    double g[3], Dd[3], u[3], d[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[i] = 1.0 / t[i];
      g[i] = mu * (3.0 * t[i] - 2.0 * s[i] - u[i]) + lam * lj * u[i];
      Dd[i] = 3.0 * mu + (mu - lam * lj) * u[i] * u[i];
      g[i] = -g[i];
    }
    sm_solve(Dd, u, lam, g, d);
    if (it == 60) {  // final polishing step at the converged point
#pragma unroll
      for (int i = 0; i < 3; ++i) t[i] += d[i];
      break;
    }
    double step = 1.0;
    for (int k = 0; k < 60; ++k) {
      if (t[0] + step * d[0] > 0 && t[1] + step * d[1] > 0 && t[2] + step * d[2] > 0) break;
      step *= 0.5;
    }
    bool done = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double dd = step * d[i];
      t[i] += dd;
      if (fabs(dd) > 1e-15 * fabs(t[i])) done = false;
    }
    if (done) it = 59;  // jump to the polishing step
  }
  double lj = log(t[0]) + log(t[1]) + log(t[2]);
  L.logJ = lj;
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    L.th[i] = t[i];
    L.u[i] = 1.0 / t[i];
    L.Dd[i] = 3.0 * mu + (mu - lam * lj) * L.u[i] * L.u[i];
    acc += L.u[i] * L.u[i] / L.Dd[i];
  }
  L.den = 1.0 + lam * acc;
}

// W = dtheta/dsigma = 2 mu (dg/dtheta)^{-1} (App. B.2).
__device__ __forceinline__ void nh_W(const NHLocal& L, double mu, double lam, double W[3][3]) {
  double a[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) a[i] = L.u[i] / L.Dd[i];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      W[i][j] = 2.0 * mu * (((i == j) ? 1.0 / L.Dd[i] : 0.0) - lam * a[i] * a[j] / L.den);
}

// ---- material models of the local step (App. B.2) ----
// 0 Neo-Hookean (above), 1 as-rigid-as-possible (theta = 1: the projection is
// the rotation of the polar decomposition, W = 0), 2 co-rotational (zeta =
// mu |theta - 1|^2 + lam/2 (sum(theta - 1))^2, so the optimality condition is
// linear: (4 mu I + lam 1 1^T)(theta - 1) = 2 mu (sigma - 1) and W is the
// constant 2 mu (4 mu I + lam 1 1^T)^{-1}).
enum : int { MAT_NEO_HOOKEAN = 0, MAT_ARAP = 1, MAT_COROT = 2 };

// x = (4 mu I + lam 1 1^T)^{-1} b by Sherman-Morrison
__device__ __forceinline__ void corot_solve(double mu, double lam, const double b[3], double x[3]) {
  const double f = lam * (b[0] + b[1] + b[2]) / (4.0 * mu + 3.0 * lam);
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i] = (b[i] - f) / (4.0 * mu);
}

// Singular values theta of the projection, the singular-value Jacobian W and
// the off-diagonal divided differences q_ij = (theta_i - theta_j)/(sigma_i -
// sigma_j) in their cancellation-free forms (NH: q_ij from g_i - g_j = 0;
// ARAP: 0; co-rot: 1/2).  For NH, L receives the Newton record (for the
// parameter derivatives).
__device__ __forceinline__ void local_projection(int model, const double s[3], double mu, double lam,
                                                 double th[3], double W[3][3], double qd[3][3], NHLocal& L) {
  if (model == MAT_ARAP) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      th[i] = 1.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) W[i][j] = qd[i][j] = 0.0;
    }
    return;
  }
  if (model == MAT_COROT) {
    double b[3] = {2.0 * mu * (s[0] - 1.0), 2.0 * mu * (s[1] - 1.0), 2.0 * mu * (s[2] - 1.0)}, d[3];
    corot_solve(mu, lam, b, d);
    const double cw = lam / (4.0 * mu + 3.0 * lam);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      th[i] = 1.0 + d[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        W[i][j] = 0.5 * (((i == j) ? 1.0 : 0.0) - cw);
        qd[i][j] = 0.5;
      }
    }
    return;
  }
  nh_theta(s, mu, lam, L);
  nh_W(L, mu, lam, W);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    th[i] = L.th[i];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      qd[i][j] = 2.0 * mu / (3.0 * mu + (mu - lam * L.logJ) / (L.th[i] * L.th[j]));
  }
}

// M_ij = (q_ij + avg_ij)/2, N_ij = (q_ij - avg_ij)/2 with avg_ij = (theta_i +
// theta_j)/(sigma_i + sigma_j), zero on the diagonal (App. B.0).
__device__ __forceinline__ void local_MN(const double th[3], const double s[3], const double qd[3][3],
                                         double M[3][3], double N[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (i == j) {
        M[i][j] = 0.0;
        N[i][j] = 0.0;
      } else {
        const double avg = (th[i] + th[j]) / (s[i] + s[j]);
        M[i][j] = 0.5 * (qd[i][j] + avg);
        N[i][j] = 0.5 * (qd[i][j] - avg);
      }
    }
}

// dtheta/dmu and dtheta/dlam at fixed sigma: -(dg/dtheta)^{-1} dg/dmu and
// -(dg/dtheta)^{-1} dg/dlam (App. B.3), with g the optimality condition of
// the model (ARAP: theta does not depend on the parameters).
__device__ __forceinline__ void local_param_derivs(int model, const double s[3], const double th[3], double mu,
                                                   double lam, const NHLocal& L, double dmu[3], double dlam[3]) {
  if (model == MAT_ARAP) {
#pragma unroll
    for (int i = 0; i < 3; ++i) dmu[i] = dlam[i] = 0.0;
    return;
  }
  double gmu[3], glam[3];
  if (model == MAT_COROT) {
    const double tr = (th[0] - 1.0) + (th[1] - 1.0) + (th[2] - 1.0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      gmu[i] = -2.0 * (2.0 * th[i] - s[i] - 1.0);
      glam[i] = -tr;
    }
    corot_solve(mu, lam, gmu, dmu);
    corot_solve(mu, lam, glam, dlam);
    return;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gmu[i] = -(3.0 * L.th[i] - 2.0 * s[i] - L.u[i]);
    glam[i] = -(L.logJ * L.u[i]);
  }
  sm_solve(L.Dd, L.u, lam, gmu, dmu);
  sm_solve(L.Dd, L.u, lam, glam, dlam);
}

// theta alone (the forward residual)
__device__ __forceinline__ void local_theta(int model, const double s[3], double mu, double lam, double th[3]) {
  if (model == MAT_ARAP) {
    th[0] = th[1] = th[2] = 1.0;
    return;
  }
  if (model == MAT_COROT) {
    double b[3] = {2.0 * mu * (s[0] - 1.0), 2.0 * mu * (s[1] - 1.0), 2.0 * mu * (s[2] - 1.0)}, d[3];
    corot_solve(mu, lam, b, d);
#pragma unroll
    for (int i = 0; i < 3; ++i) th[i] = 1.0 + d[i];
    return;
  }
  NHLocal L;
  nh_theta(s, mu, lam, L);
#pragma unroll
  for (int i = 0; i < 3; ++i) th[i] = L.th[i];
}

}  // namespace adj
