// Contact blocks, the contact-space capacitance of the Woodbury
// preconditioner, and the contact part of the gradients.
//
// Contact Jacobian (Sec. 5.2, eq:partial_contact, eq:final_diff_contact):
//   d lambda_c / d delta_c = -K_c = -R^T Khat R,
//   Khat = [[a, 0, 0], [-mu a, b, 0], [0, 0, c]],
//   a = (r - x)/(r - y) at (delta_n, lambda_n), b the same at
//   (|delta_f|, mu lambda_n - |lambda_f|), c = |lambda_f| / |delta_f|
// (the general ratio of the phi_eps partials; it equals y/x on the zero set,
// App. A.2), evaluated without cancellation:
//   r - x = (y^2 + 2 eps^2)/(r + x) for x > 0.
// R (App. A.1): built from lambda_f if |lambda_f| >= 1e-10, else from
// delta_f if |delta_f| >= 1e-12, else the identity.
// Normal-only contacts carry the 1x1 block [a] on the normal.
//
// Capacitance of the transposed system (Sec. 5.4, eq:woodbury_formula with
// K^T): C = Khat^{-T} + h^2 Hq A^{-1} Hq^T in the rotated basis Q_c = R_c frame_c;
// since A = A_s (x) I_3, the (c, c') block is h^2 D[v_c, v_c'] Q_c Q_c'^T with
// D = E^T A_s^{-1} E the scalar Delassus matrix of the contact vertices.
#include "device_common.h"

namespace adj {

__device__ __forceinline__ double fb_r_minus(double x, double y, double e2) {
  // r - x with r = sqrt(x^2 + y^2 + 2 eps^2), e2 = 2 eps^2
  double r = sqrt(x * x + y * y + e2);
  return (x > 0.0) ? (y * y + e2) / (r + x) : r - x;
}

__device__ __forceinline__ double fb_ratio(double x, double y, double e2) {
  return fb_r_minus(x, y, e2) / fb_r_minus(y, x, e2);
}

// Per contact outputs:
//   Wt[9]  world 3x3 block h^2 frame^T K_c^T frame (transpose = 1) or
//          h^2 frame^T K_c frame (transpose = 0), added to the diagonal of Acal^T / Acal
//   Q[9]   rows of R frame (normal, slip direction, perpendicular)
//   kh[4]  a, b, c, fric
//   Kc[9]  K_c in frame coordinates
//   kmu[3] k_mu = R^T [0, lambda_n, 0] in frame coordinates
__global__ void k_contact_blocks(int nc, const int* __restrict__ fric, const double* __restrict__ frame,
                                 const double* __restrict__ delta, const double* __restrict__ lam,
                                 double mu_all, const double* __restrict__ mu_c, double eps, double h2,
                                 int transpose,
                                 double* __restrict__ Wt, double* __restrict__ Q,
                                 double* __restrict__ kh, double* __restrict__ Kc,
                                 double* __restrict__ kmu) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double mu = mu_c ? mu_c[c] : mu_all;  // per-contact coefficient (batched scenes)
  const double e2 = 2.0 * eps * eps;
  const double dn = delta[3 * c], ln = lam[3 * c];
  const double a = fb_ratio(dn, ln, e2);
  double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double b = 0.0, cc = 0.0;
  const bool fr = fric[c] != 0;
  if (!fr) {
    K[0][0] = a;
  } else {
    const double d1 = delta[3 * c + 1], d2 = delta[3 * c + 2];
    const double l1 = lam[3 * c + 1], l2 = lam[3 * c + 2];
    const double ndf = sqrt(d1 * d1 + d2 * d2);
    const double nlf = sqrt(l1 * l1 + l2 * l2);
    if (nlf >= 1e-10) {
      const double u1 = -l1 / nlf, u2 = -l2 / nlf;
      R[1][1] = u1; R[1][2] = u2; R[2][1] = -u2; R[2][2] = u1;
    } else if (ndf >= 1e-12) {
      const double u1 = d1 / ndf, u2 = d2 / ndf;
      R[1][1] = u1; R[1][2] = u2; R[2][1] = -u2; R[2][2] = u1;
    }
    b = fb_ratio(ndf, mu * ln - nlf, e2);
    cc = (ndf > 0.0) ? nlf / ndf : 0.0;
    const double Kh[3][3] = {{a, 0.0, 0.0}, {-mu * a, b, 0.0}, {0.0, 0.0, cc}};
    // K = R^T Kh R
    double T[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) T[i][j] = Kh[i][0] * R[0][j] + Kh[i][1] * R[1][j] + Kh[i][2] * R[2][j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) K[i][j] = R[0][i] * T[0][j] + R[1][i] * T[1][j] + R[2][i] * T[2][j];
  }
  double Fr[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Fr[i][j] = frame[9 * c + 3 * i + j];
  // world block h^2 Fr^T K' Fr with K' = K^T (transpose) or K
  double T[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += (transpose ? K[k][i] : K[i][k]) * Fr[k][j];
      T[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += Fr[k][i] * T[k][j];
      Wt[9 * c + 3 * i + j] = h2 * s;
      Kc[9 * c + 3 * i + j] = K[i][j];
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Q[9 * c + 3 * i + j] = R[i][0] * Fr[0][j] + R[i][1] * Fr[1][j] + R[i][2] * Fr[2][j];
  kh[4 * c + 0] = a;
  kh[4 * c + 1] = b;
  kh[4 * c + 2] = cc;
  kh[4 * c + 3] = fr ? 1.0 : 0.0;
  for (int i = 0; i < 3; ++i) kmu[3 * c + i] = fr ? R[1][i] * ln : 0.0;
}

// Add the contact blocks to the diagonal block slots; the first contact of
// each vertex (contacts are sorted by vertex) adds the whole group.
__global__ void k_contact_fold(int nc, const int* __restrict__ vid, const int* __restrict__ diag_slot,
                               const double* __restrict__ Wt, double* __restrict__ val) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int v = vid[c];
  if (c > 0 && vid[c - 1] == v) return;
  double acc[9];
  for (int e = 0; e < 9; ++e) acc[e] = 0.0;
  for (int k = c; k < nc && vid[k] == v; ++k)
    for (int e = 0; e < 9; ++e) acc[e] += Wt[9 * k + e];
  double* o = val + 9 * (size_t)diag_slot[v];
  for (int e = 0; e < 9; ++e) o[e] += acc[e];
}

// C[r][r'] (row-major m x m) for the transposed system.
__global__ void k_capacitance(int m, int mp, const int* __restrict__ row_c, const int* __restrict__ row_i,
                              const int* __restrict__ cmap, int ncv, const double* __restrict__ D,
                              const double* __restrict__ Q, const double* __restrict__ kh, double mu,
                              double h2, int transpose, double* __restrict__ C) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= m || i >= m) return;
  const int c = row_c[i], a = row_i[i];
  const int c2 = row_c[j], b = row_i[j];
  const double* q1 = Q + 9 * c + 3 * a;
  const double* q2 = Q + 9 * c2 + 3 * b;
  double v = h2 * D[(size_t)cmap[c] * ncv + cmap[c2]] * (q1[0] * q2[0] + q1[1] * q2[1] + q1[2] * q2[2]);
  if (c == c2) {
    // Khat^{-T} = [[1/a, mu/b, 0], [0, 1/b, 0], [0, 0, 1/c]]; a zero c
    // (no friction magnitude) drops the row from the low-rank term.
    const double ka = kh[4 * c], kb = kh[4 * c + 1], kc = kh[4 * c + 2];
    // Khat^{-1} (forward Newton, transpose = 0) has mu/b at (1, 0) instead
    if (a == 0 && b == 0) v += 1.0 / ka;
    else if (transpose ? (a == 0 && b == 1) : (a == 1 && b == 0)) v += mu / kb;
    else if (a == 1 && b == 1) v += 1.0 / kb;
    else if (a == 2 && b == 2) v += (kc > 1e-200) ? 1.0 / kc : 1e200;
  }
  C[(size_t)i * mp + j] = v;
}

// Contact part of the state gradient and the friction-coefficient gradient:
//   dL/dqbar_v += h^2 frame^T P_f K_c^T (frame z_v)  (transpose of K_qbar's contact term)
//   dL/dmu     += -h^2 sum_c (frame z_v) . k_mu
__global__ void __launch_bounds__(256) k_vjp_contacts(int nc, const int* __restrict__ vid,
                                                      const double* __restrict__ frame,
                                                      const double* __restrict__ Kc,
                                                      const double* __restrict__ kmu,
                                                      const double* __restrict__ z, double h2,
                                                      double* __restrict__ dqbar,
                                                      double* __restrict__ partial,
                                                      double* __restrict__ gmu_c) {
  __shared__ double lds[32];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double gmu = 0.0;
  if (c < nc) {
    const int v = vid[c];
    const double zv[3] = {z[3 * v], z[3 * v + 1], z[3 * v + 2]};
    double Hz[3];
    for (int i = 0; i < 3; ++i)
      Hz[i] = frame[9 * c + 3 * i] * zv[0] + frame[9 * c + 3 * i + 1] * zv[1] + frame[9 * c + 3 * i + 2] * zv[2];
    gmu = -h2 * (Hz[0] * kmu[3 * c] + Hz[1] * kmu[3 * c + 1] + Hz[2] * kmu[3 * c + 2]);
    if (gmu_c) gmu_c[c] = gmu;
    if (!(c > 0 && vid[c - 1] == v)) {  // first contact of the vertex adds the group
      double add[3] = {0, 0, 0};
      for (int k = c; k < nc && vid[k] == v; ++k) {
        double hz[3], t[3];
        for (int i = 0; i < 3; ++i)
          hz[i] = frame[9 * k + 3 * i] * zv[0] + frame[9 * k + 3 * i + 1] * zv[1] + frame[9 * k + 3 * i + 2] * zv[2];
        for (int i = 0; i < 3; ++i)  // K_c^T (H_c z)
          t[i] = Kc[9 * k + i] * hz[0] + Kc[9 * k + 3 + i] * hz[1] + Kc[9 * k + 6 + i] * hz[2];
        t[0] = 0.0;  // P_f = Diag(0, 1, 1)
        for (int j = 0; j < 3; ++j)
          add[j] += h2 * (frame[9 * k + j] * t[0] + frame[9 * k + 3 + j] * t[1] + frame[9 * k + 6 + j] * t[2]);
      }
      for (int j = 0; j < 3; ++j) dqbar[3 * v + j] += add[j];
    }
  }
  double s = block_sum(gmu, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void launch_add_partials(hipStream_t st, const double* partial, int nb, int k, double* grad);

// dL/dqbar = M z - dL_dv/h, dL/dvbar = h M z, dL/dfext = h^2 z.
__global__ void k_vjp_vectors(int nv, const double* __restrict__ z, const double* __restrict__ gv,
                              const double* __restrict__ mass, double h, double* __restrict__ dqbar,
                              double* __restrict__ dvbar, double* __restrict__ dfext) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nv) return;
  const double m = mass[i / 3], zi = z[i];
  dqbar[i] = m * zi - gv[i] / h;
  dvbar[i] = h * m * zi;
  dfext[i] = (h * h) * zi;
}

void launch_contact_blocks(hipStream_t st, int nc, const int* fric, const double* frame,
                           const double* delta, const double* lam, double mu, const double* mu_c, double eps,
                           double h2, int transpose, double* Wt, double* Q, double* kh, double* Kc,
                           double* kmu) {
  if (nc == 0) return;
  k_contact_blocks<<<(nc + 63) / 64, 64, 0, st>>>(nc, fric, frame, delta, lam, mu, mu_c, eps, h2, transpose,
                                                   Wt, Q, kh, Kc, kmu);
}

// Bilateral bindings (eq:binding): h^2 E_b^{-1} I onto the diagonal block of
// each bound vertex (the vertices are distinct: one writer per block).
__global__ void k_binding_fold(int nb, const int* __restrict__ bvid, const double* __restrict__ bE, double h2,
                               const int* __restrict__ diag_slot, double* __restrict__ val) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double* d = val + 9LL * diag_slot[bvid[b]];
  const double c = h2 / bE[b];
  d[0] += c;
  d[4] += c;
  d[8] += c;
}

// Binding gradients (eq:differential_2, rhs_d_b and rhs_E_b) with the binding
// force lambda_b = -(q_b - d_b) / E_b:  dL/dd_b = h^2 z_b / E_b,
// dL/dE_b = -h^2 (lambda_b . z_b) / E_b.
__global__ void k_binding_vjp(int nb, const int* __restrict__ bvid, const double* __restrict__ bE, double h2,
                              const double* __restrict__ z, const double* __restrict__ q,
                              const double* __restrict__ target, double* __restrict__ dtarget,
                              double* __restrict__ dE) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int v = bvid[b];
  const double e = bE[b];
  double dot = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double zk = z[3 * v + k];
    const double lam = -(q[3 * v + k] - target[3 * b + k]) / e;
    dtarget[3 * b + k] = h2 * zk / e;
    dot += lam * zk;
  }
  dE[b] = -h2 * dot / e;
}

// Binding rows of the forward residual (eq:binding): r_v += h^2 (q_v - d_b) / E_b,
// i.e. -h^2 lambda_b with lambda_b = -(q_v - d_b) / E_b.  Bound vertices are
// distinct, so no two threads add to one row.
__global__ void k_binding_force(int nb, const int* __restrict__ bvid, const double* __restrict__ bE, double h2,
                                const double* __restrict__ q, const double* __restrict__ target,
                                double* __restrict__ r) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int v = bvid[b];
  const double c = h2 / bE[b];
  for (int k = 0; k < 3; ++k) r[3 * v + k] += c * (q[3 * v + k] - target[3 * b + k]);
}

void launch_binding_force(hipStream_t st, int nb, const int* bvid, const double* bE, double h2, const double* q,
                          const double* target, double* r) {
  if (nb == 0) return;
  k_binding_force<<<(nb + 63) / 64, 64, 0, st>>>(nb, bvid, bE, h2, q, target, r);
}

void launch_binding_fold(hipStream_t st, int nb, const int* bvid, const double* bE, double h2, const int* diag_slot,
                         double* val) {
  if (nb == 0) return;
  k_binding_fold<<<(nb + 63) / 64, 64, 0, st>>>(nb, bvid, bE, h2, diag_slot, val);
}

void launch_binding_vjp(hipStream_t st, int nb, const int* bvid, const double* bE, double h2, const double* z,
                        const double* q, const double* target, double* dtarget, double* dE) {
  if (nb == 0) return;
  k_binding_vjp<<<(nb + 63) / 64, 64, 0, st>>>(nb, bvid, bE, h2, z, q, target, dtarget, dE);
}

void launch_contact_fold(hipStream_t st, int nc, const int* vid, const int* diag_slot,
                         const double* Wt, double* val) {
  if (nc == 0) return;
  k_contact_fold<<<(nc + 63) / 64, 64, 0, st>>>(nc, vid, diag_slot, Wt, val);
}

void launch_capacitance(hipStream_t st, int m, int mp, const int* row_c, const int* row_i,
                        const int* cmap, int ncv, const double* D, const double* Q, const double* kh,
                        double mu, double h2, int transpose, double* C) {
  if (m == 0) return;
  dim3 grid((m + 255) / 256, m);
  k_capacitance<<<grid, 256, 0, st>>>(m, mp, row_c, row_i, cmap, ncv, D, Q, kh, mu, h2, transpose, C);
}

void launch_vjp_contacts(hipStream_t st, int nc, const int* vid, const double* frame, const double* Kc,
                         const double* kmu, const double* z, double h2, double* dqbar, double* partial,
                         double* grad, double* gmu_c) {
  if (nc == 0) return;
  const int nb = (nc + 255) / 256;
  k_vjp_contacts<<<nb, 256, 0, st>>>(nc, vid, frame, Kc, kmu, z, h2, dqbar, partial, gmu_c);
  if (grad) launch_add_partials(st, partial, nb, 1, grad + 2);
}

void launch_vjp_vectors(hipStream_t st, int nv, const double* z, const double* gv, const double* mass,
                        double h, double* dqbar, double* dvbar, double* dfext) {
  k_vjp_vectors<<<(3 * nv + 255) / 256, 256, 0, st>>>(nv, z, gv, mass, h, dqbar, dvbar, dfext);
}

}  // namespace adj
