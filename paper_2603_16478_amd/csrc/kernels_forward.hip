// Kernels of the forward step (eq:dynamics): inertial prediction, contact
// candidates, elastic forces of the local projections, per-vertex residual
// gather and small reductions.  The Newton matrix reuses the adjoint's
// per-tet Jacobian and assembly kernels (the reduced Newton matrix is Acal).
#include "device_common.h"
#include "nh_local.h"

namespace adj {

// Prediction and detection are evaluated left to right without contraction
// so that the candidate decisions are reproducible bit for bit.
#pragma clang fp contract(off)

// qtilde = (qbar + h vbar) + (h*h) (g + f/m);  utilde = h vbar + (h*h) (g + f/m)
__global__ void k_fwd_predict(int nv, const double* __restrict__ qbar, const double* __restrict__ vbar,
                              const double* __restrict__ fext, const double* __restrict__ mass, double h,
                              double gx, double gy, double gz, double* __restrict__ utilde,
                              double* __restrict__ qtilde) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nv) return;
  const int c = i % 3;
  const double g = (c == 0) ? gx : (c == 1) ? gy : gz;
  const double acc = g + fext[i] / mass[i / 3];
  const double hh = h * h;
  qtilde[i] = (qbar[i] + h * vbar[i]) + hh * acc;
  utilde[i] = h * vbar[i] + hh * acc;
}

// mask bit 2p: gap to collider p at qtilde <= margin; bit 2p+1: gap <= 0.
// Colliders 0..nplanes-1 are the planes, then the kinematic spheres: a
// sphere's contact plane has the normal n = (qbar_v - c_old)/|qbar_v - c_old|
// and the offset n . c_new + r (the tangent plane at the step's new pose).
__global__ void k_fwd_detect(int nv, const double* __restrict__ qbar, const double* __restrict__ qtilde,
                             int nplanes, const double* __restrict__ planes, int nspheres,
                             const double* __restrict__ sph_old, const double* __restrict__ sph_new, double margin,
                             int* __restrict__ mask) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  int mk = 0;
  const double x0 = qtilde[3 * v], x1 = qtilde[3 * v + 1], x2 = qtilde[3 * v + 2];
  for (int p = 0; p < nplanes && p < 15; ++p) {
    const double* pl = planes + 4 * p;
    const double gap = ((pl[0] * x0 + pl[1] * x1) + pl[2] * x2) - pl[3];
    if (gap <= margin) mk |= 1 << (2 * p);
    if (gap <= 0.0) mk |= 1 << (2 * p + 1);
  }
  for (int s = 0; s < nspheres && nplanes + s < 15; ++s) {
    const double* c0 = sph_old + 4 * s;
    const double* c1 = sph_new + 4 * s;
    const double d0 = qbar[3 * v] - c0[0], d1 = qbar[3 * v + 1] - c0[1], d2 = qbar[3 * v + 2] - c0[2];
    const double nrm = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
    if (nrm == 0.0) continue;
    const double n0 = d0 / nrm, n1 = d1 / nrm, n2 = d2 / nrm;
    const double dn = ((n0 * c1[0] + n1 * c1[1]) + n2 * c1[2]) + c1[3];
    const double gap = ((n0 * x0 + n1 * x1) + n2 * x2) - dn;
    const int p = nplanes + s;
    if (gap <= margin) mk |= 1 << (2 * p);
    if (gap <= 0.0) mk |= 1 << (2 * p + 1);
  }
  mask[v] = mk;
}

#pragma clang fp contract(on)

__global__ void k_add_vec(long long n, const double* __restrict__ a, const double* __restrict__ b, double alpha,
                          double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + alpha * b[i];
}

__global__ void k_scale_vec(long long n, const double* __restrict__ a, double alpha, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = alpha * a[i];
}

// Elastic force of the local projections (eq:internal, eq:dynamics):
// h^2 w_i G_i^T (G_i q - p_i), w_i = 2 mu_i V_i, p_i = vec(U Theta V^T).
// out[t*12 + 3k + r] = h^2 w_i sum_c Bt[k][c] (F - P)[r][c].
__global__ void __launch_bounds__(128) k_tet_force(int nt, const int* __restrict__ tets,
                                                   const double* __restrict__ Bt,
                                                   const double* __restrict__ vol,
                                                   const double* __restrict__ lmu,
                                                   const double* __restrict__ llam, double h2,
                                                   const double* __restrict__ q, double* __restrict__ out,
                                                   int* __restrict__ err, int model) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double x[4][3], B[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int v = tets[(size_t)k * nt + t];  // tets and Bt entry-major (entry e of tet t at e nt + t)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[k][c] = q[3 * v + c];
      B[k][c] = Bt[(size_t)(3 * k + c) * nt + t];
    }
  }
  double F[3][3];
  deformation_gradient(x, B, F);
  if (!(det3(F) > 0.0)) {
    err[1] = 1;
    for (int e = 0; e < 12; ++e) out[12 * (size_t)t + e] = 0.0;
    return;
  }
  const double mu = lmu[t], lam = llam[t];
  double U[3][3], s[3], V[3][3];
  svd3(F, U, s, V);
  double th[3];
  local_theta(model, s, mu, lam, th);
  double Dm[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Dm[r][c] = F[r][c] - (U[r][0] * th[0] * V[c][0] + U[r][1] * th[1] * V[c][1] + U[r][2] * th[2] * V[c][2]);
  const double sc = h2 * 2.0 * mu * vol[t];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r)
      out[12 * (size_t)t + 3 * k + r] = sc * (B[k][0] * Dm[r][0] + B[k][1] * Dm[r][1] + B[k][2] * Dm[r][2]);
}

// r_v = m_v (u_v - utilde_v) + sum over incident (tet, corner) of the element force
__global__ void k_gather_force(int nv, const int* __restrict__ vptr, const int* __restrict__ vcode,
                               const double* __restrict__ force, const double* __restrict__ mass,
                               const double* __restrict__ u, const double* __restrict__ utilde,
                               double* __restrict__ r) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int p = vptr[v]; p < vptr[v + 1]; ++p) {
    const int code = vcode[p];
    const double* f = force + 12 * (size_t)(code >> 2) + 3 * (code & 3);
    a0 += f[0];
    a1 += f[1];
    a2 += f[2];
  }
  const double m = mass[v];
  r[3 * v] = m * (u[3 * v] - utilde[3 * v]) + a0;
  r[3 * v + 1] = m * (u[3 * v + 1] - utilde[3 * v + 1]) + a1;
  r[3 * v + 2] = m * (u[3 * v + 2] - utilde[3 * v + 2]) + a2;
}

// out[v] += sum of vec over the contacts at v (contacts sorted by vertex)
__global__ void k_add_contact_vec(int nc, const int* __restrict__ vid, const double* __restrict__ vec,
                                  double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int v = vid[c];
  if (c > 0 && vid[c - 1] == v) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int k = c; k < nc && vid[k] == v; ++k) {
    a0 += vec[3 * k];
    a1 += vec[3 * k + 1];
    a2 += vec[3 * k + 2];
  }
  out[3 * v] += a0;
  out[3 * v + 1] += a1;
  out[3 * v + 2] += a2;
}

__global__ void k_gather_contact_rows(int nc, const int* __restrict__ vid, const double* __restrict__ x,
                                      double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int v = vid[c];
  out[3 * c] = x[3 * v];
  out[3 * c + 1] = x[3 * v + 1];
  out[3 * c + 2] = x[3 * v + 2];
}

// out[0] = sum x_i^2, out[1] = max |x_i|: per-block partials, then one
// block sums them in fixed order.
__global__ void __launch_bounds__(256) k_norms(long long n, const double* __restrict__ x,
                                               double* __restrict__ partial) {
  __shared__ double lds[32];
  __shared__ double mx[8];
  double s = 0.0, m = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = x[i];
    s += v * v;
    m = fmax(m, fabs(v));
  }
  s = block_sum(s, lds);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) mx[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int i = 0; i < (int)blockDim.x / 64; ++i) mm = fmax(mm, mx[i]);
    partial[2 * blockIdx.x] = s;
    partial[2 * blockIdx.x + 1] = mm;
  }
}

__global__ void __launch_bounds__(64) k_norms_finish(const double* __restrict__ partial, int nb,
                                                     double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < nb; ++i) {
    a += partial[2 * i];
    b = fmax(b, partial[2 * i + 1]);
  }
  out[0] = a;
  out[1] = b;
}

void launch_fwd_predict(hipStream_t st, int nv, const double* qbar, const double* vbar, const double* fext,
                        const double* mass, double h, const double* g, double* utilde, double* qtilde) {
  k_fwd_predict<<<(3 * nv + 255) / 256, 256, 0, st>>>(nv, qbar, vbar, fext, mass, h, g[0], g[1], g[2], utilde,
                                                      qtilde);
}

void launch_fwd_detect(hipStream_t st, int nv, const double* qbar, const double* qtilde, int nplanes,
                       const double* planes, int nspheres, const double* sph_old, const double* sph_new,
                       double margin, int* mask) {
  k_fwd_detect<<<(nv + 255) / 256, 256, 0, st>>>(nv, qbar, qtilde, nplanes, planes, nspheres, sph_old, sph_new,
                                                 margin, mask);
}

// ---- active stress of an actuated body: tet t of group g carries the
// first Piola stress a_g d d^T (fibre d), nodal force -V a_g (d d^T) grad N_k.

__global__ void k_act_tet(int nt, const int* __restrict__ group, const double* __restrict__ fibre,
                          const double* __restrict__ Bt, const double* __restrict__ vol, const double* __restrict__ a,
                          double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const double d0 = fibre[3 * t], d1 = fibre[3 * t + 1], d2 = fibre[3 * t + 2];
  const double sc = -vol[t] * a[group[t]];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double* g = Bt + (size_t)(3 * k) * nt + t;  // entry-major
    const double c = sc * (d0 * g[0] + d1 * g[nt] + d2 * g[2 * (size_t)nt]);
    double* o = out + 12 * (size_t)t + 3 * k;
    o[0] = c * d0;
    o[1] = c * d1;
    o[2] = c * d2;
  }
}

// out_v = sum over the incident (tet, corner) pairs of the per-tet values
__global__ void k_gather_vec(int nv, const int* __restrict__ vptr, const int* __restrict__ vcode,
                             const double* __restrict__ v12, double* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int p = vptr[v]; p < vptr[v + 1]; ++p) {
    const int code = vcode[p];
    const double* f = v12 + 12 * (size_t)(code >> 2) + 3 * (code & 3);
    a0 += f[0];
    a1 += f[1];
    a2 += f[2];
  }
  out[3 * v] = a0;
  out[3 * v + 1] = a1;
  out[3 * v + 2] = a2;
}

// s_t = -V_t sum_k (g_{v_k} . d)(d . grad N_k): tet t's share of dL/da_g
__global__ void k_act_vjp_tet(int nt, const int* __restrict__ tets, const double* __restrict__ fibre,
                              const double* __restrict__ Bt, const double* __restrict__ vol,
                              const double* __restrict__ g, double* __restrict__ s) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const double d0 = fibre[3 * t], d1 = fibre[3 * t + 1], d2 = fibre[3 * t + 2];
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int v = tets[(size_t)k * nt + t];  // entry-major
    const double* b = Bt + (size_t)(3 * k) * nt + t;
    acc += (g[3 * v] * d0 + g[3 * v + 1] * d1 + g[3 * v + 2] * d2) * (d0 * b[0] + d1 * b[nt] + d2 * b[2 * (size_t)nt]);
  }
  s[t] = -vol[t] * acc;
}

// out[g] = sum of s over the tets of group g in list order (one block per group)
__global__ void __launch_bounds__(256) k_group_sum(int ng, const int* __restrict__ gptr, const int* __restrict__ gtets,
                                                   const double* __restrict__ s, double* __restrict__ out) {
  __shared__ double lds[32];
  const int g = blockIdx.x;
  if (g >= ng) return;
  double a = 0.0;
  for (int p = gptr[g] + threadIdx.x; p < gptr[g + 1]; p += blockDim.x) a += s[gtets[p]];
  a = block_sum(a, lds);
  if (threadIdx.x == 0) out[g] = a;
}

void launch_actuation_force(hipStream_t st, int nt, int nv, const int* group, const double* fibre, const double* Bt,
                            const double* vol, const int* vptr, const int* vcode, const double* a, double* buf12,
                            double* f) {
  k_act_tet<<<(nt + 255) / 256, 256, 0, st>>>(nt, group, fibre, Bt, vol, a, buf12);
  k_gather_vec<<<(nv + 255) / 256, 256, 0, st>>>(nv, vptr, vcode, buf12, f);
}

void launch_actuation_vjp(hipStream_t st, int nt, int ng, const int* tets, const double* fibre, const double* Bt,
                          const double* vol, const int* gptr, const int* gtets, const double* g, double* s,
                          double* da) {
  k_act_vjp_tet<<<(nt + 255) / 256, 256, 0, st>>>(nt, tets, fibre, Bt, vol, g, s);
  k_group_sum<<<ng, 256, 0, st>>>(ng, gptr, gtets, s, da);
}

void launch_add_vec(hipStream_t st, long long n, const double* a, const double* b, double alpha, double* out) {
  k_add_vec<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a, b, alpha, out);
}

void launch_scale_vec(hipStream_t st, long long n, const double* a, double alpha, double* out) {
  k_scale_vec<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a, alpha, out);
}

void launch_tet_force(hipStream_t st, int nt, const int* tets, const double* Bt, const double* vol,
                      const double* lmu, const double* llam, double h2, const double* q, double* out, int* err,
                      int model) {
  k_tet_force<<<(nt + 127) / 128, 128, 0, st>>>(nt, tets, Bt, vol, lmu, llam, h2, q, out, err, model);
}

void launch_gather_force(hipStream_t st, int nv, const int* vptr, const int* vcode, const double* force,
                         const double* mass, const double* u, const double* utilde, double* r) {
  k_gather_force<<<(nv + 255) / 256, 256, 0, st>>>(nv, vptr, vcode, force, mass, u, utilde, r);
}

void launch_add_contact_vec(hipStream_t st, int nc, const int* vid, const double* vec, double* out) {
  if (nc == 0) return;
  k_add_contact_vec<<<(nc + 255) / 256, 256, 0, st>>>(nc, vid, vec, out);
}

void launch_gather_contact_rows(hipStream_t st, int nc, const int* vid, const double* x, double* out) {
  if (nc == 0) return;
  k_gather_contact_rows<<<(nc + 255) / 256, 256, 0, st>>>(nc, vid, x, out);
}

void launch_norms(hipStream_t st, long long n, const double* x, double* partial, double* out) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 256) blocks = 256;
  k_norms<<<blocks, 256, 0, st>>>(n, x, partial);
  k_norms_finish<<<1, 64, 0, st>>>(partial, blocks, out);
}

}  // namespace adj
