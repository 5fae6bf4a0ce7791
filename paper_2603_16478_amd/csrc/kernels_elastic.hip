// Elastic part of the adjoint matrix and of the parameter gradients.
//
// k_tet_blocks: one thread per tet.  Deformation gradient, SVD, Neo-Hookean
// prox singular values, and the element matrix
//     E_i = h^2 w_i G_i^T (I - J_i) G_i,   w_i = 2 mu_i V_i,
// with J_i = dvecP/dvecF = (V(x)U)[D W D^T + Diag(vec M) + Diag(vec N) T](V(x)U)^T
// (Sec. 5.3, App. B.0; the T term carries N, as the element-wise derivation
// requires).  With BV = Bt V (4x3) the 3x3 block (k,l) of G^T J G is
// U Y^{kl} U^T where
//     Y_ab = W_ab BV_ka BV_lb + [a=b] sum_{j!=a} M_aj BV_kj BV_lj + [a!=b] N_ab BV_kb BV_la,
// so E_kl = h^2 w ((Bt_k . Bt_l) I - U Y^{kl} U^T).  The 10 blocks k <= l are
// stored pair-major (E_lk = E_kl^T): out[(pair*nt + t)*9 + 3r + c].
//
// k_assemble: nine threads per block slot of Acal^T (one per entry); each
// sums its entry over the slot's element contributions in the fixed order of
// the element-to-entry map (Sec. 5.4, matrix assembly) and adds the lumped
// mass on the diagonal.
#include "device_common.h"
#include "nh_local.h"

namespace adj {

__constant__ int c_pairK[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__constant__ int c_pairL[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

// tets and Bt entry-major: vertex k of tet t at tets[k nt + t], B~[k][c] at Bt[(3k + c) nt + t]
__device__ __forceinline__ void load_tet(int t, int nt, const int* __restrict__ tets,
                                         const double* __restrict__ Bt, const double* __restrict__ q,
                                         double x[4][3], double B[4][3], int vid[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    vid[k] = tets[(size_t)k * nt + t];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[k][c] = q[3 * vid[k] + c];
      B[k][c] = Bt[(size_t)(3 * k + c) * nt + t];
    }
  }
}

__global__ void __launch_bounds__(128) k_tet_blocks(int nt, const int* __restrict__ tets,
                                                    const double* __restrict__ Bt,
                                                    const double* __restrict__ vol,
                                                    const double* __restrict__ lmu,
                                                    const double* __restrict__ llam, double h2,
                                                    const double* __restrict__ q,
                                                    double* __restrict__ out, int* __restrict__ err,
                                                    int model) {
  // pair-major output, out[(pr nt + t) 9 + 3r + c]: per pair the block's 128
  // tets write one contiguous run, staged through LDS
  __shared__ double stage[128 * 9];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int t0 = blockIdx.x * blockDim.x, nloc = min((int)blockDim.x, nt - t0);
  bool ok = false;
  double U[3][3], B[4][3], W[3][3], M[3][3], N[3][3], BV[4][3];
  double scale = 0.0;
  if (t < nt) {
    double x[4][3];
    int vid[4];
    load_tet(t, nt, tets, Bt, q, x, B, vid);
    double F[3][3];
    deformation_gradient(x, B, F);
    ok = det3(F) > 0.0;
    if (!ok) {
      err[0] = 1;  // inverted element: its blocks are written as zeros
    } else {
      const double mu = lmu[t], lam = llam[t];
      double s[3], V[3][3];
      svd3(F, U, s, V);
      NHLocal L;
      double th[3], qd[3][3];
      local_projection(model, s, mu, lam, th, W, qd, L);
      local_MN(th, s, qd, M, N);
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) BV[k][j] = B[k][0] * V[0][j] + B[k][1] * V[1][j] + B[k][2] * V[2][j];
      scale = h2 * 2.0 * mu * vol[t];
    }
  }
#pragma unroll
  for (int pr = 0; pr < 10; ++pr) {
    double o[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) o[e] = 0.0;
    if (ok) {
      const int k = c_pairK[pr], l = c_pairL[pr];
      double Y[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          double y = W[a][b] * BV[k][a] * BV[l][b];
          if (a == b) {
#pragma unroll
            for (int j = 0; j < 3; ++j)
              if (j != a) y += M[a][j] * BV[k][j] * BV[l][j];
          } else {
            y += N[a][b] * BV[k][b] * BV[l][a];
          }
          Y[a][b] = y;
        }
      // T = U Y, R = T U^T
      double T[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b) T[r][b] = U[r][0] * Y[0][b] + U[r][1] * Y[1][b] + U[r][2] * Y[2][b];
      const double bb = B[k][0] * B[l][0] + B[k][1] * B[l][1] + B[k][2] * B[l][2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double uyu = T[r][0] * U[c][0] + T[r][1] * U[c][1] + T[r][2] * U[c][2];
          o[3 * r + c] = scale * (((r == c) ? bb : 0.0) - uyu);
        }
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) stage[9 * threadIdx.x + e] = o[e];
    __syncthreads();
    double* dst = out + ((size_t)pr * nt + t0) * 9;
    for (int i = threadIdx.x; i < 9 * nloc; i += blockDim.x) dst[i] = stage[i];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_assemble(int nnzb, int nt, const int* __restrict__ slot_ptr,
                                                  const int* __restrict__ slot_code,
                                                  const double* __restrict__ tetblk,
                                                  const int* __restrict__ row_of_slot,
                                                  const int* __restrict__ col,
                                                  const double* __restrict__ mass,
                                                  double* __restrict__ val) {
  // nine threads per slot, one per entry: the nine threads of a slot read
  // each element block's 72 contiguous bytes together, and the slots' values
  // are written contiguously.  Blocks go to the eight XCDs round-robin, each
  // with its own L2; the logical block index gives XCD x one contiguous
  // range of rows, so the element blocks shared by nearby rows (a tet's
  // blocks feed the rows of its four vertices) are fetched into one L2.
  const unsigned nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, x8 = blockIdx.x % 8;
  const unsigned lb = x8 * q8 + min(x8, r8) + blockIdx.x / 8;
  const long long g = (long long)lb * blockDim.x + threadIdx.x;
  if (g >= 9LL * nnzb) return;
  const int sl = (int)(g / 9), e = (int)(g - 9LL * sl);
  const int r = e / 3, c = e - 3 * r;
  const int et = 3 * c + r;  // the same entry of the transposed block
  double acc = 0.0;
  const int p0 = slot_ptr[sl], p1 = slot_ptr[sl + 1];
#pragma unroll 4
  for (int p = p0; p < p1; ++p) {
    const int code = slot_code[p];
    const int t = code >> 5, pr = (code >> 1) & 15, tr = code & 1;
    acc += tetblk[((size_t)pr * nt + t) * 9 + (tr ? et : e)];
  }
  if (r == c) {
    const int row = row_of_slot[sl];
    if (col[sl] == row) acc += mass[row];
  }
  val[g] = acc;
}

// Per-tet parameter gradients (App. B.3, with w_i = 2 mu_i V_i):
//   dL/dmu_i  = 2 h^2 V_i (G_i z) . (mu_i dp/dmu + p_i - G_i q)
//   dL/dlam_i = 2 h^2 V_i mu_i (G_i z) . dp/dlam
// dp/dmu = vec(U Diag(dtheta/dmu) V^T), dtheta/dmu = -(dg/dtheta)^{-1}(3 theta - 2 sigma - 1/theta),
// dtheta/dlam = -(dg/dtheta)^{-1}(log J / theta); then the chain rule to E, nu.
// Writes per-tet dE, dnu (accumulate) when requested and per-block partial
// sums (partial[2b], partial[2b+1]); k_add_partials adds the totals to
// grad[0], grad[1].
__global__ void __launch_bounds__(256) k_vjp_tets(int nt, const int* __restrict__ tets,
                                                  const double* __restrict__ Bt,
                                                  const double* __restrict__ vol,
                                                  const double* __restrict__ lmu,
                                                  const double* __restrict__ llam,
                                                  const double* __restrict__ Ev,
                                                  const double* __restrict__ nuv, double h2,
                                                  const double* __restrict__ q,
                                                  const double* __restrict__ z,
                                                  double* __restrict__ dE_tet,
                                                  double* __restrict__ dnu_tet,
                                                  double* __restrict__ partial, int model) {
  __shared__ double lds[32];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double gE = 0.0, gnu = 0.0;
  if (t < nt) {
    double x[4][3], B[4][3], zz[4][3];
    int vid[4];
    load_tet(t, nt, tets, Bt, q, x, B, vid);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) zz[k][c] = z[3 * vid[k] + c];
    double F[3][3], Fz[3][3];
    deformation_gradient(x, B, F);
    deformation_gradient(zz, B, Fz);
    const double mu = lmu[t], lam = llam[t];
    double U[3][3], s[3], V[3][3];
    svd3(F, U, s, V);
    NHLocal L;
    double th[3], W[3][3], qd[3][3], dmu[3], dlam[3];
    local_projection(model, s, mu, lam, th, W, qd, L);
    local_param_derivs(model, s, th, mu, lam, L, dmu, dlam);
    // (G z) . vec(U Diag(d) V^T) = sum_i d_i (U^T Fz V)_ii ; (G z).(p - G q) = Fz : (P - F)
    double zmu = 0.0, zlam = 0.0, zp = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double xi = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) xi += U[r][i] * Fz[r][c] * V[c][i];
      zmu += dmu[i] * xi;
      zlam += dlam[i] * xi;
      zp += th[i] * xi;  // Fz : P
    }
    double zf = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) zf += Fz[r][c] * F[r][c];
    const double V2 = 2.0 * h2 * vol[t];
    const double gm = V2 * (mu * zmu + zp - zf);
    const double gl = V2 * mu * zlam;
    const double E = Ev[t], nu = nuv[t];
    const double opn = 1.0 + nu, omn = 1.0 - 2.0 * nu;
    gE = gm / (2.0 * opn) + gl * nu / (opn * omn);
    gnu = -gm * E / (2.0 * opn * opn) + gl * E * (1.0 + 2.0 * nu * nu) / (opn * opn * omn * omn);
    if (dE_tet) dE_tet[t] += gE;
    if (dnu_tet) dnu_tet[t] += gnu;
  }
  double sE = block_sum(gE, lds);
  double sN = block_sum(gnu, lds);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sE;
    partial[2 * blockIdx.x + 1] = sN;
  }
}

// One block: grad[c] += sum_b partial[b * k + c], c < k (fixed order).
__global__ void __launch_bounds__(256) k_add_partials(const double* __restrict__ partial, int nb, int k,
                                                      double* __restrict__ grad) {
  __shared__ double lds[32];
  for (int c = 0; c < k; ++c) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) a += partial[(size_t)b * k + c];
    a = block_sum(a, lds);
    if (threadIdx.x == 0) grad[c] += a;
  }
}

void launch_add_partials(hipStream_t st, const double* partial, int nb, int k, double* grad) {
  if (nb <= 0) return;
  k_add_partials<<<1, 256, 0, st>>>(partial, nb, k, grad);
}

void launch_tet_blocks(hipStream_t st, int nt, const int* tets, const double* Bt, const double* vol,
                       const double* lmu, const double* llam, double h2, const double* q, double* out,
                       int* err, int model) {
  k_tet_blocks<<<(nt + 127) / 128, 128, 0, st>>>(nt, tets, Bt, vol, lmu, llam, h2, q, out, err, model);
}

// tetblk: the pair-major element blocks of k_tet_blocks for nt tets
void launch_assemble(hipStream_t st, int nnzb, int nt, const int* slot_ptr, const int* slot_code,
                     const double* tetblk, const int* row_of_slot, const int* col, const double* mass,
                     double* val) {
  k_assemble<<<(unsigned)((9LL * nnzb + 255) / 256), 256, 0, st>>>(nnzb, nt, slot_ptr, slot_code, tetblk,
                                                                    row_of_slot, col, mass, val);
}

void launch_vjp_tets(hipStream_t st, int nt, const int* tets, const double* Bt, const double* vol,
                     const double* lmu, const double* llam, const double* Ev, const double* nuv,
                     double h2, const double* q, const double* z, double* dE_tet, double* dnu_tet,
                     double* partial, double* grad, int model) {
  const int nb = (nt + 255) / 256;
  k_vjp_tets<<<nb, 256, 0, st>>>(nt, tets, Bt, vol, lmu, llam, Ev, nuv, h2, q, z, dE_tet, dnu_tet, partial,
                                 model);
  if (grad) launch_add_partials(st, partial, nb, 2, grad);
}

}  // namespace adj
