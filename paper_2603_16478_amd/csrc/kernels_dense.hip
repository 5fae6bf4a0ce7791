// Delassus operator of the contact vertices and the dense inverse of the
// Woodbury capacitance (Sec. 5.4, eq:woodbury_formula).
//
// With A^{-1} = S^T S (Sec. 3.4) and E the selector of the contact vertices,
//   Y = S E           (n_v x n_cv, the columns of S at the contact vertices)
//   D = Y^T Y = E^T A_s^{-1} E       (the scalar Delassus matrix)
//   Z = S^T Y = A_s^{-1} E           (used by every preconditioner apply)
// D and Z depend only on the contact vertex set and are reused while it
// stays the same (the paper caches the Delassus operator across the step).
//
// The capacitance is inverted by block Gauss-Jordan elimination with 32x32
// diagonal block pivots (each inverted with partial pivoting), which keeps
// every step a dense rank-32 update: X = C^{-1} in place, so a
// preconditioner apply needs one dense matrix-vector product.
#include "device_common.h"

namespace adj {

__global__ void k_fill_zero(size_t n, double* __restrict__ a) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

// Y[r][c] = S[r][cv[c]] from the rows of S^T (row-major n_v x ncv).
__global__ void k_fill_Y(int ncv, const int* __restrict__ cv, const long long* __restrict__ STp,
                         const int* __restrict__ STj, const double* __restrict__ STx,
                         double* __restrict__ Y) {
  const int c = blockIdx.x;
  if (c >= ncv) return;
  const int v = cv[c];
  for (long long p = STp[v] + threadIdx.x; p < STp[v + 1]; p += blockDim.x)
    Y[(size_t)STj[p] * ncv + c] = STx[p];
}

// D = Y^T Y, 16x16 output tile per 256-thread block, K split over 16 rows.
__global__ void __launch_bounds__(256) k_syrk(int nv, int ncv, const double* __restrict__ Y,
                                              double* __restrict__ D) {
  __shared__ double ta[16][17], tb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int a0 = blockIdx.y * 16, b0 = blockIdx.x * 16;
  double acc = 0.0;
  for (int r0 = 0; r0 < nv; r0 += 16) {
    const int r = r0 + ty;
    ta[ty][tx] = (r < nv && a0 + tx < ncv) ? Y[(size_t)r * ncv + a0 + tx] : 0.0;
    tb[ty][tx] = (r < nv && b0 + tx < ncv) ? Y[(size_t)r * ncv + b0 + tx] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += ta[k][ty] * tb[k][tx];
    __syncthreads();
  }
  if (a0 + ty < ncv && b0 + tx < ncv) D[(size_t)(a0 + ty) * ncv + b0 + tx] = acc;
}

// Z[v][c] = sum_p S^T[v][p] Y[p][c]  (one block per vertex row)
__global__ void __launch_bounds__(256) k_spmm_Z(int nv, int ncv, const long long* __restrict__ STp,
                                                const int* __restrict__ STj,
                                                const double* __restrict__ STx,
                                                const double* __restrict__ Y, double* __restrict__ Z) {
  const int v = blockIdx.x;
  if (v >= nv) return;
  for (int c = threadIdx.x; c < ncv; c += blockDim.x) {
    double acc = 0.0;
    for (long long p = STp[v]; p < STp[v + 1]; ++p) acc += STx[p] * Y[(size_t)STj[p] * ncv + c];
    Z[(size_t)v * ncv + c] = acc;
  }
}

constexpr int kNB = 32;

// Step 1 of block k: invert the diagonal block (partial pivoting inside the
// block) into P, and save the old column block of C into colbuf (m x nb).
__global__ void __launch_bounds__(256) k_gj_diag(int m, int k0, int kb, double* __restrict__ C,
                                                 double* __restrict__ P, double* __restrict__ colbuf,
                                                 int* __restrict__ err) {
  __shared__ double A[kNB][2 * kNB + 1];
  __shared__ int piv;
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * 2 * kNB; e += blockDim.x) {
    const int i = e / (2 * kNB), j = e % (2 * kNB);
    A[i][j] = (j < kb) ? C[(size_t)(k0 + i) * m + k0 + j] : ((j - kNB == i) ? 1.0 : 0.0);
  }
  for (size_t e = tid; e < (size_t)m * kb; e += blockDim.x) {
    const int i = (int)(e / kb), j = (int)(e % kb);
    colbuf[(size_t)i * kNB + j] = C[(size_t)i * m + k0 + j];
  }
  __syncthreads();
  for (int p = 0; p < kb; ++p) {
    if (tid == 0) {
      int best = p;
      double bv = fabs(A[p][p]);
      for (int i = p + 1; i < kb; ++i)
        if (fabs(A[i][p]) > bv) {
          bv = fabs(A[i][p]);
          best = i;
        }
      piv = best;
      if (!(bv > 0.0) || !isfinite(bv)) err[0] = 2;
    }
    __syncthreads();
    const int b = piv;
    if (b != p)
      for (int j = tid; j < 2 * kNB; j += blockDim.x) {
        double t = A[p][j];
        A[p][j] = A[b][j];
        A[b][j] = t;
      }
    __syncthreads();
    const double inv = 1.0 / A[p][p];
    __syncthreads();
    for (int j = tid; j < 2 * kNB; j += blockDim.x) A[p][j] *= inv;
    __syncthreads();
    for (int e = tid; e < kb * 2 * kNB; e += blockDim.x) {
      const int i = e / (2 * kNB), j = e % (2 * kNB);
      if (i != p && j != p) A[i][j] -= A[i][p] * A[p][j];
    }
    __syncthreads();
    // column p is read by the sweep above and only cleared afterwards
    for (int i = tid; i < kb; i += blockDim.x)
      if (i != p) A[i][p] = 0.0;
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += blockDim.x) {
    const int i = e / kb, j = e % kb;
    P[i * kNB + j] = A[i][kNB + j];
  }
}

// Step 2: row block k of C <- P * (row block k), columns outside the block.
__global__ void __launch_bounds__(256) k_gj_row(int m, int k0, int kb, double* __restrict__ C,
                                                const double* __restrict__ P) {
  __shared__ double Ps[kNB][kNB + 1];
  __shared__ double R[kNB][65];
  const int tid = threadIdx.x;
  const int j0 = blockIdx.x * 64;
  for (int e = tid; e < kb * kb; e += blockDim.x) Ps[e / kb][e % kb] = P[(e / kb) * kNB + e % kb];
  for (int e = tid; e < kb * 64; e += blockDim.x) {
    const int i = e / 64, j = j0 + e % 64;
    R[i][e % 64] = (j < m) ? C[(size_t)(k0 + i) * m + j] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < kb * 64; e += blockDim.x) {
    const int i = e / 64, jj = e % 64, j = j0 + jj;
    if (j >= m || (j >= k0 && j < k0 + kb)) continue;
    double acc = 0.0;
    for (int l = 0; l < kb; ++l) acc += Ps[i][l] * R[l][jj];
    C[(size_t)(k0 + i) * m + j] = acc;
  }
}

// Step 3: every other row: C_ij -= colbuf_i . C_kj (j outside block k);
// C_ik = -colbuf_i P; diagonal block <- P.
__global__ void __launch_bounds__(256) k_gj_update(int m, int k0, int kb, double* __restrict__ C,
                                                   const double* __restrict__ P,
                                                   const double* __restrict__ colbuf) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= m) return;
  const bool jin = (j >= k0 && j < k0 + kb);
  if (i >= k0 && i < k0 + kb) {
    if (jin) C[(size_t)i * m + j] = P[(i - k0) * kNB + (j - k0)];
    return;
  }
  const double* cb = colbuf + (size_t)i * kNB;
  double acc = 0.0;
  if (jin) {
    for (int l = 0; l < kb; ++l) acc -= cb[l] * P[l * kNB + (j - k0)];
    C[(size_t)i * m + j] = acc;
  } else {
    for (int l = 0; l < kb; ++l) acc += cb[l] * C[(size_t)(k0 + l) * m + j];
    C[(size_t)i * m + j] -= acc;
  }
}

void launch_fill_zero(hipStream_t st, size_t n, double* a) {
  if (n == 0) return;
  k_fill_zero<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a);
}

void launch_delassus(hipStream_t st, int nv, int ncv, const int* cv, const long long* STp,
                     const int* STj, const double* STx, double* Y, double* D, double* Z) {
  if (ncv == 0) return;
  launch_fill_zero(st, (size_t)nv * ncv, Y);
  k_fill_Y<<<ncv, 256, 0, st>>>(ncv, cv, STp, STj, STx, Y);
  dim3 g((ncv + 15) / 16, (ncv + 15) / 16);
  k_syrk<<<g, 256, 0, st>>>(nv, ncv, Y, D);
  k_spmm_Z<<<nv, 256, 0, st>>>(nv, ncv, STp, STj, STx, Y, Z);
}

void launch_gauss_jordan(hipStream_t st, int m, double* C, double* P, double* colbuf, int* err) {
  for (int k0 = 0; k0 < m; k0 += kNB) {
    const int kb = (m - k0 < kNB) ? (m - k0) : kNB;
    k_gj_diag<<<1, 256, 0, st>>>(m, k0, kb, C, P, colbuf, err);
    k_gj_row<<<(m + 63) / 64, 256, 0, st>>>(m, k0, kb, C, P);
    dim3 g((m + 255) / 256, m);
    k_gj_update<<<g, 256, 0, st>>>(m, k0, kb, C, P, colbuf);
  }
}

}  // namespace adj
