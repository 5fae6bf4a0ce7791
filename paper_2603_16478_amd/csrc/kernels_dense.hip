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

// Gauss-Jordan exchange step for the diagonal block k (rows/cols k0..k0+32)
// of the padded mp x mp matrix (mp a multiple of 32, padding = identity):
//   P = A_kk^{-1};  B_kk = P;  B_kj = P A_kj;  B_ik = -A_ik P;
//   B_ij = A_ij - A_ik P A_kj
// from buffer A into buffer B (ping-pong, so no block reads what another
// block writes).  After all blocks the last output buffer is the inverse.
//
// One block of 256 threads per 32x32 output tile (I, J).  Wavefront 0
// inverts A_kk in registers: lane c holds column c of [A_kk | I]; pivot
// rows are found from uniform copies of the pivot column (readlane), so
// the 32 elimination steps need no LDS round trips.

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_readlane(lo, lane);
  hi = __builtin_amdgcn_readlane(hi, lane);
  return __hiloint2double(hi, lo);
}

// One Gauss-Jordan pivot step (compile-time pivot index P, so every array
// index below is a constant and the columns stay in registers).
template <int P>
__device__ __forceinline__ void gj_pivot(double (&col)[kNB], bool& bad) {
  double f[kNB];
#pragma unroll
  for (int i = 0; i < kNB; ++i) f[i] = readlane_d(col[i], P);
  int idx = P;
  double best = fabs(f[P]);
#pragma unroll
  for (int i = P + 1; i < kNB; ++i)
    if (fabs(f[i]) > best) {
      best = fabs(f[i]);
      idx = i;
    }
  if (!(best > 0.0) || !isfinite(best)) bad = true;
  const double cp = col[P], fp = f[P];
  double cs = cp, fs = fp;
#pragma unroll
  for (int i = P + 1; i < kNB; ++i)
    if (i == idx) {
      cs = col[i];
      fs = f[i];
      col[i] = cp;
      f[i] = fp;
    }
  const double inv = 1.0 / fs;
  col[P] = cs * inv;
#pragma unroll
  for (int i = 0; i < kNB; ++i)
    if (i != P) col[i] -= f[i] * col[P];
  if constexpr (P + 1 < kNB) gj_pivot<P + 1>(col, bad);
}

__device__ __forceinline__ void invert32_wave(const double* __restrict__ Akk, int mp,
                                              double (*Ps)[kNB + 1], int* __restrict__ err) {
  const int lane = threadIdx.x & 63;
  double col[kNB];
#pragma unroll
  for (int i = 0; i < kNB; ++i)
    col[i] = (lane < kNB) ? Akk[(size_t)i * mp + lane] : ((lane - kNB == i) ? 1.0 : 0.0);
  bool bad = false;
  gj_pivot<0>(col, bad);
  if (lane == 0 && bad) err[0] = 2;
  if (lane >= kNB) {
#pragma unroll
    for (int i = 0; i < kNB; ++i) Ps[i][lane - kNB] = col[i];
  }
}

__global__ void __launch_bounds__(256) k_gj_step(int mp, int k0, const double* __restrict__ A,
                                                 double* __restrict__ B, int* __restrict__ err) {
  __shared__ double Ps[kNB][kNB + 1];   // P = A_kk^{-1}
  __shared__ double Cs[kNB][kNB + 1];   // A_{I,k}
  __shared__ double Rs[kNB][kNB + 1];   // A_{k,J}
  __shared__ double Ws[kNB][kNB + 1];   // W = A_{I,k} P
  const int tid = threadIdx.x;
  const int I0 = blockIdx.y * kNB, J0 = blockIdx.x * kNB;
  const bool Ik = (I0 == k0), Jk = (J0 == k0);
  if (tid < 64) invert32_wave(A + (size_t)k0 * mp + k0, mp, Ps, err);
  for (int e = tid; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    Cs[r][c] = A[(size_t)(I0 + r) * mp + k0 + c];
    Rs[r][c] = A[(size_t)(k0 + r) * mp + J0 + c];
  }
  __syncthreads();
  if (!Ik) {
    for (int e = tid; e < kNB * kNB; e += 256) {
      const int r = e / kNB, c = e % kNB;
      double acc = 0.0;
#pragma unroll 8
      for (int l = 0; l < kNB; ++l) acc += Cs[r][l] * Ps[l][c];
      Ws[r][c] = acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    double v;
    if (Ik && Jk) {
      v = Ps[r][c];
    } else if (Ik) {
      double acc = 0.0;
#pragma unroll 8
      for (int l = 0; l < kNB; ++l) acc += Ps[r][l] * Rs[l][c];
      v = acc;
    } else if (Jk) {
      v = -Ws[r][c];
    } else {
      double acc = 0.0;
#pragma unroll 8
      for (int l = 0; l < kNB; ++l) acc += Ws[r][l] * Rs[l][c];
      v = A[(size_t)(I0 + r) * mp + J0 + c] - acc;
    }
    B[(size_t)(I0 + r) * mp + J0 + c] = v;
  }
}

// identity padding of rows/cols m..mp-1 of a row-major mp x mp matrix
__global__ void k_pad_identity(int m, int mp, double* __restrict__ C) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= mp || i >= mp) return;
  if (i < m && j < m) return;
  C[(size_t)i * mp + j] = (i == j) ? 1.0 : 0.0;
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

// Inverse of the m x m capacitance held in the top-left of the row-major
// mp x mp buffer C0 (mp = 32 * ceil(m/32)); returns the buffer (C0 or C1)
// that holds the inverse.
double* launch_gauss_jordan(hipStream_t st, int m, int mp, double* C0, double* C1, int* err) {
  if (mp > m) {
    dim3 gpad((mp + 255) / 256, mp);
    k_pad_identity<<<gpad, 256, 0, st>>>(m, mp, C0);
  }
  double* A = C0;
  double* B = C1;
  const int nb = mp / kNB;
  for (int k = 0; k < nb; ++k) {
    dim3 g(nb, nb);
    k_gj_step<<<g, 256, 0, st>>>(mp, k * kNB, A, B, err);
    double* t = A;
    A = B;
    B = t;
  }
  return A;
}

}  // namespace adj
