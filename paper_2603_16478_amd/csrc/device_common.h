// Device helpers shared by the HIP kernels of the adjoint library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace adj {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over groups of `width` consecutive lanes (width a power of two <= 64).
template <int width>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = width / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// a += B x for one 3x3 block p of the block-sparse Acal^T.  With FP32
// block values (mixed precision) the diagonal blocks are read from the FP64
// values instead: vertex-obstacle contacts and bindings put their stiffness
// (up to ~1/eps^2 times the elastic scale) on the diagonal blocks only, and
// FP32 rounding of those terms would make the inner solves diverge from the
// FP64 refinement residual; off-diagonal blocks are purely elastic.
template <class MT>
__device__ __forceinline__ void block_madd(const MT* __restrict__ val, const double* __restrict__ val64, size_t p,
                                           bool diag, double x0, double x1, double x2, double& a0, double& a1,
                                           double& a2, long long soa = 0) {
  // entry k of block p: val[9 p + k] (soa = 0), or val[k soa + p] (the
  // entry-major copy, soa = number of blocks: each entry's loads coalesce)
  const size_t base = soa ? p : 9 * p, ks = soa ? (size_t)soa : 1;
  if constexpr (sizeof(MT) == 4) {
    if (diag) {
      const double* b = val64 + base;
      a0 += b[0] * x0 + b[ks] * x1 + b[2 * ks] * x2;
      a1 += b[3 * ks] * x0 + b[4 * ks] * x1 + b[5 * ks] * x2;
      a2 += b[6 * ks] * x0 + b[7 * ks] * x1 + b[8 * ks] * x2;
      return;
    }
  }
  const MT* b = val + base;
  a0 += (double)b[0] * x0 + (double)b[ks] * x1 + (double)b[2 * ks] * x2;
  a1 += (double)b[3 * ks] * x0 + (double)b[4 * ks] * x1 + (double)b[5 * ks] * x2;
  a2 += (double)b[6 * ks] * x0 + (double)b[7 * ks] * x1 + (double)b[8 * ks] * x2;
}

// Block-wide sum for blockDim.x <= 1024; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds /* >= 16 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + kWave - 1) / kWave;
    for (int i = 0; i < nw; ++i) r += lds[i];
  }
  __syncthreads();
  return r;
}

// Partial dot products of one CSR row with a vector of 3-vectors:
// a_k += sum_p val[p] * x[3 col[p] + k] over the entries p = b + t,
// b + t + STEP, ... below e (t: this thread's index among the STEP threads
// sharing the row).  U entries per thread are loaded before any is used, so
// U index loads and then 3U dependent gathers are in flight per pass instead
// of one; masked slots read x[0..2] (in bounds for any non-empty x) with a
// zero weight.
template <int STEP, int U, class MT>
__device__ __forceinline__ void row_dot3(long long b, long long e, int t, const int* __restrict__ col,
                                         const MT* __restrict__ val, const double* __restrict__ x, double& a0,
                                         double& a1, double& a2) {
  for (long long p = b + t; p < e; p += (long long)STEP * U) {
    double v[U];
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long q = p + (long long)u * STEP;
      v[u] = 0.0;
      c[u] = 0;
      if (q < e) {
        v[u] = (double)val[q];
        c[u] = col[q];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double* xp = x + 3LL * c[u];
      a0 = fma(v[u], xp[0], a0);
      a1 = fma(v[u], xp[1], a1);
      a2 = fma(v[u], xp[2], a2);
    }
  }
}

// Woodbury gather rows: t_r = sum_k X[r][k] g[k], k < m (g in LDS), for
// rows r = r0 + w, r0 + w + 4, ... below r1, row r at Xr + (r - r0) ld; four
// X loads per lane in flight per pass.
template <class MT>
__device__ __forceinline__ void wb_gather_rows(int r0, int r1, int m, const MT* __restrict__ Xr, long long ld,
                                               const double* __restrict__ g, double* __restrict__ t) {
  const int lane = threadIdx.x & 63;
  for (int r = r0 + (threadIdx.x >> 6); r < r1; r += 4) {
    const MT* xr = Xr + (size_t)(r - r0) * ld;
    double acc = 0.0;
    for (int k0 = lane; k0 < m; k0 += 4 * 64) {
      double x[4];
      int kk[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 64 * q;
        kk[q] = k < m ? k : 0;
        x[q] = k < m ? (double)xr[k] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc = fma(x[q], g[kk[q]], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) t[r] = acc;
  }
}

// Woodbury correction rows: y_v = u_v - h2 sum_k Z[v][k] tp[k] (tp: [ncv][3]
// in LDS) for rows v = v0 + w, v0 + w + 4, ... below v1 (w: wavefront of a
// 256-thread block), Z row v at Zr + (v - v0) ncv; four Z loads per lane in
// flight per pass.
template <class MT>
__device__ __forceinline__ void wb_rows(int v0, int v1, int ncv, const MT* __restrict__ Zr,
                                        const double* __restrict__ tp, double h2, const double* __restrict__ u,
                                        double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  for (int v = v0 + (threadIdx.x >> 6); v < v1; v += 4) {
    const MT* zr = Zr + (size_t)(v - v0) * ncv;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k0 = lane; k0 < ncv; k0 += 4 * 64) {
      double z[4];
      int kk[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 64 * q;
        kk[q] = k < ncv ? k : 0;
        z[q] = k < ncv ? (double)zr[k] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a0 = fma(z[q], tp[3 * kk[q]], a0);
        a1 = fma(z[q], tp[3 * kk[q] + 1], a1);
        a2 = fma(z[q], tp[3 * kk[q] + 2], a2);
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
      y[3 * v] = u[3 * v] - h2 * a0;
      y[3 * v + 1] = u[3 * v + 1] - h2 * a1;
      y[3 * v + 2] = u[3 * v + 2] - h2 * a2;
    }
  }
}

// res[i] = sum_b P[b * ld + i] for i < cnt (cnt <= 256), fixed order; all
// 256 threads of the block take part; tmp: 256 doubles of LDS.
__device__ __forceinline__ void sum_partials(const double* __restrict__ P, int nb, int ld, int cnt,
                                             double* __restrict__ res, double* __restrict__ tmp) {
  int G = 1;
  while (2 * G * cnt <= 256) G *= 2;  // threads per entry (power of two)
  const int t = threadIdx.x, i = t / G, g = t % G;
  double a = 0.0;
  if (i < cnt)
    for (int b = g; b < nb; b += G) a += P[(size_t)b * ld + i];
  tmp[t] = a;
  __syncthreads();
  for (int h = G / 2; h > 0; h >>= 1) {
    if (g < h && i < cnt) tmp[t] += tmp[t + h];
    __syncthreads();
  }
  if (g == 0 && i < cnt) res[i] = tmp[t];
  __syncthreads();
}

}  // namespace adj
