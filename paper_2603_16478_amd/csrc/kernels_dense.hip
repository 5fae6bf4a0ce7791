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

#include <algorithm>

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

// D = Y^T Y on the matrix cores.  One 256-thread block per 64x64 tile of
// the lower triangle of D (tile row >= tile column) and per K-slice of the
// n_v rows of Y; each wavefront owns a 32x32 quarter of the tile as 2x2
// MFMA 16x16 accumulators.  16-row panels of Y are staged through LDS.
// FP64 products and sums (v_mfma_f64_16x16x4f64).  D is kept in FP64 in
// both precision modes: for stiff contacts the Woodbury correction cancels
// A^{-1} r almost exactly, and FP32 rounding of D would be amplified by the
// contact-to-elastic stiffness ratio.
// 16x16x4 operand layout (lane l = 16 kq + i, i < 16, kq < 4): the A operand
// of lane l is A[i][kq], the B operand B[kq][i]; accumulator value e (0..3)
// of lane l is C[r][i] with r = kq + 4 e (checked on the device; the f32
// variant of the instruction uses r = 4 kq + e instead).
// With ks > 1 K-slices the block writes its partial tile to P[slice], and
// k_syrk_reduce sums the slices in fixed order; with one slice it writes D.
// Both triangles of D are written (D is symmetric).
typedef double d4 __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<double> {
  using V = d4;
  static __device__ __forceinline__ V step(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int e) { return kq + 4 * e; }
};

constexpr int kSyT = 64;  // output tile edge
constexpr int kSyK = 16;  // rows of Y per LDS panel

// Panel occupancy of Y: bit p of column group g (kSyT consecutive contact
// vertices) is set when a vertex of the group has a nonzero of S in rows
// [kSyK p, kSyK (p + 1)), i.e. on its elimination-tree path.  A tile of D
// only needs the panels where both of its column groups have entries
// (integer OR: the bitmap does not depend on the order of the updates).
__global__ void k_y_panels(int ncv, const int* __restrict__ cv, const long long* __restrict__ STp,
                           const int* __restrict__ STj, int npw, unsigned* __restrict__ bm) {
  const int c = blockIdx.x;
  if (c >= ncv) return;
  unsigned* w = bm + (size_t)(c / kSyT) * npw;
  for (long long p = STp[cv[c]] + threadIdx.x; p < STp[cv[c] + 1]; p += blockDim.x) {
    const int pnl = STj[p] / kSyK;
    atomicOr(&w[pnl >> 5], 1u << (pnl & 31));
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_syrk_mfma(int nv, int ncv, int rows_per_slice,
                                                   const double* __restrict__ Y, double* __restrict__ out,
                                                   const unsigned* __restrict__ bm, int npw) {
  __shared__ T As[kSyK][kSyT + 1];
  __shared__ T Bs[kSyK][kSyT + 1];
  // blockIdx.x enumerates lower-triangle tiles: x = ti (ti + 1) / 2 + tj, tj <= ti
  const int x = blockIdx.x;
  int ti = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
  while (ti * (ti + 1) / 2 > x) --ti;
  const int tj = x - ti * (ti + 1) / 2;
  const int a0 = ti * kSyT, b0 = tj * kSyT;
  const int r_begin = blockIdx.y * rows_per_slice;
  const int r_end = min(nv, r_begin + rows_per_slice);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wa = 32 * (w >> 1), wb = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
  using V = typename MfmaAcc<T>::V;
  V acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = V{0, 0, 0, 0};
  const unsigned* bi = bm ? bm + (size_t)ti * npw : nullptr;
  const unsigned* bj = bm ? bm + (size_t)tj * npw : nullptr;
  for (int r0 = r_begin; r0 < r_end; r0 += kSyK) {
    if (bm) {
      const int pnl = r0 / kSyK;
      if (!(((bi[pnl >> 5] & bj[pnl >> 5]) >> (pnl & 31)) & 1u)) continue;  // a zero panel of Y
    }
#pragma unroll
    for (int e = 0; e < (kSyK * kSyT) / 256; ++e) {
      const int idx = tid + 256 * e;
      const int kr = idx / kSyT, c = idx % kSyT;
      const int r = r0 + kr;
      const bool rin = r < r_end;
      As[kr][c] = (rin && a0 + c < ncv) ? (T)Y[(size_t)r * ncv + a0 + c] : (T)0;
      Bs[kr][c] = (rin && b0 + c < ncv) ? (T)Y[(size_t)r * ncv + b0 + c] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < kSyK; k4 += 4) {
      T av[2], bv[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        av[p] = As[k4 + lk][wa + 16 * p + li];
        bv[p] = Bs[k4 + lk][wb + 16 * p + li];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = MfmaAcc<T>::step(av[p], bv[q], acc[p][q]);
    }
    __syncthreads();
  }
  double* dst = out + (size_t)blockIdx.y * ncv * ncv;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = a0 + wa + 16 * p + MfmaAcc<T>::row(lk, e);
        const int j = b0 + wb + 16 * q + li;
        if (i < ncv && j < ncv) {
          const double v = (double)acc[p][q][e];
          dst[(size_t)i * ncv + j] = v;
          if (ti != tj) dst[(size_t)j * ncv + i] = v;
        }
      }
}

// D[i][j] = sum over slices of P[s][i][j] (fixed order), all i, j
__global__ void k_syrk_reduce(int ncv, int ks, const double* __restrict__ P, double* __restrict__ D) {
  const size_t n = (size_t)ncv * ncv;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int s = 0; s < ks; ++s) a += P[(size_t)s * n + i];
  D[i] = a;
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

// Capacitance inverse by block Gauss-Jordan elimination with 32x32 pivot
// blocks (partial pivoting inside each block), from buffer A into buffer B
// per block step (ping-pong, so no block reads what another block writes).
// After the last step the last output buffer holds the inverse.

// Inverse of the 32x32 pivot block by one wavefront, row per lane: lane r
// (r < 32) holds row r of A_kk, lane 32 + r row r of the identity.  Step k
// picks the unused row with the largest |A[r][k]| (partial pivoting),
// broadcasts that row through LDS and eliminates column k from every other
// row.  Rows are never swapped: with p_k the row chosen at step k, the
// eliminated A part is a permutation and row k of the inverse is row p_k of
// the transformed identity.  The argmax runs on DPP lane moves inside each
// 16-lane row (quad xor 1, quad xor 2, half-row mirror, row mirror) and one
// readlane per row, so the step's critical path stays in the vector ALU.
// The column index is a template parameter, so register indices are static.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within each 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within each 16 lanes

// 1 / a to full double precision: hardware reciprocal estimate refined by
// two Newton steps (each doubles the correct bits).
__device__ __forceinline__ double rcp_newton(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  e = fma(-a, r, 1.0);
  return fma(r, e, r);
}

// 32-bit max over the 16 lanes of each DPP row
template <int CTRL>
__device__ __forceinline__ unsigned max_dpp(unsigned v) {
  return max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false));
}

template <int K>
__device__ __forceinline__ void gj_rows_step(double (&x)[kNB], bool& used, int& step_of_row, bool& bad,
                                             double* __restrict__ prow) {
  const int lane = threadIdx.x & 63, r = lane & 31;
  // pivot column value of this lane's row (the A part lives in lanes < 32;
  // the identity lanes need it only for the update, so the shuffle runs
  // beside the search instead of before it)
  const double own = x[K];
  const double ak = __shfl(own, r, 64);
  // pivot choice on a 32-bit key: |a_rk| rounded to float with its low 5
  // bits replaced by 31 - r (ties within ~2^-18 relative go to the lower
  // row), used rows 0, unused rows at least 32; one DPP max per level.  Only
  // the A lanes' keys are read.
  const unsigned mag = __float_as_uint((float)fabs(own)) & ~31u;
  unsigned key = (used || lane >= 32) ? 0u : (max(mag, 32u) | (unsigned)(31 - r));
  key = max_dpp<kDppXor1>(key);
  key = max_dpp<kDppXor2>(key);
  key = max_dpp<kDppHalfMirror>(key);
  key = max_dpp<kDppMirror>(key);
  const unsigned kb = max((unsigned)__builtin_amdgcn_readlane((int)key, 0),
                          (unsigned)__builtin_amdgcn_readlane((int)key, 16));
  const int p = 31 - (int)(kb & 31u);
  const double apk = readlane_d(ak, p);
  if (!(fabs(apk) > 0.0) || !isfinite(apk)) bad = true;
  const double inv = rcp_newton(apk);
  // broadcast the pivot row: A part to prow[0..31], identity part to prow[32..63]
  const bool piv = (r == p);
  if (piv) {
#pragma unroll
    for (int c = 0; c < kNB; ++c) prow[(lane & 32) + c] = x[c];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const double* pr = prow + (lane & 32);
  // pivot row: x <- x / a_pk (= x + (1/a_pk - 1) x, its own row); others:
  // x <- x - (a_rk / a_pk) pivot row.  One FMA per entry, no divergence.
  const double g = piv ? inv - 1.0 : -ak * inv;
#pragma unroll
  for (int c = 0; c < kNB; ++c) x[c] = fma(g, pr[c], x[c]);
  if (piv) {
    used = true;
    step_of_row = K;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if constexpr (K + 1 < kNB) gj_rows_step<K + 1>(x, used, step_of_row, bad, prow);
}

// P = A_kk^{-1} into Ps (wavefront 0 of the block; prow: 64 doubles of LDS)
__device__ __forceinline__ void invert32_rows(const double* __restrict__ Akk, int mp, double (*Ps)[kNB + 1],
                                              double* __restrict__ prow, int* __restrict__ err) {
  const int lane = threadIdx.x & 63, r = lane & 31;
  double x[kNB];
  if (lane < kNB) {
#pragma unroll
    for (int c = 0; c < kNB; ++c) x[c] = Akk[(size_t)r * mp + c];
  } else {
#pragma unroll
    for (int c = 0; c < kNB; ++c) x[c] = (c == r) ? 1.0 : 0.0;
  }
  bool used = false, bad = false;
  int step_of_row = 0;
  gj_rows_step<0>(x, used, step_of_row, bad, prow);
  if (lane == 0 && bad) err[0] = 2;
  if (lane >= kNB) {
#pragma unroll
    for (int c = 0; c < kNB; ++c) Ps[step_of_row][c] = x[c];
  }
}

// Gauss-Jordan block step on the matrix cores.  With the 32 pivot rows and
// columns at k0 and P = A_kk^{-1}, every output entry is one formula:
//   B = Ahat - What Rhat,
//   Ahat = A with the pivot rows and pivot columns set to 0,
//   What_i = A_ik P (row i outside the pivot rows),   -P_i (pivot row i),
//   Rhat_j = A_kj (column j outside the pivot columns), e_j (pivot column j),
// which gives P A_kj in the pivot rows, -A_ik P in the pivot columns, P in
// the pivot block and A_ij - A_ik P A_kj elsewhere.
// One 256-thread block per 64x64 output tile (mp a multiple of 64), with P
// inverted beforehand (the lookahead below); the two products (What for the
// tile rows, then the update) are 16x16x4 FP64 MFMAs with 2x2 (What) and 2x2
// (update) accumulator tiles per wave.
constexpr int kGT = 64;

// 42 KB, so three blocks fit in one CU's LDS; the step kernel is held to
// 168 registers (three waves per SIMD) with the A tile loaded after the
// panels are staged.
struct GjShared {
  double Ps[kNB][kNB + 1];   // P = A_kk^{-1}
  double Cs[kGT][kNB + 1];   // A_{I,k} (tile rows, pivot columns), then -What
  double Rs[kNB][kGT + 1];   // Rhat (pivot rows, tile columns)
  double prow[2 * kNB];      // pivot row broadcast of the block inversion
};

// One 64x64 output tile (I0, J0) of the block step at pivot k0.  Offsets
// into the matrix are 32-bit (mp^2 < 2^32 for any capacitance size the
// library accepts), which halves the address registers of the hoisted loads.  P
// is read from Pg (32 x 32, row-major), inverted once per step beforehand.
__device__ __forceinline__ void gj_tile(int mp, int k0, int I0, int J0, const double* __restrict__ A,
                                        double* __restrict__ B, GjShared& sh, const double* __restrict__ Pg) {
  auto& Ps = sh.Ps;
  auto& Cs = sh.Cs;
  auto& Rs = sh.Rs;
  auto& Ws = sh.Cs;  // wave w reads and then overwrites only rows 16 w .. 16 w + 15
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // output sub-tiles of this wave: rows wr + 16 p, cols wc + 16 q (p, q < 2)
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  for (int e = tid; e < kNB * kNB; e += 256) Ps[e / kNB][e % kNB] = Pg[e];
  for (int e = tid; e < kGT * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    Cs[r][c] = A[(unsigned)((I0 + r) * mp + k0 + c)];
  }
  for (int e = tid; e < kNB * kGT; e += 256) {
    const int r = e / kGT, c = e % kGT;
    const int j = J0 + c;
    Rs[r][c] = (j >= k0 && j < k0 + kNB) ? ((j - k0 == r) ? 1.0 : 0.0) : A[(unsigned)((k0 + r) * mp + j)];
  }
  __syncthreads();
  // accumulators start at Ahat (f64 MFMA result layout: row lk + 4 e, col
  // li); loaded after the panels are staged, so these loads overlap the
  // -What products and do not add to the staging's live registers
  d4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = I0 + wr + 16 * p + lk + 4 * e;
        const int j = J0 + wc + 16 * q + li;
        const bool zero = (i >= k0 && i < k0 + kNB) || (j >= k0 && j < k0 + kNB);
        acc[p][q][e] = zero ? 0.0 : A[(unsigned)(i * mp + j)];
      }
  // -What for the 64 tile rows: wave w computes rows 16 w .. 16 w + 15, both
  // 16-column halves of the 32 pivot columns.
  {
    d4 wacc[2];
    wacc[0] = d4{0, 0, 0, 0};
    wacc[1] = d4{0, 0, 0, 0};
#pragma unroll
    for (int k4 = 0; k4 < kNB; k4 += 4) {
      const double a = Cs[16 * w + li][k4 + lk];
#pragma unroll
      for (int q = 0; q < 2; ++q)
        wacc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ps[k4 + lk][16 * q + li], wacc[q], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * w + lk + 4 * e;
        const int c = 16 * q + li;
        const int i = I0 + r;
        Ws[r][c] = (i >= k0 && i < k0 + kNB) ? Ps[i - k0][c] : -wacc[q][e];
      }
  }
  __syncthreads();
  // update: acc += (-What) Rhat over the 32 pivot indices
#pragma unroll
  for (int k4 = 0; k4 < kNB; k4 += 4) {
    double av[2], bv[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) av[p] = Ws[wr + 16 * p + li][k4 + lk];
#pragma unroll
    for (int q = 0; q < 2; ++q) bv[q] = Rs[k4 + lk][wc + 16 * q + li];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = I0 + wr + 16 * p + lk + 4 * e;
        const int j = J0 + wc + 16 * q + li;
        B[(unsigned)(i * mp + j)] = acc[p][q][e];
      }
}

// Batched block steps with a one-step lookahead on the pivot chain.
// kb_gj_pivot: one wavefront per listed scene inverts the first pivot block
// (k0 = 0) into P slot s.  kb_gj_step_mfma, at pivot k0 = 32 k: blocks
// [0, npiv) are next-pivot tasks, one per scene that has a step k + 1; from
// the step's input A they form that step's pivot block,
//   A_k1k1 - (A_k1k0 P_k) A_k0k1   (k1 = k0 + 32),
// which is exactly the block the tiles of step k write there, invert it and
// store it in the other P slot.  The remaining blocks are the output tiles
// {scene, I tile, J tile, -} of step k, reading P_k.  So the serial pivot
// inversion of step k + 1 runs beside the tiles of step k instead of after
// them; the scene's matrix is at A + xoff[s] (B + xoff[s]) with row length
// mps[s], its P at P + 1024 s.
__device__ __forceinline__ void gj_next_pivot(int mp, int k0, const double* __restrict__ A,
                                              const double* __restrict__ Pc, double* __restrict__ Pn,
                                              int* __restrict__ err, GjShared& sh) {
  const int k1 = k0 + kNB, tid = threadIdx.x;
  // Cs[0..31] = A_k1k0, Cs[32..63] = A_k1k1, Ps = P_k, Rs[.][0..31] = A_k0k1
  // and Rs[.][32..63] = A_k1k0 P_k
  for (int e = tid; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    sh.Cs[r][c] = A[(size_t)(k1 + r) * mp + k0 + c];
    sh.Cs[kNB + r][c] = A[(size_t)(k1 + r) * mp + k1 + c];
    sh.Ps[r][c] = Pc[e];
    sh.Rs[r][c] = A[(size_t)(k0 + r) * mp + k1 + c];
  }
  __syncthreads();
  // one 16 x 16 output tile per wavefront, FP64 MFMA (A operand row li,
  // k lk; B operand k lk, column li; result row lk + 4 e, column li)
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int R0 = 16 * (w >> 1), C0 = 16 * (w & 1);
  {
    d4 acc = d4{0, 0, 0, 0};
#pragma unroll
    for (int k4 = 0; k4 < kNB; k4 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sh.Cs[R0 + li][k4 + lk], sh.Ps[k4 + lk][C0 + li], acc, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) sh.Rs[R0 + lk + 4 * e][kNB + C0 + li] = acc[e];
  }
  __syncthreads();
  // A_k1k1 -= (A_k1k0 P_k) A_k0k1
  {
    d4 acc;
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] = sh.Cs[kNB + R0 + lk + 4 * e][C0 + li];
#pragma unroll
    for (int k4 = 0; k4 < kNB; k4 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-sh.Rs[R0 + li][kNB + k4 + lk], sh.Rs[k4 + lk][C0 + li], acc, 0, 0,
                                                 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) sh.Cs[kNB + R0 + lk + 4 * e][C0 + li] = acc[e];
  }
  __syncthreads();
  if (tid < 64) invert32_rows(&sh.Cs[kNB][0], kNB + 1, sh.Ps, sh.prow, err);
  __syncthreads();
  for (int e = tid; e < kNB * kNB; e += 256) Pn[e] = sh.Ps[e / kNB][e % kNB];
}

__global__ void __launch_bounds__(64) kb_gj_pivot(const int* __restrict__ scenes, const long long* __restrict__ xoff,
                                                  const int* __restrict__ mps, const double* __restrict__ A,
                                                  double* __restrict__ Pb, int* __restrict__ err) {
  __shared__ double Ps[kNB][kNB + 1];
  __shared__ double prow[2 * kNB];
  const int s = scenes[blockIdx.x];
  invert32_rows(A + xoff[s], mps[s], Ps, prow, err);
  __syncthreads();
  double* P = Pb + (size_t)s * kNB * kNB;
  for (int e = threadIdx.x; e < kNB * kNB; e += blockDim.x) P[e] = Ps[e / kNB][e % kNB];
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
kb_gj_step_mfma(const int* __restrict__ next_scenes, int npiv,
                                                       const int4* __restrict__ tiles, int k0,
                                                       const long long* __restrict__ xoff,
                                                       const int* __restrict__ mps, const double* __restrict__ A,
                                                       double* __restrict__ B, const double* __restrict__ Pcur,
                                                       double* __restrict__ Pnext, int* __restrict__ err) {
  __shared__ GjShared sh;
  if ((int)blockIdx.x < npiv) {
    const int s = next_scenes[blockIdx.x];
    const size_t po = (size_t)s * kNB * kNB;
    gj_next_pivot(mps[s], k0, A + xoff[s], Pcur + po, Pnext + po, err, sh);
    return;
  }
  const int4 e = tiles[blockIdx.x - npiv];
  const long long o = xoff[e.x];
  gj_tile(mps[e.x], k0, e.y * kGT, e.z * kGT, A + o, B + o, sh, Pcur + (size_t)e.x * kNB * kNB);
}

// Wide block Gauss-Jordan for large single capacitances (mp a multiple of
// 128): 128 pivot columns per step instead of 32, so the matrix is read and
// written mp/128 times instead of mp/32 times and every step is a rank-128
// update (16 flop per byte moved, above the chip's FP64 ridge) on the
// matrix cores.  The same B = Ahat - What Rhat step as above, with K the
// 128 pivot indices k0 .. k0 + 127 and P = A_KK^{-1}; per step three
// launches:
//   k_gjw_panel  What (mp x 128): A_{i,K} P for rows i outside K, -P_i in K;
//   k_gjw_tiles  the 128 x 128 output tiles of B; the tile that is the next
//                step's pivot block is also inverted (lookahead), so the
//                serial pivot chain runs beside the tiles.
// P = A_KK^{-1} of the first step comes from k_gjw_pivot.  The 128 x 128
// inversions take four Gauss-Jordan sub-steps on their 32 x 32 diagonal
// blocks in LDS (the same 32-block partial pivoting as the narrow kernels).
constexpr int kWB = 128;        // pivot block width
constexpr int kWL = kWB + 1;    // LDS row stride of the pivot block
constexpr int kWKC = 32;        // k-chunk of the staged panels

// In-place inverse of the 128 x 128 block M (LDS, row stride kWL) by one
// 256-thread block: four Gauss-Jordan sub-steps on its 32 x 32 diagonal
// blocks (P32 of each from invert32_rows, partial pivoting inside the
// sub-block); the sub-step's products run on the matrix cores, 16 x 16
// output tiles spread over the four wavefronts.  Ps (32 x 33) and prow (64)
// are LDS scratch.  Every sub-step, with O = the 96 indices outside it:
//   (a) W = M_{O,sb} P32, stored negated in place of M_{O,sb};
//   (b) M_{O,O} += (-W) M_{sb,O};
//   (c) M_{sb,O} = P32 M_{sb,O} (from the pivot rows as they were before);
//   (d) M_{sb,sb} = P32.
__device__ __forceinline__ void invert128_lds(double* __restrict__ M, double (*Ps)[kNB + 1], double* __restrict__ prow,
                                              int* __restrict__ err) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll 1
  for (int sb = 0; sb < kWB; sb += kNB) {
    if (tid < 64) invert32_rows(M + sb * kWL + sb, kWL, Ps, prow, err);
    __syncthreads();
    // first row (column) of outer 16-tile t: tiles never straddle the sub-block
    auto outer = [&](int t) { return 16 * t < sb ? 16 * t : 16 * t + kNB; };
    // (a): 6 x 2 tiles, three per wavefront
    d4 wa[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int t = 3 * w + u, r0 = outer(t >> 1), c0 = 16 * (t & 1);
      d4 acc = d4{0, 0, 0, 0};
#pragma unroll
      for (int k4 = 0; k4 < kNB; k4 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(M[(r0 + li) * kWL + sb + k4 + lk], Ps[k4 + lk][c0 + li], acc, 0,
                                                   0, 0);
      wa[u] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int t = 3 * w + u, r0 = outer(t >> 1), c0 = 16 * (t & 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) M[(r0 + lk + 4 * e) * kWL + sb + c0 + li] = -wa[u][e];
    }
    __syncthreads();
    // (b): 6 x 6 tiles, nine per wavefront, in place
#pragma unroll 1
    for (int u = 0; u < 9; ++u) {
      const int t = 9 * w + u, r0 = outer(t / 6), c0 = outer(t % 6);
      d4 acc;
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = M[(r0 + lk + 4 * e) * kWL + c0 + li];
#pragma unroll
      for (int k4 = 0; k4 < kNB; k4 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(M[(r0 + li) * kWL + sb + k4 + lk], M[(sb + k4 + lk) * kWL + c0 + li],
                                                   acc, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) M[(r0 + lk + 4 * e) * kWL + c0 + li] = acc[e];
    }
    // (c): 2 x 6 tiles, three per wavefront, held until (b) has read the pivot rows
    d4 ca[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int t = 3 * w + u, r0 = 16 * (t / 6), c0 = outer(t % 6);
      d4 acc = d4{0, 0, 0, 0};
#pragma unroll
      for (int k4 = 0; k4 < kNB; k4 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ps[r0 + li][k4 + lk], M[(sb + k4 + lk) * kWL + c0 + li], acc, 0, 0,
                                                   0);
      ca[u] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int t = 3 * w + u, r0 = 16 * (t / 6), c0 = outer(t % 6);
#pragma unroll
      for (int e = 0; e < 4; ++e) M[(sb + r0 + lk + 4 * e) * kWL + c0 + li] = ca[u][e];
    }
    for (int e = tid; e < kNB * kNB; e += 256) M[(sb + e / kNB) * kWL + sb + e % kNB] = Ps[e / kNB][e % kNB];
    __syncthreads();
  }
}

// The shared memory of one block of the wide steps: the staged panels of an
// output tile, or the 128 x 128 block being inverted.
union GjwShared {
  struct {
    double Ws[kWB][kWKC + 1];
    double Rs[kWKC][kWB + 1];
  } t;
  struct {
    double M[kWB * kWL];
    double Ps[kNB][kNB + 1];
    double prow[2 * kNB];
  } p;
};

__global__ void __launch_bounds__(256) k_gjw_pivot(int mp, int k0, const double* __restrict__ A,
                                                   double* __restrict__ Pout, int* __restrict__ err) {
  __shared__ GjwShared sh;
  double* M = sh.p.M;
  const int tid = threadIdx.x;
  for (int e = tid; e < kWB * kWB; e += 256) {
    const int r = e / kWB, c = e % kWB;
    M[r * kWL + c] = A[(size_t)(k0 + r) * mp + k0 + c];
  }
  __syncthreads();
  invert128_lds(M, sh.p.Ps, sh.p.prow, err);
  for (int e = tid; e < kWB * kWB; e += 256) Pout[e] = M[(e / kWB) * kWL + e % kWB];
}

__global__ void __launch_bounds__(256) k_gjw_panel(int mp, int k0, const double* __restrict__ A,
                                                   const double* __restrict__ P, double* __restrict__ W) {
  __shared__ double As[64][kWKC + 1];
  __shared__ double Bs[kWKC][kWB + 1];
  const int r0 = blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  if (r0 >= k0 && r0 < k0 + kWB) {  // pivot rows (64-row slabs never straddle K: k0 % 128 == 0)
    for (int e = tid; e < 64 * kWB; e += 256) {
      const int r = e / kWB, c = e % kWB;
      W[(size_t)(r0 + r) * kWB + c] = -P[(size_t)(r0 - k0 + r) * kWB + c];
    }
    return;
  }
  d4 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = d4{0, 0, 0, 0};
  for (int kc = 0; kc < kWB; kc += kWKC) {
    for (int e = tid; e < 64 * kWKC; e += 256) {
      const int r = e / kWKC, c = e % kWKC;
      As[r][c] = A[(size_t)(r0 + r) * mp + k0 + kc + c];
    }
    for (int e = tid; e < kWKC * kWB; e += 256) {
      const int r = e / kWB, c = e % kWB;
      Bs[r][c] = P[(size_t)(kc + r) * kWB + c];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < kWKC; k4 += 4) {
      const double a = As[16 * w + li][k4 + lk];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[k4 + lk][16 * q + li], acc[q], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) W[(size_t)(r0 + 16 * w + lk + 4 * e) * kWB + 16 * q + li] = acc[q][e];
}

// The panels of the next k-chunk are loaded into registers while the
// current chunk's products run, and stored to LDS after them (one LDS
// buffer, two blocks per CU).  The chunk-0 panels are requested before the
// output tile, so that their wait does not include the tile's loads.
constexpr int kWPre = kWB * kWKC / 256;  // panel entries per thread and chunk

// With k1 >= 0 (a step follows), the tile (k1, k1) is the next step's pivot
// block: block 0 computes it (blocks are dispatched in index order, so it
// starts first), then inverts it in LDS and writes P_{k+1} to Pnext while
// the other tiles of the step run.
__global__ void __launch_bounds__(256, 1) k_gjw_tiles(int mp, int k0, int k1, const double* __restrict__ A,
                                                      const double* __restrict__ W, double* __restrict__ B,
                                                      double* __restrict__ Pnext, int* __restrict__ err) {
  __shared__ GjwShared sh;
  auto& Ws = sh.t.Ws;
  auto& Rs = sh.t.Rs;
  const int nt = mp / kWB;
  int t = blockIdx.x;
  if (k1 >= 0) {
    const int diag = (k1 / kWB) * nt + k1 / kWB;
    t = (t == 0) ? diag : (t == diag ? 0 : t);
  }
  const int I0 = (t / nt) * kWB, J0 = (t % nt) * kWB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
  const bool rowsK = I0 == k0, colsK = J0 == k0;  // tiles are aligned with K
  double wpre[kWPre], rpre[kWPre];
  auto load_chunk = [&](int kc) {
#pragma unroll
    for (int u = 0; u < kWPre; ++u) {
      const int e = tid + 256 * u;
      const int rw = e / kWKC, cw = e % kWKC;
      wpre[u] = W[(size_t)(I0 + rw) * kWB + kc + cw];
      const int rr = e / kWB, cr = e % kWB;
      rpre[u] = colsK ? ((cr == kc + rr) ? 1.0 : 0.0) : A[(size_t)(k0 + kc + rr) * mp + J0 + cr];
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < kWPre; ++u) {
      const int e = tid + 256 * u;
      Ws[e / kWKC][e % kWKC] = wpre[u];
      Rs[e / kWB][e % kWB] = rpre[u];
    }
  };
  load_chunk(0);
  d4 acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = I0 + wr + 16 * p + lk + 4 * e, j = J0 + wc + 16 * q + li;
        acc[p][q][e] = (rowsK || colsK) ? 0.0 : A[(size_t)i * mp + j];
      }
  store_chunk();
  __syncthreads();
  for (int kc = 0; kc < kWB; kc += kWKC) {
    const bool more = kc + kWKC < kWB;
    if (more) load_chunk(kc + kWKC);
#pragma unroll
    for (int k4 = 0; k4 < kWKC; k4 += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) av[p] = -Ws[wr + 16 * p + li][k4 + lk];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = Rs[k4 + lk][wc + 16 * q + li];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      store_chunk();
      __syncthreads();
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        B[(size_t)(I0 + wr + 16 * p + lk + 4 * e) * mp + J0 + wc + 16 * q + li] = acc[p][q][e];
  if (k1 < 0 || I0 != k1 || J0 != k1) return;
  // the next pivot block: into LDS (the panels are no longer needed), invert
  double* M = sh.p.M;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) M[(wr + 16 * p + lk + 4 * e) * kWL + wc + 16 * q + li] = acc[p][q][e];
  __syncthreads();
  invert128_lds(M, sh.p.Ps, sh.p.prow, err);
  for (int e = tid; e < kWB * kWB; e += 256) Pnext[e] = M[(e / kWB) * kWL + e % kWB];
}

// identity padding of rows/cols m..mp-1 of a row-major mp x mp matrix
__global__ void k_pad_identity(int m, int mp, double* __restrict__ C) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= mp || i >= mp) return;
  if (i < m && j < m) return;
  C[(size_t)i * mp + j] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_fill_int(size_t n, int* __restrict__ a, int v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

void launch_fill_int(hipStream_t st, size_t n, int* a, int v) {
  if (n == 0) return;
  k_fill_int<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a, v);
}

void launch_fill_zero(hipStream_t st, size_t n, double* a) {
  if (n == 0) return;
  k_fill_zero<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a);
}

// K-slices for the Delassus product: enough blocks to cover the chip
// (~512) when the tile count is small, each slice at least 256 rows.
int delassus_slices(int nv, int ncv) {
  const int nt = (ncv + kSyT - 1) / kSyT;
  const int tiles = nt * (nt + 1) / 2;
  int ks = (512 + tiles - 1) / tiles;
  ks = std::min(ks, std::max(1, nv / 256));
  return std::max(ks, 1);
}

// Words of the panel bitmap per column group of Y
int y_panel_words(int nv) { return ((nv + kSyK - 1) / kSyK + 31) / 32; }

// bm: [ceil(ncv / 64)][y_panel_words(nv)] scratch for the panel occupancy
// (nullptr: every panel is multiplied).
void launch_delassus(hipStream_t st, int nv, int ncv, const int* cv, const long long* STp,
                     const int* STj, const double* STx, double* Y, double* D, double* Z, double* Pws,
                     unsigned* bm) {
  if (ncv == 0) return;
  launch_fill_zero(st, (size_t)nv * ncv, Y);
  k_fill_Y<<<ncv, 256, 0, st>>>(ncv, cv, STp, STj, STx, Y);
  const int nt = (ncv + kSyT - 1) / kSyT;
  const int npw = y_panel_words(nv);
  if (bm) {
    launch_fill_int(st, (size_t)nt * npw, (int*)bm, 0);
    k_y_panels<<<ncv, 256, 0, st>>>(ncv, cv, STp, STj, npw, bm);
  }
  const int ks = delassus_slices(nv, ncv);
  const int rows = (((nv + ks - 1) / ks) + kSyK - 1) / kSyK * kSyK;
  dim3 g(nt * (nt + 1) / 2, ks);
  double* out = (ks > 1) ? Pws : D;
  k_syrk_mfma<double><<<g, 256, 0, st>>>(nv, ncv, rows, Y, out, bm, npw);
  if (ks > 1) {
    const size_t n = (size_t)ncv * ncv;
    k_syrk_reduce<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(ncv, ks, Pws, D);
  }
  if (Z) k_spmm_Z<<<nv, 256, 0, st>>>(nv, ncv, STp, STj, STx, Y, Z);
}

// Inverse of the m x m capacitance held in the top-left of the row-major
// mp x mp buffer C0 (mp a multiple of 64): launch_gj_pad sets the padding
// rows and columns to the identity; then kb_gj_pivot inverts the first
// pivot block and launchb_gj_step runs block step k (k = 0 .. mp/32 - 1)
// from A into B, the two buffers swapping roles each step; after the last
// step the inverse is in C0 when mp/32 is even, else in C1.
void launch_gj_pad(hipStream_t st, int m, int mp, double* C0) {
  if (mp <= m) return;
  dim3 gpad((mp + 255) / 256, mp);
  k_pad_identity<<<gpad, 256, 0, st>>>(m, mp, C0);
}

void launchb_gj_pivot(hipStream_t st, int nscenes, const int* scenes, const long long* xoff, const int* mps,
                      const double* A, double* Pb, int* err) {
  if (!nscenes) return;
  kb_gj_pivot<<<nscenes, 64, 0, st>>>(scenes, xoff, mps, A, Pb, err);
}

void launchb_gj_step(hipStream_t st, int npiv, const int* next_scenes, int ntiles, const int4* tiles, int k0,
                     const long long* xoff, const int* mps, const double* A, double* B, const double* Pcur,
                     double* Pnext, int* err) {
  if (!ntiles) return;
  kb_gj_step_mfma<<<npiv + ntiles, 256, 0, st>>>(next_scenes, npiv, tiles, k0, xoff, mps, A, B, Pcur, Pnext, err);
}

// Wide Gauss-Jordan (mp a multiple of 128): the inverse of the padded matrix
// in C0 after mp/128 steps, ping-ponging between C0 and C1; returns the
// buffer holding it.  P: 128 x 128 scratch (the current pivot block's
// inverse), W: mp x 128 scratch.
double* launch_gj_wide(hipStream_t st, int mp, double* C0, double* C1, double* P, double* W, int* err) {
  double* A = C0;
  double* B = C1;
  const int nt = mp / kWB;
  k_gjw_pivot<<<1, 256, 0, st>>>(mp, 0, A, P, err);
  for (int k0 = 0; k0 < mp; k0 += kWB) {
    const int k1 = k0 + kWB < mp ? k0 + kWB : -1;
    k_gjw_panel<<<mp / 64, 256, 0, st>>>(mp, k0, A, P, W);
    // P is consumed by the panel kernel before the tiles write P_{k+1} into it
    k_gjw_tiles<<<nt * nt, 256, 0, st>>>(mp, k0, k1, A, W, B, P, err);
    std::swap(A, B);
  }
  return A;
}

// LDS one block of the wide Gauss-Jordan pivot kernel needs
size_t gj_wide_lds_bytes() { return sizeof(GjwShared); }

// Block LU of a large capacitance (mp a multiple of 128), in place and with
// the same pivoting as the Gauss-Jordan steps (partial pivoting inside each
// 128 x 128 diagonal block, which C's dominant contact diagonal allows):
//   C = L U,  L unit block-lower with L_iK = A_iK P_k,  U_KK = A_KK,
//   U_Kj = A_Kj (j > K),
// with A the Schur complement at step k and P_k = A_KK^{-1}.  The factors
// overwrite C as: strictly lower blocks L_iK; strictly upper blocks
// V_Kj = P_k A_Kj (= U_KK^{-1} U_Kj, so that the backward substitution is
// unit as well); diagonal blocks unused; P_k stored apart, mp/128 blocks of
// 128 x 128.  Then C^{-1} g = V^{-1} diag(P) L^{-1} g with V unit
// block-upper: two block substitutions and one block-diagonal product.
// Work: the trailing rank-128 updates, 2/3 mp^3, against 2 mp^3 for the
// explicit inverse.  Per step (K = k0 .. k0 + 127):
//   k_lu_colpanel  L_iK = A_iK P_k for the rows below K, in place;
//   k_lu_tiles_next, k_lu_tiles_rest  A_ij -= L_iK A_Kj for the 128 x 128
//                  tiles below and right of K, in place; the first tile is
//                  the next pivot block and is also inverted (P_{k+1});
// and, for each step once its next-column and trailing updates have run,
// k_lu_rowpanels: V_Kj = P_k A_Kj for the columns right of K, in place (row
// panels are not read again after that).
// P_0 comes from k_gjw_pivot.
__global__ void __launch_bounds__(256) k_lu_colpanel(int mp, int k0, double* __restrict__ A,
                                                     const double* __restrict__ P) {
  __shared__ double As[64][kWKC + 1];
  __shared__ double Bs[kWKC][kWB + 1];
  const int r0 = k0 + kWB + blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  // chunk kc of the panel (64 x 32) and of P (32 x 128), staged through
  // registers; the next chunk is in flight during the current products
  double ap[8], bp[16];
  auto load = [&](int kc) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      ap[u] = A[(size_t)(r0 + (e >> 5)) * mp + k0 + kc + (e & 31)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u;
      bp[u] = P[(size_t)(kc + (e >> 7)) * kWB + (e & 127)];
    }
  };
  d4 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = d4{0, 0, 0, 0};
  load(0);
  for (int kc = 0; kc < kWB; kc += kWKC) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      As[e >> 5][e & 31] = ap[u];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u;
      Bs[e >> 7][e & 127] = bp[u];
    }
    __syncthreads();
    if (kc + kWKC < kWB) load(kc + kWKC);
#pragma unroll
    for (int k4 = 0; k4 < kWKC; k4 += 4) {
      const double a = As[16 * w + li][k4 + lk];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[k4 + lk][16 * q + li], acc[q], 0, 0, 0);
    }
    __syncthreads();
  }
  // every block reads all of its rows' panel entries before this point
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) A[(size_t)(r0 + 16 * w + lk + 4 * e) * mp + k0 + 16 * q + li] = acc[q][e];
}

// V_Kj = P_k A_Kj for the steps k_lo <= k < k_hi at once (no step reads a
// row panel again once its own next-column and trailing updates have run),
// one block per 128 x 64 column slab right of each diagonal block; block b
// is slab b - S(k) of step k, S(k) = sum_{k_lo <= i < k} 2 (nb - 1 - i).
__global__ void __launch_bounds__(256) k_lu_rowpanels(int mp, int k_lo, double* __restrict__ A,
                                                      const double* __restrict__ Pall) {
  __shared__ double Ps[kWB][kWKC + 1];
  __shared__ double Bs[kWKC][64 + 1];
  const int nb = mp / kWB;
  int k = k_lo, b = blockIdx.x;
  while (b >= 2 * (nb - 1 - k)) {
    b -= 2 * (nb - 1 - k);
    ++k;
  }
  const int k0 = k * kWB, j0 = k0 + kWB + 64 * b;
  const double* P = Pall + (size_t)k * kWB * kWB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  double pp[16], ap[8];
  auto load = [&](int kc) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u;
      pp[u] = P[(size_t)(e >> 5) * kWB + kc + (e & 31)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      ap[u] = A[(size_t)(k0 + kc + (e >> 6)) * mp + j0 + (e & 63)];
    }
  };
  d4 acc[2][4];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = d4{0, 0, 0, 0};
  load(0);
  for (int kc = 0; kc < kWB; kc += kWKC) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u;
      Ps[e >> 5][e & 31] = pp[u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      Bs[e >> 6][e & 63] = ap[u];
    }
    __syncthreads();
    if (kc + kWKC < kWB) load(kc + kWKC);
#pragma unroll
    for (int k4 = 0; k4 < kWKC; k4 += 4) {
      double av[2], bv[4];
#pragma unroll
      for (int p = 0; p < 2; ++p) av[p] = Ps[32 * w + 16 * p + li][k4 + lk];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = Bs[k4 + lk][16 * q + li];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
    __syncthreads();
  }
  // the block has read all of its slab before this point
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        A[(size_t)(k0 + 32 * w + 16 * p + lk + 4 * e) * mp + j0 + 16 * q + li] = acc[p][q][e];
}

// One 128 x 128 tile (I0, J0) of the trailing update at step k0,
// A_ij -= L_iK A_Kj, in place: the panels in KC-wide chunks through LDS
// (the next chunk loaded into registers while the current one is
// multiplied), each wavefront a 64 x 64 quadrant of 4 x 4 FP64 MFMA tiles.
// On return acc holds the updated tile (already written to A).
template <int KC>
__device__ __forceinline__ void lu_tile(int mp, int k0, int I0, int J0, double* __restrict__ A,
                                        double (*__restrict__ Ws)[KC + 1], double (*__restrict__ Rs)[kWB + 1],
                                        d4 (&acc)[4][4]) {
  constexpr int NP = kWB * KC / 256;  // panel entries per thread and chunk
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
  double wpre[NP], rpre[NP];
  auto load_chunk = [&](int kc) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = tid + 256 * u;
      wpre[u] = A[(size_t)(I0 + e / KC) * mp + k0 + kc + e % KC];
      rpre[u] = A[(size_t)(k0 + kc + e / kWB) * mp + J0 + e % kWB];
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = tid + 256 * u;
      Ws[e / KC][e % KC] = wpre[u];
      Rs[e / kWB][e % kWB] = rpre[u];
    }
  };
  load_chunk(0);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        acc[p][q][e] = A[(size_t)(I0 + wr + 16 * p + lk + 4 * e) * mp + J0 + wc + 16 * q + li];
  store_chunk();
  __syncthreads();
  for (int kc = 0; kc < kWB; kc += KC) {
    const bool more = kc + KC < kWB;
    if (more) load_chunk(kc + KC);
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) av[p] = -Ws[wr + 16 * p + li][k4 + lk];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = Rs[k4 + lk][wc + 16 * q + li];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      store_chunk();
      __syncthreads();
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        A[(size_t)(I0 + wr + 16 * p + lk + 4 * e) * mp + J0 + wc + 16 * q + li] = acc[p][q][e];
}

// The trailing update of step k0 in two launches on two streams:
//   k_lu_tiles_next  the first tile column (the next step's panel), one
//                    block per tile and CU (141 KB of LDS); block 0 is the
//                    next pivot block (blocks start in index order) and
//                    also inverts it (P_{k+1});
//   k_lu_tiles_rest  every other trailing tile, two blocks per CU (34 KB of
//                    LDS, 16-wide chunks, the tile's old values read beside
//                    the products), no inversion,
// so that the pivot chain runs beside the bulk of the update.  Both read the column panel left of the
// trailing matrix and the row panel above it, which neither writes.
__global__ void __launch_bounds__(256, 1) k_lu_tiles_next(int mp, int k0, double* __restrict__ A,
                                                          double* __restrict__ Pnext, int* __restrict__ err) {
  __shared__ GjwShared sh;
  const int I0 = k0 + kWB + blockIdx.x * kWB, J0 = k0 + kWB;
  d4 acc[4][4];
  lu_tile<kWKC>(mp, k0, I0, J0, A, sh.t.Ws, sh.t.Rs, acc);
  if (blockIdx.x != 0) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
  double* M = sh.p.M;
  __syncthreads();  // the panels in LDS are no longer read
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) M[(wr + 16 * p + lk + 4 * e) * kWL + wc + 16 * q + li] = acc[p][q][e];
  __syncthreads();
  invert128_lds(M, sh.p.Ps, sh.p.prow, err);
  for (int e = tid; e < kWB * kWB; e += 256) Pnext[e] = M[(e / kWB) * kWL + e % kWB];
}

// One 128 x 128 tile of the bulk trailing update with the tile's own old
// values read beside the products instead of before them: the accumulators
// start at zero, and in each of the eight 16-wide panel chunks one batch of
// eight old values per lane is requested with the next chunk's panels and
// added once the chunk's products are done (a batch has one chunk of
// products to arrive, and only eight registers are held for it).  Two blocks
// per CU, so that one block's barriers and waits are covered by the other's
// products.
constexpr int kRestKC = 16;
__device__ __forceinline__ void lu_tile_rest(int mp, int k0, int I0, int J0, double* __restrict__ A,
                                             double (*__restrict__ Ws)[kRestKC + 1],
                                             double (*__restrict__ Rs)[kWB + 1]) {
  constexpr int KC = kRestKC, NP = kWB * KC / 256, NCH = kWB / KC;
  static_assert(NCH == 8, "one batch of eight old values per chunk");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
  double wpre[NP], rpre[NP], ob[8];
  auto load_chunk = [&](int kc) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = tid + 256 * u;
      wpre[u] = A[(size_t)(I0 + e / KC) * mp + k0 + kc + e % KC];
      rpre[u] = A[(size_t)(k0 + kc + e / kWB) * mp + J0 + e % kWB];
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = tid + 256 * u;
      Ws[e / KC][e % KC] = wpre[u];
      Rs[e / kWB][e % kWB] = rpre[u];
    }
  };
  d4 acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = d4{0, 0, 0, 0};
  load_chunk(0);
  store_chunk();
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (c + 1 < NCH) load_chunk((c + 1) * KC);
    // batch c: row block p = c / 2, column blocks 2 (c % 2) and 2 (c % 2) + 1
    const int pb = c >> 1, q0 = 2 * (c & 1);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      ob[u] = A[(size_t)(I0 + wr + 16 * pb + lk + 4 * (u & 3)) * mp + J0 + wc + 16 * (q0 + (u >> 2)) + li];
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) av[p] = -Ws[wr + 16 * p + li][k4 + lk];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = Rs[k4 + lk][wc + 16 * q + li];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[pb][q0 + (u >> 2)][u & 3] += ob[u];
    if (c + 1 < NCH) {
      __syncthreads();  // every wave is done with the chunk in LDS
      store_chunk();
      __syncthreads();
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        A[(size_t)(I0 + wr + 16 * p + lk + 4 * e) * mp + J0 + wc + 16 * q + li] = acc[p][q][e];
}

__global__ void __launch_bounds__(256, 2) k_lu_tiles_rest(int mp, int k0, double* __restrict__ A) {
  __shared__ double Ws[kWB][kRestKC + 1];
  __shared__ double Rs[kRestKC][kWB + 1];
  const int base = k0 + kWB, nt = (mp - base) / kWB, nc = nt - 1;
  // Tile order for the L2s: blocks go to the eight XCDs round-robin, so the
  // logical index L gives XCD x one contiguous range of L, and L runs down
  // groups of eight tile rows column by column, so the tiles an XCD holds at
  // once share about eight row panels and eight column panels (2 MB of its
  // 4 MB L2) instead of touching every column panel.
  const unsigned nb = gridDim.x, q = nb / 8, r = nb % 8, x = blockIdx.x % 8;
  const int L = (int)(x * q + min(x, r) + blockIdx.x / 8);
  const int per = 8 * nc, g0 = (L / per) * 8, gh = min(8, nt - g0), w = L % per;
  const int I0 = base + (g0 + w % gh) * kWB, J0 = base + kWB + (w / gh) * kWB;
  lu_tile_rest(mp, k0, I0, J0, A, Ws, Rs);
}

// Pall: mp/128 blocks of 128 x 128 (the inverted pivot blocks P_k).  The
// factorisation is launch_lu_pivot0, then per step k = 0 .. mp/128 - 2
// launch_lu_colpanel, then launch_lu_tiles_next and launch_lu_tiles_rest
// (concurrently; the next step's launch_lu_tiles_next also waits for this
// step's rest); launch_lu_rowpanels and launch_lu_groups over ranges of
// finished steps and groups, beside later steps or after the last.
void launch_lu_pivot0(hipStream_t st, int mp, double* A, double* Pall, int* err) {
  k_gjw_pivot<<<1, 256, 0, st>>>(mp, 0, A, Pall, err);
}
void launch_lu_colpanel(hipStream_t st, int mp, int k, double* A, const double* Pall) {
  const int k0 = k * kWB;
  k_lu_colpanel<<<(mp - k0 - kWB) / 64, 256, 0, st>>>(mp, k0, A, Pall + (size_t)k * kWB * kWB);
}
// The trailing update of step k: the next panel's column with the pivot
// inversion, and the other tiles (no launch when there are none).
void launch_lu_tiles_next(hipStream_t st, int mp, int k, double* A, double* Pall, int* err) {
  const int k0 = k * kWB, nt = (mp - k0 - kWB) / kWB;
  k_lu_tiles_next<<<nt, 256, 0, st>>>(mp, k0, A, Pall + (size_t)(k + 1) * kWB * kWB, err);
}
void launch_lu_tiles_rest(hipStream_t st, int mp, int k, double* A) {
  const int k0 = k * kWB, nt = (mp - k0 - kWB) / kWB;
  if (nt > 1) k_lu_tiles_rest<<<nt * (nt - 1), 256, 0, st>>>(mp, k0, A);
}
void launch_lu_rowpanels(hipStream_t st, int mp, double* A, const double* Pall, int k_lo, int k_hi) {
  const int nb = mp / kWB;
  if (k_hi > nb - 1) k_hi = nb - 1;
  int blocks = 0;
  for (int k = k_lo; k < k_hi; ++k) blocks += 2 * (nb - 1 - k);
  if (blocks > 0) k_lu_rowpanels<<<blocks, 256, 0, st>>>(mp, k_lo, A, Pall);
}


// ---- Grouped substitutions ----
// The substitutions with the block-LU factors take one launch per group of
// kLuGroup consecutive diagonal blocks instead of one per block: with G a
// group, L_GG its unit block-lower diagonal part and V_GG its unit
// block-upper one, the factors are rewritten once after the factorisation:
//   strictly lower blocks inside G   <- L_GG^{-1}   (unit diagonal implied),
//   strictly upper blocks inside G   <- V_GG^{-1},
//   lower blocks left of G, below it <- L_iG L_GG^{-1},
//   upper blocks right of G, above   <- V_iG V_GG^{-1}.
// Forward, group by group: y_G = L_GG^{-1} t_G, and t_i -= (L_iG L_GG^{-1})
// t_G for the rows below, both from the group's t before the launch; the
// backward pass mirrors it with V.  Extra work at setup: about
// 2 kLuGroup-1/kLuGroup 128 mp^2 flops; per solve, about a quarter of the
// launches.
constexpr int kLuGroup = 4;

struct LuGemmShared {
  double Ws[kWB][kWKC + 1];
  double Rs[kWKC][kWB + 1];
};

// acc (each wavefront's 64 x 64 quadrant of a 128 x 128 block, the
// lu_tile layout) += Ablk Bblk, both 128 x 128 blocks of a row-major
// matrix with leading dimension ld, staged through LDS in 32-wide chunks.
__device__ __forceinline__ void mma128(d4 (&acc)[4][4], const double* __restrict__ Ab, const double* __restrict__ Bb,
                                       int ld, LuGemmShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
  for (int kc = 0; kc < kWB; kc += kWKC) {
    double wv[kWPre], rv[kWPre];
#pragma unroll
    for (int u = 0; u < kWPre; ++u) {
      const int e = tid + 256 * u;
      wv[u] = Ab[(size_t)(e / kWKC) * ld + kc + e % kWKC];
      rv[u] = Bb[(size_t)(kc + e / kWB) * ld + e % kWB];
    }
    __syncthreads();  // the previous chunk's products have read the panels
#pragma unroll
    for (int u = 0; u < kWPre; ++u) {
      const int e = tid + 256 * u;
      sh.Ws[e / kWKC][e % kWKC] = wv[u];
      sh.Rs[e / kWB][e % kWB] = rv[u];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < kWKC; k4 += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) av[p] = sh.Ws[wr + 16 * p + li][k4 + lk];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = sh.Rs[k4 + lk][wc + 16 * q + li];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void acc_io(d4 (&acc)[4][4], double* __restrict__ Cb, int ld, bool store, double sgn) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double* c = Cb + (size_t)(wr + 16 * p + lk + 4 * e) * ld + wc + 16 * q + li;
        if (store)
          *c = sgn * acc[p][q][e];
        else
          acc[p][q][e] = *c;
      }
}

// Blocks written here are read back by other wavefronts of the block: the
// stores complete device-wide before the barrier, and every wavefront's
// view of the cache is refreshed after it.
__device__ __forceinline__ void publish_block() {
  __threadfence();
  __syncthreads();
  __threadfence();
}

// L_GG^{-1} and V_GG^{-1} of the groups in place, two blocks per group
// (blockIdx.y 0: the lower triangle, 1: the upper one; they touch disjoint
// blocks):
//   Linv_ab = -(L_ab + sum_{b<c<a} L_ac Linv_cb)  (a > b; columns b ascending,
//             rows a ascending, so L_ac is still the factor),
//   Vinv_ab = -(V_ab + sum_{a<c<b} V_ac Vinv_cb)  (a < b; columns b
//             descending, rows a descending).
// Within a triangle the columns stay in that order: a column reads factor
// blocks of the later columns, which those columns overwrite.
__global__ void __launch_bounds__(256) k_lu_group_inv(int mp, int g_lo, double* __restrict__ A) {
  __shared__ LuGemmShared sh;
  const int nb = mp / kWB, b0 = (g_lo + (int)blockIdx.x) * kLuGroup, g = min(kLuGroup, nb - b0);
  auto blk = [&](int a, int b) { return A + (size_t)(b0 + a) * kWB * mp + (size_t)(b0 + b) * kWB; };
  d4 acc[4][4];
  if (blockIdx.y == 0) {
    for (int b = 0; b + 1 < g; ++b)
      for (int a = b + 1; a < g; ++a) {
        acc_io(acc, blk(a, b), mp, false, 1.0);
        for (int c = b + 1; c < a; ++c) mma128(acc, blk(a, c), blk(c, b), mp, sh);
        acc_io(acc, blk(a, b), mp, true, -1.0);
        publish_block();
      }
  } else {
    for (int b = g - 1; b >= 1; --b)
      for (int a = b - 1; a >= 0; --a) {
        acc_io(acc, blk(a, b), mp, false, 1.0);
        for (int c = a + 1; c < b; ++c) mma128(acc, blk(a, c), blk(c, b), mp, sh);
        acc_io(acc, blk(a, b), mp, true, -1.0);
        publish_block();
      }
  }
}

// The blocks outside the groups, one block per (128-row block r, group):
// below the group (lower) L_rb <- L_rb + sum_{c>b} L_rc Linv_cb, columns b
// ascending; above it (upper) V_rb <- V_rb + sum_{c<b} V_rc Vinv_cb, columns
// b descending.  Each output is written once and not read again here.
__global__ void __launch_bounds__(256) k_lu_group_apply(int mp, int g_lo, double* __restrict__ A) {
  __shared__ LuGemmShared sh;
  const int nb = mp / kWB, r = blockIdx.x, b0 = (g_lo + (int)blockIdx.y) * kLuGroup, g = min(kLuGroup, nb - b0);
  auto blk = [&](int i, int j) { return A + (size_t)i * kWB * mp + (size_t)j * kWB; };
  d4 acc[4][4];
  if (r >= b0 + g) {
    for (int b = 0; b + 1 < g; ++b) {
      acc_io(acc, blk(r, b0 + b), mp, false, 1.0);
      for (int c = b + 1; c < g; ++c) mma128(acc, blk(r, b0 + c), blk(b0 + c, b0 + b), mp, sh);
      acc_io(acc, blk(r, b0 + b), mp, true, 1.0);
    }
  } else if (r < b0) {
    for (int b = g - 1; b >= 1; --b) {
      acc_io(acc, blk(r, b0 + b), mp, false, 1.0);
      for (int c = 0; c < b; ++c) mma128(acc, blk(r, b0 + c), blk(b0 + c, b0 + b), mp, sh);
      acc_io(acc, blk(r, b0 + b), mp, true, 1.0);
    }
  }
}

// Groups g_lo <= G < g_hi (a group's blocks are final once its last step's
// updates have run, and no later step reads them; groups touch disjoint
// block columns).
void launch_lu_groups(hipStream_t st, int mp, double* A, int g_lo, int g_hi) {
  const int nb = mp / kWB, ng = (nb + kLuGroup - 1) / kLuGroup;
  if (g_hi > ng) g_hi = ng;
  if (nb < 2 || g_hi <= g_lo) return;
  k_lu_group_inv<<<dim3(g_hi - g_lo, 2), 256, 0, st>>>(mp, g_lo, A);
  k_lu_group_apply<<<dim3(nb, g_hi - g_lo), 256, 0, st>>>(mp, g_lo, A);
}

int lu_group_blocks() { return kLuGroup; }

}  // namespace adj
