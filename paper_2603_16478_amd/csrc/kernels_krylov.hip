// Krylov solve of the adjoint system (Sec. 5.4): right-preconditioned
// restarted GMRES, classical Gram-Schmidt applied twice, Givens rotations,
// the Woodbury preconditioner
//     P r = A^{-1} r - h^2 A^{-1} Hq^T X Hq A^{-1} r,   X = C^{-1}
// with A^{-1} = S^T S applied as two sparse products (Sec. 3.4) and
// A^{-1} Hq^T = Z (x) Q^T, and the matrix-free product with Acal^T as one
// block-sparse product (contacts act on diagonal blocks only, so they are
// folded into those blocks at setup).
//
// The basis is stored unnormalised with per-vector scale factors: V_i =
// scale[i] * Vt_i, which spares a normalisation pass.  Iterations run from
// device-side state (current index j and an `active` flag), so the host can
// launch a chunk of iterations without reading anything back; kernels of an
// inactive cycle return immediately.
#include "device_common.h"
#include "krylov_state.h"

namespace adj {


__device__ __forceinline__ bool gm_inactive(const GmresState* s) { return s && s->active == 0; }

// y = S x (3 interleaved right-hand sides); one wavefront per row.
// `st` only gates the launch (inactive cycle -> return).  With use_j = 1
// the input is the current basis vector, x = xbase + j*stride scaled by
// scale[j] (st and scale must then be non-null); otherwise x = xbase.
__global__ void __launch_bounds__(256) k_spmv_csr3(int nrows, const long long* __restrict__ rp,
                                                   const int* __restrict__ cj,
                                                   const double* __restrict__ cx,
                                                   const double* __restrict__ xbase, long long stride,
                                                   const double* __restrict__ scale,
                                                   const GmresState* __restrict__ st, int use_j,
                                                   double* __restrict__ y) {
  if (gm_inactive(st)) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (row >= nrows) return;
  const double* x = xbase;
  double sc = 1.0;
  if (use_j) {
    x = xbase + (long long)st->j * stride;
    sc = scale[st->j];
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (long long p = rp[row] + lane; p < rp[row + 1]; p += 64) {
    const double v = cx[p];
    const int c = cj[p];
    a0 += v * x[3 * c];
    a1 += v * x[3 * c + 1];
    a2 += v * x[3 * c + 2];
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  if (lane == 0) {
    y[3 * row] = sc * a0;
    y[3 * row + 1] = sc * a1;
    y[3 * row + 2] = sc * a2;
  }
}

// Load-balanced variant: the host packs rows into tasks of one block each:
// a long row (flag kBigRow) is reduced by the whole block, otherwise up to
// four short rows are handled by one wavefront each (-1 = empty slot).
constexpr int kBigRow = 0x40000000;

// ACC: y[row] += alpha * (row . x) instead of y[row] = scale * (row . x)
// (rows not listed in the tasks keep their values).
template <class MT, bool ACC = false>
__global__ void __launch_bounds__(256) k_spmv_tasks(const int4* __restrict__ tasks,
                                                    const long long* __restrict__ rp,
                                                    const int* __restrict__ cj,
                                                    const MT* __restrict__ cx,
                                                    const double* __restrict__ xbase, long long stride,
                                                    const double* __restrict__ scale,
                                                    const GmresState* __restrict__ st, int use_j,
                                                    double* __restrict__ y, double alpha = 0.0) {
  // the task is loaded before the state is checked, so the two loads overlap
  // (the level launches of a sweep are chains of a few dependent loads)
  const int4 t = tasks[blockIdx.x];
  if (gm_inactive(st) && t.x != INT_MIN) return;  // t.x is never INT_MIN: keeps the task load first
  __shared__ double lds[32];
  const double* x = xbase;
  double sc = 1.0;
  if (use_j) {
    x = xbase + (long long)st->j * stride;
    sc = scale[st->j];
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (t.x >= 0 && (t.x & kBigRow)) {
    const int row = t.x & ~kBigRow;
    row_dot3<256, 4>(rp[row], rp[row + 1], threadIdx.x, cj, cx, x, a0, a1, a2);
    a0 = block_sum(a0, lds);
    a1 = block_sum(a1, lds);
    a2 = block_sum(a2, lds);
    if (threadIdx.x == 0) {
      if constexpr (ACC) {
        y[3 * row] += alpha * a0;
        y[3 * row + 1] += alpha * a1;
        y[3 * row + 2] += alpha * a2;
      } else {
        y[3 * row] = sc * a0;
        y[3 * row + 1] = sc * a1;
        y[3 * row + 2] = sc * a2;
      }
    }
    return;
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = (w == 0) ? t.x : (w == 1) ? t.y : (w == 2) ? t.z : t.w;
  if (row < 0) return;
  row_dot3<64, 4>(rp[row], rp[row + 1], lane, cj, cx, x, a0, a1, a2);
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  if (lane == 0) {
    if constexpr (ACC) {
      y[3 * row] += alpha * a0;
      y[3 * row + 1] += alpha * a1;
      y[3 * row + 2] += alpha * a2;
    } else {
      y[3 * row] = sc * a0;
      y[3 * row + 1] = sc * a1;
      y[3 * row + 2] = sc * a2;
    }
  }
}

// The k lowest levels of a sweep in one launch, one block per independent
// part of those levels (host: sweep_parts): per height h (forward: 0 .. k-1;
// backward: k-1 .. 0) the block forms tmp[row] -= A_row . out for the part's
// rows at h, then out[row] = D_row . tmp, with a block barrier after each
// phase, since every entry an A row reads lies in the part (or, backwards,
// above the fused levels, finished by the launches before).  Forward: A = the
// rows of L left of their segment, D = the inverted diagonal blocks, out = y;
// backward: A = the columns of L below their segment, D = the transposed
// inverses, out = z.  16 lanes per row, 16 rows at a time.
template <class MT>
__global__ void __launch_bounds__(256) k_sweep_parts(int fwd, int k, const int* __restrict__ rows,
                                                     const int* __restrict__ off, const long long* __restrict__ Ap,
                                                     const int* __restrict__ Aj, const MT* __restrict__ Ax,
                                                     const long long* __restrict__ Dp, const int* __restrict__ Dj,
                                                     const MT* __restrict__ Dx, const GmresState* __restrict__ st,
                                                     double* out, double* tmp) {
  if (gm_inactive(st)) return;
  const int* o = off + (size_t)blockIdx.x * (k + 1);
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  for (int s = 0; s < k; ++s) {
    const int h = fwd ? s : k - 1 - s;
    const int r0 = o[h], r1 = o[h + 1];
    for (int i = r0 + g; i < r1; i += 16) {
      const int row = rows[i];
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      row_dot3<16, 4>(Ap[row], Ap[row + 1], l, Aj, Ax, out, a0, a1, a2);
      a0 = group_sum<16>(a0);
      a1 = group_sum<16>(a1);
      a2 = group_sum<16>(a2);
      if (l == 0) {
        tmp[3 * row] -= a0;
        tmp[3 * row + 1] -= a1;
        tmp[3 * row + 2] -= a2;
      }
    }
    __syncthreads();
    for (int i = r0 + g; i < r1; i += 16) {
      const int row = rows[i];
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      row_dot3<16, 4>(Dp[row], Dp[row + 1], l, Dj, Dx, tmp, a0, a1, a2);
      a0 = group_sum<16>(a0);
      a1 = group_sum<16>(a1);
      a2 = group_sum<16>(a2);
      if (l == 0) {
        out[3 * row] = a0;
        out[3 * row + 1] = a1;
        out[3 * row + 2] = a2;
      }
    }
    __syncthreads();
  }
}

template <class MT>
static void sweep_parts_impl(hipStream_t s, int nparts, int fwd, int k, const int* rows, const int* off,
                             const long long* Ap, const int* Aj, const MT* Ax, const long long* Dp, const int* Dj,
                             const MT* Dx, const GmresState* st, double* out, double* tmp) {
  if (nparts <= 0 || k <= 0) return;
  k_sweep_parts<MT><<<nparts, 256, 0, s>>>(fwd, k, rows, off, Ap, Aj, Ax, Dp, Dj, Dx, st, out, tmp);
}
void launch_sweep_parts(hipStream_t s, int nparts, int fwd, int k, const int* rows, const int* off,
                        const long long* Ap, const int* Aj, const double* Ax, const long long* Dp, const int* Dj,
                        const double* Dx, const GmresState* st, double* out, double* tmp) {
  sweep_parts_impl(s, nparts, fwd, k, rows, off, Ap, Aj, Ax, Dp, Dj, Dx, st, out, tmp);
}
void launch_sweep_parts(hipStream_t s, int nparts, int fwd, int k, const int* rows, const int* off,
                        const long long* Ap, const int* Aj, const float* Ax, const long long* Dp, const int* Dj,
                        const float* Dx, const GmresState* st, double* out, double* tmp) {
  sweep_parts_impl(s, nparts, fwd, k, rows, off, Ap, Aj, Ax, Dp, Dj, Dx, st, out, tmp);
}

// Y values of the Woodbury correction gathered from the rows of S^T:
// yval[e] = STx[src[e]].
__global__ void k_gather_values(long long n, const long long* __restrict__ src, const double* __restrict__ STx,
                                double* __restrict__ yval) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) yval[e] = STx[src[e]];
}

void launch_gather_values(hipStream_t s, long long n, const long long* src, const double* STx, double* yval) {
  if (n <= 0) return;
  k_gather_values<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, src, STx, yval);
}

// Block-Jacobi preconditioner: y_v = B_v^{-1} x_v with B_v the 3x3
// diagonal block of the assembled matrix (row v's block at slot
// diag_slot[v], row-major), inverted per apply by the adjugate (B_v is the
// mass block plus stiffness and contact terms, far from singular); with
// `point` set, only the block's diagonal is inverted (point Jacobi).  The
// input vector follows the same lazily scaled basis convention as the
// sparse-inverse product.
template <class MT>
__global__ void k_block_jacobi(int nv, const int* __restrict__ diag_slot, const MT* __restrict__ val,
                               const double* __restrict__ xbase, long long stride, const double* __restrict__ scale,
                               const GmresState* __restrict__ st, int use_j, int point, double* __restrict__ y) {
  if (gm_inactive(st)) return;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const double* x = xbase;
  double sc = 1.0;
  if (use_j) {
    x = xbase + (long long)st->j * stride;
    sc = scale[st->j];
  }
  const MT* b = val + 9LL * diag_slot[v];
  if (point) {
    y[3 * v] = sc * x[3 * v] / (double)b[0];
    y[3 * v + 1] = sc * x[3 * v + 1] / (double)b[4];
    y[3 * v + 2] = sc * x[3 * v + 2] / (double)b[8];
    return;
  }
  const double a00 = b[0], a01 = b[1], a02 = b[2], a10 = b[3], a11 = b[4], a12 = b[5], a20 = b[6], a21 = b[7],
               a22 = b[8];
  const double c00 = a11 * a22 - a12 * a21, c01 = a02 * a21 - a01 * a22, c02 = a01 * a12 - a02 * a11;
  const double c10 = a12 * a20 - a10 * a22, c11 = a00 * a22 - a02 * a20, c12 = a02 * a10 - a00 * a12;
  const double c20 = a10 * a21 - a11 * a20, c21 = a01 * a20 - a00 * a21, c22 = a00 * a11 - a01 * a10;
  const double inv = sc / (a00 * c00 + a01 * c10 + a02 * c20);
  const double x0 = x[3 * v], x1 = x[3 * v + 1], x2 = x[3 * v + 2];
  y[3 * v] = inv * (c00 * x0 + c01 * x1 + c02 * x2);
  y[3 * v + 1] = inv * (c10 * x0 + c11 * x1 + c12 * x2);
  y[3 * v + 2] = inv * (c20 * x0 + c21 * x1 + c22 * x2);
}

// t = X (Hq u): each block first forms g = Hq u (m entries) in LDS, then one
// wavefront per row of X.
template <class MT>
__global__ void __launch_bounds__(256) k_wb_gather(int m, int mp, int rows, const int* __restrict__ row_c,
                                                   const int* __restrict__ row_i,
                                                   const int* __restrict__ vid,
                                                   const double* __restrict__ Q,
                                                   const MT* __restrict__ X,
                                                   const double* __restrict__ u,
                                                   const GmresState* __restrict__ st,
                                                   double* __restrict__ t) {
  if (gm_inactive(st)) return;
  extern __shared__ double g[];
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    const int c = row_c[r];
    const double* q = Q + 9 * c + 3 * row_i[r];
    const int v = vid[c];
    g[r] = q[0] * u[3 * v] + q[1] * u[3 * v + 1] + q[2] * u[3 * v + 2];
  }
  __syncthreads();
  const int r0 = blockIdx.x * rows;
  wb_gather_rows(r0, min(m, r0 + rows), m, X + (size_t)r0 * mp, mp, g, t);
}

// y = u - h^2 Z t' with t'_cv = sum over the contacts at vertex cv of Q_c^T t_c
// (computed per block in LDS); one wavefront per vertex row.
template <class MT>
__global__ void __launch_bounds__(256) k_wb_correct(int nv, int ncv, int rows, const int* __restrict__ cv_ptr,
                                                    const int* __restrict__ c_row0,
                                                    const int* __restrict__ c_nrow,
                                                    const double* __restrict__ Q,
                                                    const double* __restrict__ t,
                                                    const MT* __restrict__ Z, double h2,
                                                    const double* __restrict__ u,
                                                    const GmresState* __restrict__ st,
                                                    double* __restrict__ y) {
  if (gm_inactive(st)) return;
  extern __shared__ double tp[];  // [ncv][3]
  for (int a = threadIdx.x; a < ncv; a += blockDim.x) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int c = cv_ptr[a]; c < cv_ptr[a + 1]; ++c)
      for (int i = 0; i < c_nrow[c]; ++i) {
        const double tv = t[c_row0[c] + i];
        const double* q = Q + 9 * c + 3 * i;
        s0 += q[0] * tv;
        s1 += q[1] * tv;
        s2 += q[2] * tv;
      }
    tp[3 * a] = s0;
    tp[3 * a + 1] = s1;
    tp[3 * a + 2] = s2;
  }
  __syncthreads();
  const int v0 = blockIdx.x * rows;
  wb_rows(v0, min(nv, v0 + rows), ncv, Z + (size_t)v0 * ncv, tp, h2, u, y);
}

// w = Acal^T x, block-sparse 3x3; LANES lanes per block row (256 / LANES
// rows per block).  Output to outbase + (j+1)*stride when state is given.
template <class MT, int LANES>
__global__ void __launch_bounds__(256) k_bsr_spmv(int nv, const int* __restrict__ rowptr,
                                                  const int* __restrict__ col,
                                                  const MT* __restrict__ val,
                                                  const double* __restrict__ val64, long long soa,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ outbase, long long stride,
                                                  const GmresState* __restrict__ st) {
  if (gm_inactive(st)) return;
  const int sub = threadIdx.x & (LANES - 1);
  const int row = blockIdx.x * (blockDim.x / LANES) + threadIdx.x / LANES;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (row < nv) {
    for (int p = rowptr[row] + sub; p < rowptr[row + 1]; p += LANES) {
      const int c = col[p];
      const double x0 = x[3 * c], x1 = x[3 * c + 1], x2 = x[3 * c + 2];
      block_madd<MT>(val, val64, (size_t)p, c == row, x0, x1, x2, a0, a1, a2, soa);
    }
  }
  a0 = group_sum<LANES>(a0);
  a1 = group_sum<LANES>(a1);
  a2 = group_sum<LANES>(a2);
  if (row < nv && sub == 0) {
    double* out = outbase + (st ? (long long)(st->j + 1) * stride : 0);
    out[3 * row] = a0;
    out[3 * row + 1] = a1;
    out[3 * row + 2] = a2;
  }
}

// Reductions without inter-block handshakes.  A kernel that needs a global
// sum writes one partial per block; the kernels that consume the sum re-add
// the partials themselves (every block, in the same fixed order, so all of
// them get the same bits), and state that must have a single writer is
// updated by a one-block kernel.  A "last block reduces" handshake (fence +
// atomic counter) serialises the blocks on this multi-die GPU and costs
// more than one extra launch.
constexpr int kLd = 130;  // partials of one block: [0 .. 129], basis index i

// w = Acal^T y fused with the first Gram-Schmidt pass: the block writes its
// rows of w = Vt_{j+1} and the partial dots Vt_i . w over those rows
// (i <= j) to P[blockIdx.x * kLd + i].  jfix >= 0 overrides j (PCG: w =
// Acal^T p with p = Vt_0, w = Vt_1, partial p . w).  With Zb given, the
// block also stores its rows of y (the preconditioned basis vector) as
// Zb_j, the flexible-GMRES basis the solution is formed from.
template <class MT, int LANES>
__global__ void __launch_bounds__(256) k_bsr_dots(int nv, const int* __restrict__ rowptr,
                                                  const int* __restrict__ col, const MT* __restrict__ val,
                                                  const double* __restrict__ val64, long long soa,
                                                  const double* __restrict__ y, double* __restrict__ Vt,
                                                  long long stride, const GmresState* __restrict__ st, int jfix,
                                                  double* __restrict__ P, double* __restrict__ Zb) {
  if (st->active == 0) return;
  constexpr int R = 256 / LANES;  // rows per block
  __shared__ double wl[3 * R];
  const int j = jfix >= 0 ? jfix : st->j;
  double* w = Vt + (long long)(j + 1) * stride;
  const int sub = threadIdx.x & (LANES - 1), rl = threadIdx.x / LANES;
  const int row0 = blockIdx.x * R, row = row0 + rl;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (row < nv) {
    const int pe = rowptr[row + 1];
#pragma unroll 2
    for (int p = rowptr[row] + sub; p < pe; p += LANES) {
      const int c = col[p];
      const double x0 = y[3 * c], x1 = y[3 * c + 1], x2 = y[3 * c + 2];
      block_madd<MT>(val, val64, (size_t)p, c == row, x0, x1, x2, a0, a1, a2, soa);
    }
  }
  a0 = group_sum<LANES>(a0);
  a1 = group_sum<LANES>(a1);
  a2 = group_sum<LANES>(a2);
  if (sub == 0) {
    const bool ok = row < nv;
    wl[3 * rl] = ok ? a0 : 0.0;
    wl[3 * rl + 1] = ok ? a1 : 0.0;
    wl[3 * rl + 2] = ok ? a2 : 0.0;
    if (ok) {
      w[3 * row] = a0;
      w[3 * row + 1] = a1;
      w[3 * row + 2] = a2;
    }
  }
  if (Zb) {
    const long long e0 = 3LL * row0, ne = 3LL * min(R, nv - row0);
    double* zj = Zb + (long long)j * stride;
    for (long long e = threadIdx.x; e < ne; e += 256) zj[e0 + e] = y[e0 + e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
  const long long e0 = 3LL * row0;
  const int ne = 3 * min(R, nv - row0);
  for (int i = wid; i <= j; i += 4) {
    const double* vi = Vt + (long long)i * stride + e0;
    double d = 0.0;
    for (int e = lane; e < ne; e += 64) d += vi[e] * wl[e];
    d = wave_sum(d);
    if (lane == 0) P[(size_t)blockIdx.x * kLd + i] = d;
  }
}

// Gram-Schmidt update on `rpb` rows per block (64, 128 or 256; T = 256/rpb
// threads per row split the basis range): with c_i = scale_i^2 * sum_b
// Pin[b][i], w -= sum_i c_i Vt_i, where w = Vt_{j+1}.  Block 0 records the
// projection coefficients h_i = scale_i * sum_b Pin[b][i] in hbuf[hoff + i].
// mode 0 (after the first pass): partial dots Vt_i . w -> Pout[b][i];
// mode 1 (after the second pass): partial |w|^2 -> Pout[b][0].
__global__ void __launch_bounds__(256) k_gm_update(long long n, int rpb, double* __restrict__ Vt,
                                                   long long stride, const double* __restrict__ scale,
                                                   const GmresState* __restrict__ st,
                                                   const double* __restrict__ Pin, int nbin,
                                                   double* __restrict__ Pout, double* __restrict__ hbuf,
                                                   int mode) {
  if (st->active == 0) return;
  __shared__ double hs[kLd];
  __shared__ double tmp[256];
  const int j = st->j;
  double* w = Vt + (long long)(j + 1) * stride;
  sum_partials(Pin, nbin, kLd, j + 1, hs, tmp);
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i <= j; i += blockDim.x) hbuf[(mode == 0 ? 0 : kLd) + i] = scale[i] * hs[i];
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += blockDim.x) hs[i] *= scale[i] * scale[i];
  __syncthreads();
  const long long r0 = (long long)blockIdx.x * rpb;
  const int T = blockDim.x / rpb;
  const int rl = threadIdx.x % rpb, part = threadIdx.x / rpb;
  const long long r = r0 + rl;
  double acc = 0.0;
  if (r < n)
    for (int i = part; i <= j; i += T) acc += hs[i] * Vt[(long long)i * stride + r];
  tmp[threadIdx.x] = acc;
  __syncthreads();
  if (part == 0 && r < n) {
    double a = tmp[rl];
    for (int t = 1; t < T; ++t) a += tmp[rl + t * rpb];
    w[r] -= a;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64, nw = blockDim.x / 64;
  if (mode == 0) {
    for (int i = wid; i <= j; i += nw) {
      const double* vi = Vt + (long long)i * stride;
      double d = 0.0;
      for (long long rr = r0 + lane; rr < r0 + rpb && rr < n; rr += 64) d += vi[rr] * w[rr];
      d = wave_sum(d);
      if (lane == 0) Pout[(size_t)blockIdx.x * kLd + i] = d;
    }
  } else {
    double d = 0.0;
    for (long long rr = r0 + threadIdx.x; rr < r0 + rpb && rr < n; rr += blockDim.x) d += w[rr] * w[rr];
    d = block_sum(d, tmp);
    if (threadIdx.x == 0) Pout[(size_t)blockIdx.x * kLd] = d;
  }
}

// One block: |w| from the partial norms, the new Hessenberg column
// (h + h2, |w|), its Givens rotations, the residual estimate and the state.
__global__ void __launch_bounds__(256) k_gm_givens(GmresState* __restrict__ st, const double* __restrict__ P,
                                                   int nb, double* __restrict__ scale,
                                                   const double* __restrict__ hbuf, double* __restrict__ H,
                                                   double* __restrict__ cs, double* __restrict__ sn,
                                                   double* __restrict__ gvec) {
  if (st->active == 0) return;
  __shared__ double nn[1];
  __shared__ double tmp[256];
  sum_partials(P, nb, kLd, 1, nn, tmp);
  if (threadIdx.x != 0) return;
  const int j = st->j;
  const double nrm = sqrt(nn[0]);
  const int R = st->restart;
  double* Hc = H + (size_t)j * (R + 1);  // column j, column-major (R+1) x R
  for (int i = 0; i <= j; ++i) Hc[i] = hbuf[i] + hbuf[kLd + i];
  Hc[j + 1] = nrm;
  scale[j + 1] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
  for (int i = 0; i < j; ++i) {
    const double a = Hc[i], b = Hc[i + 1];
    Hc[i] = cs[i] * a + sn[i] * b;
    Hc[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = Hc[j], b = Hc[j + 1];
  const double rr = sqrt(a * a + b * b);
  const double c = (rr > 0.0) ? a / rr : 1.0, sv = (rr > 0.0) ? b / rr : 0.0;
  cs[j] = c;
  sn[j] = sv;
  Hc[j] = rr;
  Hc[j + 1] = 0.0;
  gvec[j + 1] = -sv * gvec[j];
  gvec[j] = c * gvec[j];
  st->res = fabs(gvec[j + 1]);
  st->j = j + 1;
  if (st->res <= st->tol || j + 1 >= R || !(nrm > 0.0) || !isfinite(st->res)) st->active = 0;
}

// y_i = scale_i * (H^{-1} g)_i for the completed iterations (upper
// triangular; scale null: y_i = (H^{-1} g)_i, the coefficients of the
// flexible basis), by column-oriented back substitution in one wavefront:
// step l divides y_l, then every lane i < l subtracts H[i][l] y_l (column l
// of the column-major H is contiguous, so the reads coalesce).
__global__ void __launch_bounds__(64) k_gm_solve_small(const GmresState* __restrict__ st,
                                                       const double* __restrict__ H,
                                                       const double* __restrict__ gvec,
                                                       const double* __restrict__ scale,
                                                       double* __restrict__ coef) {
  __shared__ double y[130];
  const int k = st->j, R = st->restart;
  const int t = threadIdx.x;
  for (int i = t; i < k; i += 64) y[i] = gvec[i];
  __syncthreads();
  for (int l = k - 1; l >= 0; --l) {
    const double* Hl = H + (size_t)l * (R + 1);
    const double yl = y[l] / Hl[l];
    __syncthreads();
    for (int i = t; i < l; i += 64) y[i] -= Hl[i] * yl;
    if (t == 0) y[l] = yl;
    __syncthreads();
  }
  for (int i = t; i < k; i += 64) coef[i] = scale ? y[i] * scale[i] : y[i];
  if (t == 0) coef[128] = (double)k;
}

// out = sum_{i<k} coef_i Vt_i
__global__ void k_gm_combine(long long n, const double* __restrict__ Vt, long long stride,
                             const double* __restrict__ coef, double* __restrict__ out) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int k = (int)coef[128];
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += coef[i] * Vt[(long long)i * stride + r];
  out[r] = acc;
}

// z += dz; r = b - Acal^T z is formed by k_bsr_spmv into r then k_residual.
__global__ void k_axpy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] += a * x[r];
}

// r = b - r (r holds Acal^T x on entry), v0 = r when given; partial |r|^2
// per block to P[b] (contiguous).
__global__ void __launch_bounds__(256) k_residual(long long n, const double* __restrict__ b,
                                                  double* __restrict__ r, double* __restrict__ v0,
                                                  double* __restrict__ P) {
  __shared__ double lds[32];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = b[i] - r[i];
    r[i] = v;
    if (v0) v0[i] = v;
    acc += v * v;
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) P[blockIdx.x] = acc;
}

// One block: |r| -> rnorm, res; j = 0; active = (|r| > tol); when scale is
// given (GMRES restart) also scale[0] = 1/|r| and g = (|r|, 0, ...).
__global__ void __launch_bounds__(256) k_residual_finish(const double* __restrict__ P, int nb,
                                                         GmresState* __restrict__ st,
                                                         double* __restrict__ scale,
                                                         double* __restrict__ gvec) {
  __shared__ double nn[1];
  __shared__ double tmp[256];
  sum_partials(P, nb, 1, 1, nn, tmp);
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(nn[0]);
  st->rnorm = nrm;
  st->res = nrm;
  st->j = 0;
  st->active = (nrm > st->tol) ? 1 : 0;
  if (scale) {
    scale[0] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
    gvec[0] = nrm;
  }
}

// Preconditioned conjugate gradients for the symmetric case (no frictional
// contact, or mu = 0: Acal^T is symmetric positive definite and so is the
// Woodbury preconditioner).  Device scalars sc = {rz, -, beta, -}; the
// GmresState carries the iteration count (j), the active flag, the
// absolute tolerance, the iteration limit (restart) and the residual norm
// of the recurrence (res).  Per iteration:
//   k_bsr_dots (w = Acal^T p, partials p.w) -> k_pcg_xr (alpha from the
//   partials, x += alpha p, r -= alpha w, partials |r|^2) -> preconditioner
//   (z = P r) -> k_dot_partials (r.z) -> k_pcg_scalar (one block: beta,
//   rz, res, j, active) -> k_pcg_p (p = z + beta p).

__global__ void __launch_bounds__(256) k_pcg_xr(long long n, double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ w,
                                                const double* __restrict__ Ppw, int nbpw,
                                                const GmresState* __restrict__ st,
                                                const double* __restrict__ sc, double* __restrict__ Prr) {
  if (st->active == 0) return;
  __shared__ double pw[1];
  __shared__ double tmp[256];
  sum_partials(Ppw, nbpw, kLd, 1, pw, tmp);
  const double alpha = (pw[0] > 0.0 && isfinite(pw[0])) ? sc[0] / pw[0] : 0.0;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double v = r[i] - alpha * w[i];
    r[i] = v;
    acc += v * v;
  }
  acc = block_sum(acc, tmp);
  if (threadIdx.x == 0) Prr[blockIdx.x] = acc;
}

// partial a . b per block to P[b] (gated by the state)
__global__ void __launch_bounds__(256) k_dot_partials(long long n, const double* __restrict__ a,
                                                      const double* __restrict__ b,
                                                      const GmresState* __restrict__ st, double* __restrict__ P) {
  if (st->active == 0) return;
  __shared__ double lds[32];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc += a[i] * b[i];
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) P[blockIdx.x] = acc;
}

// One block.  first = 1: rz = r.z, beta = 0 (start of a pass).  Otherwise:
// beta = (r.z) / rz, rz = r.z, res = |r|, j += 1, and the pass stops when
// res <= tol, j reaches the limit, p.w <= 0 (breakdown) or a value is not
// finite.
__global__ void __launch_bounds__(256) k_pcg_scalar(GmresState* __restrict__ st, const double* __restrict__ Prz,
                                                    int nbrz, const double* __restrict__ Prr, int nbrr,
                                                    const double* __restrict__ Ppw, int nbpw,
                                                    double* __restrict__ sc, int first) {
  if (st->active == 0) return;
  __shared__ double v[3];
  __shared__ double tmp[256];
  sum_partials(Prz, nbrz, 1, 1, v, tmp);
  if (!first) {
    sum_partials(Prr, nbrr, 1, 1, v + 1, tmp);
    sum_partials(Ppw, nbpw, kLd, 1, v + 2, tmp);
  }
  if (threadIdx.x != 0) return;
  const double rz = v[0];
  if (first) {
    sc[2] = 0.0;
    sc[0] = rz;
    if (!isfinite(rz)) st->active = 0;
    return;
  }
  const double res = sqrt(v[1]);
  sc[2] = rz / sc[0];
  sc[0] = rz;
  st->res = res;
  st->j += 1;
  if (res <= st->tol || st->j >= st->restart || !(v[2] > 0.0) || !isfinite(res) || !isfinite(rz))
    st->active = 0;
}

__global__ void k_pcg_p(long long n, const double* __restrict__ z, double* __restrict__ p,
                        const GmresState* __restrict__ st, const double* __restrict__ sc) {
  if (st->active == 0) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = z[i] + sc[2] * p[i];
}

// host-side launchers ------------------------------------------------------

void launch_spmv_csr3(hipStream_t s, int nrows, const long long* rp, const int* cj, const double* cx,
                      const double* xbase, long long stride, const double* scale,
                      const GmresState* st, double* y) {
  // the basis vector is addressed through the state only when both are given
  const int use_j = (st != nullptr && scale != nullptr) ? 1 : 0;
  k_spmv_csr3<<<(nrows + 3) / 4, 256, 0, s>>>(nrows, rp, cj, cx, xbase, stride, scale, st, use_j, y);
}

template <class MT>
static void spmv_tasks_impl(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                            const MT* cx, const double* xbase, long long stride, const double* scale,
                            const GmresState* st, double* y) {
  const int use_j = (st != nullptr && scale != nullptr) ? 1 : 0;
  k_spmv_tasks<MT><<<ntasks, 256, 0, s>>>(tasks, rp, cj, cx, xbase, stride, scale, st, use_j, y);
}
void launch_spmv_tasks(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                       const double* cx, const double* xbase, long long stride, const double* scale,
                       const GmresState* st, double* y) {
  spmv_tasks_impl(s, ntasks, tasks, rp, cj, cx, xbase, stride, scale, st, y);
}
void launch_spmv_tasks(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                       const float* cx, const double* xbase, long long stride, const double* scale,
                       const GmresState* st, double* y) {
  spmv_tasks_impl(s, ntasks, tasks, rp, cj, cx, xbase, stride, scale, st, y);
}
// y[row] += alpha * (row . x) over the listed rows (FP64)
void launch_spmv_tasks_acc(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                           const double* cx, const double* x, double alpha, const GmresState* st, double* y) {
  if (ntasks <= 0) return;
  k_spmv_tasks<double, true><<<ntasks, 256, 0, s>>>(tasks, rp, cj, cx, x, 0, nullptr, st, 0, y, alpha);
}
void launch_spmv_tasks_acc(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                           const float* cx, const double* x, double alpha, const GmresState* st, double* y) {
  if (ntasks <= 0) return;
  k_spmv_tasks<float, true><<<ntasks, 256, 0, s>>>(tasks, rp, cj, cx, x, 0, nullptr, st, 0, y, alpha);
}

// r = b - Acal^T x with every product and sum carried as an unevaluated
// pair (error-free product by FMA, two-sum; compensated dot product), rounded
// once at the end, one thread per DOF.  The residual of the FP64 refinement:
// FP64 Krylov solves stagnate near a relative residual of 1e-10 on stiff
// contacts, and only a residual resolved below that lets the refinement
// reach the solution to working accuracy.  Contraction is off so that the
// error terms are formed exactly as written.
__global__ void k_bsr_residual_dd(int nv, const int* __restrict__ rowptr, const int* __restrict__ col,
                                  const double* __restrict__ val, const double* __restrict__ x,
                                  const double* __restrict__ b, double* __restrict__ r) {
#pragma clang fp contract(off)
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * nv) return;
  const int row = e / 3, c = e - 3 * row;
  double hi = b[e], lo = 0.0;
  for (int p = rowptr[row]; p < rowptr[row + 1]; ++p) {
    const double* blk = val + 9 * (size_t)p + 3 * c;
    const double* xj = x + 3 * (size_t)col[p];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double prod = -blk[k] * xj[k];
      const double perr = __builtin_fma(-blk[k], xj[k], -prod);  // -blk x = prod + perr exactly
      const double s = hi + prod;
      const double bb = s - hi;
      const double serr = (hi - (s - bb)) + (prod - bb);  // hi + prod = s + serr exactly
      hi = s;
      lo += serr + perr;
    }
  }
  r[e] = hi + lo;
}

void launch_bsr_residual_dd(hipStream_t s, int nv, const int* rowptr, const int* col, const double* val,
                            const double* x, const double* b, double* r) {
  k_bsr_residual_dd<<<(3 * nv + 255) / 256, 256, 0, s>>>(nv, rowptr, col, val, x, b, r);
}

// Permutation into and out of the elimination order of the sweeps:
// t[i] = sc x[perm[i]] (x the current basis vector and sc its scale when
// use_j), and out[perm[i]] = z[i]; three components per entry.
__global__ void k_perm_gather(int n, const int* __restrict__ perm, const double* __restrict__ xbase,
                              long long stride, const double* __restrict__ scale,
                              const GmresState* __restrict__ st, int use_j, double* __restrict__ t) {
  if (gm_inactive(st)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  const double* x = xbase;
  double sc = 1.0;
  if (use_j) {
    x = xbase + (long long)st->j * stride;
    sc = scale[st->j];
  }
  const int i = e / 3, c = e - 3 * i;
  t[e] = sc * x[3 * perm[i] + c];
}

__global__ void k_perm_scatter(int n, const int* __restrict__ perm, const double* __restrict__ z,
                               const GmresState* __restrict__ st, double* __restrict__ out) {
  if (gm_inactive(st)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  const int i = e / 3, c = e - 3 * i;
  out[3 * perm[i] + c] = z[e];
}

void launch_perm_gather(hipStream_t s, int n, const int* perm, const double* xbase, long long stride,
                        const double* scale, const GmresState* st, double* t) {
  const int use_j = (st != nullptr && scale != nullptr) ? 1 : 0;
  k_perm_gather<<<(3 * n + 255) / 256, 256, 0, s>>>(n, perm, xbase, stride, scale, st, use_j, t);
}
void launch_perm_scatter(hipStream_t s, int n, const int* perm, const double* z, const GmresState* st,
                         double* out) {
  k_perm_scatter<<<(3 * n + 255) / 256, 256, 0, s>>>(n, perm, z, st, out);
}

void launch_block_jacobi(hipStream_t s, int nv, const int* diag_slot, const double* val, const double* x,
                         long long stride, const double* scale, const GmresState* st, int point, double* y) {
  const int use_j = (st != nullptr && scale != nullptr) ? 1 : 0;
  k_block_jacobi<double><<<(nv + 255) / 256, 256, 0, s>>>(nv, diag_slot, val, x, stride, scale, st, use_j, point,
                                                          y);
}
void launch_block_jacobi(hipStream_t s, int nv, const int* diag_slot, const float* val, const double* x,
                         long long stride, const double* scale, const GmresState* st, int point, double* y) {
  const int use_j = (st != nullptr && scale != nullptr) ? 1 : 0;
  k_block_jacobi<float><<<(nv + 255) / 256, 256, 0, s>>>(nv, diag_slot, val, x, stride, scale, st, use_j, point,
                                                         y);
}
template <class MT>
static void wb_gather_impl(hipStream_t s, int m, int mp, const int* row_c, const int* row_i, const int* vid,
                           const double* Q, const MT* X, const double* u, const GmresState* st, double* t) {
  if (m == 0) return;
  const int rows = wb_rows_per_block(m);
  k_wb_gather<MT><<<(m + rows - 1) / rows, 256, (size_t)m * sizeof(double), s>>>(m, mp, rows, row_c, row_i, vid, Q, X,
                                                                               u, st, t);
}
void launch_wb_gather(hipStream_t s, int m, int mp, const int* row_c, const int* row_i, const int* vid,
                      const double* Q, const double* X, const double* u, const GmresState* st, double* t) {
  wb_gather_impl(s, m, mp, row_c, row_i, vid, Q, X, u, st, t);
}
template <class MT>
static void wb_correct_impl(hipStream_t s, int nv, int ncv, const int* cv_ptr, const int* c_row0,
                            const int* c_nrow, const double* Q, const double* t, const MT* Z, double h2,
                            const double* u, const GmresState* st, double* y) {
  const int rows = wb_rows_per_block(nv);
  k_wb_correct<MT><<<(nv + rows - 1) / rows, 256, (size_t)3 * ncv * sizeof(double), s>>>(nv, ncv, rows, cv_ptr,
                                                                                        c_row0, c_nrow, Q, t, Z, h2,
                                                                                        u, st, y);
}
// t = Hq u (the capacitance right-hand side of the Woodbury correction; the
// block-LU path solves with the factors afterwards).  One thread per row.
__global__ void k_wb_hq(int m, const int* __restrict__ row_c, const int* __restrict__ row_i,
                        const int* __restrict__ vid, const double* __restrict__ Q, const double* __restrict__ u,
                        const GmresState* __restrict__ st, double* __restrict__ t) {
  if (gm_inactive(st)) return;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const int c = row_c[r];
  const double* q = Q + 9 * c + 3 * row_i[r];
  const int v = vid[c];
  t[r] = q[0] * u[3 * v] + q[1] * u[3 * v + 1] + q[2] * u[3 * v + 2];
}

// t_K = P_k t_K for every 128-block K (P: mp/128 blocks of 128 x 128), one
// block per K.
__global__ void __launch_bounds__(256) k_lu_diag(const double* __restrict__ Pall, const GmresState* __restrict__ st,
                                                 double* __restrict__ t) {
  if (gm_inactive(st)) return;
  __shared__ double tk[128];
  const int k0 = blockIdx.x * 128;
  if (threadIdx.x < 128) tk[threadIdx.x] = t[k0 + threadIdx.x];
  __syncthreads();
  const double* P = Pall + (size_t)blockIdx.x * 128 * 128;
  const int l = threadIdx.x & 15;
  for (int r = threadIdx.x >> 4; r < 128; r += 16) {
    const double2* f = reinterpret_cast<const double2*>(P + (size_t)r * 128);
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 a = f[l + 16 * u];
      const int c = 2 * (l + 16 * u);
      acc = fma(a.x, tk[c], acc);
      acc = fma(a.y, tk[c + 1], acc);
    }
    acc = group_sum<16>(acc);
    if (l == 0) t[k0 + r] = acc;
  }
}

// One group [c0, c1) of the grouped substitutions (group inverses inside,
// transformed blocks outside; see the factor kernels): with the group's
// entries a_G of a (read before the launch changes anything),
//   rows r of the group:  b_r = a_r + sum_c F[r][c] a_c over the group's
//                         columns strictly before (fwd) / after (bwd) r's
//                         128-block;
//   rows r outside:       a_r -= sum_{c in [c0, c1)} F[r][c] a_c,
// for rows [c0, mp) (fwd: below and in the group) or [0, c1) (bwd).  No row
// reads what another row writes.  16 lanes per row, 16 rows per block.
__global__ void __launch_bounds__(256) k_lu_gsweep(int mp, int c0, int c1, int fwd, const double* __restrict__ F,
                                                   const GmresState* __restrict__ st, double* __restrict__ a,
                                                   double* __restrict__ b) {
  if (gm_inactive(st)) return;
  __shared__ double ag[512];
  for (int c = threadIdx.x; c < c1 - c0; c += 256) ag[c] = a[c0 + c];
  __syncthreads();
  const int rbeg = fwd ? c0 : 0, rend = fwd ? mp : c1;
  const int row = rbeg + blockIdx.x * 16 + (threadIdx.x >> 4);
  const int l = threadIdx.x & 15;
  if (row >= rend) return;
  const bool in = row >= c0 && row < c1;
  const int rb = row & ~127;
  const int cb = in ? (fwd ? c0 : rb + 128) : c0, ce = in ? (fwd ? rb : c1) : c1;
  const double2* f = reinterpret_cast<const double2*>(F + (size_t)row * mp);
  double acc = 0.0;
  const int n2 = (ce - cb) / 32;  // double2 loads per lane
#pragma unroll 4
  for (int u = 0; u < n2; ++u) {
    const int c = cb + 2 * l + 32 * u;
    const double2 v = f[c >> 1];
    acc = fma(v.x, ag[c - c0], acc);
    acc = fma(v.y, ag[c - c0 + 1], acc);
  }
  acc = group_sum<16>(acc);
  if (l == 0) {
    if (in)
      b[row] = a[row] + acc;
    else
      a[row] -= acc;
  }
}

// t = X Hq u with X = C^{-1} held as the grouped block-LU factors F and the
// inverted pivot blocks P: forward substitution group by group (t -> y),
// y_K = P_k y_K, backward substitution (y -> t).  t and y have mp entries;
// rows m .. mp - 1 of t must hold zeros (C is padded with the identity).
void launch_wb_lu(hipStream_t s, int m, int mp, const int* row_c, const int* row_i, const int* vid,
                  const double* Q, const double* F, const double* P, int group, const double* u,
                  const GmresState* st, double* t, double* y) {
  k_wb_hq<<<(m + 255) / 256, 256, 0, s>>>(m, row_c, row_i, vid, Q, u, st, t);
  const int gw = 128 * group, ng = (mp + gw - 1) / gw;
  for (int G = 0; G < ng; ++G) {
    const int c0 = G * gw, c1 = c0 + gw < mp ? c0 + gw : mp;
    k_lu_gsweep<<<(mp - c0 + 15) / 16, 256, 0, s>>>(mp, c0, c1, 1, F, st, t, y);
  }
  k_lu_diag<<<mp / 128, 256, 0, s>>>(P, st, y);
  for (int G = ng - 1; G >= 0; --G) {
    const int c0 = G * gw, c1 = c0 + gw < mp ? c0 + gw : mp;
    k_lu_gsweep<<<(c1 + 15) / 16, 256, 0, s>>>(mp, c0, c1, 0, F, st, y, t);
  }
}

// Pipelined substitutions: the same forward pass, P_k step and backward
// pass in two launches instead of one launch per group.  The rows are cut
// into stripes of 16 (one block each, 16 lanes per row); a stripe computes
// the final value of each of its rows in the left-looking form
//   fwd:  a_r = t_r - sum_{c < c0(G)} F[r][c] a_c,   y_r = a_r + sum_{c0 <= c < rb} F[r][c] a_c,
//   bwd:  a_r = (P y)_r - sum_{c >= c1(G)} F[r][c] a_c,   t_r = a_r + sum_{rb+128 <= c < c1} F[r][c] a_c,
// (G the row's group [c0, c1), rb its 128-block), i.e. the group steps'
// updates gathered per row, so each row reads its own part of F once.
// Every a_r is published once, by an agent-scope atomic store, into a
// buffer whose entries start as kLuPending (a signalling-NaN pattern that
// arithmetic never produces); a stripe polls the entries it needs until
// they are no longer pending.  The value is its own flag, so no fence is
// needed.  Blocks take their stripe from a ticket counter in the order the
// dependencies run (fwd: top stripe first; bwd: bottom first), so a stripe
// only waits for stripes with smaller tickets, which blocks already running
// hold: every wait ends.  A wait still pending after kLuSpin polls (not
// possible unless the buffers were not reset) raises err[2] and stops all
// waits.  Each pass resets the other pass's buffer and ticket for the next
// launch (stream order separates them).
constexpr unsigned long long kLuPending = 0x7FF4C0DE0000A11FULL;
constexpr int kLuSpin = 1 << 18;
constexpr int kLuGW = 512;  // group width of the pipelined passes (4 blocks of 128)

// Waits until *p is no longer pending; v: a value of *p read earlier.
__device__ __forceinline__ double lu_poll(double* p, unsigned long long v, int* err) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  for (int n = 1; v == kLuPending; ++n) {
    if ((n & 1023) == 0 && (n >= kLuSpin || __hip_atomic_load(err + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
      __hip_atomic_store(err + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
    v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return __longlong_as_double((long long)v);
}

__device__ __forceinline__ unsigned long long lu_peek(const double* p) {
  return __hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lu_publish(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double lu_pending() { return __longlong_as_double((long long)kLuPending); }

// sum over the steps i < n of a[h_i .. h_i + w_i) . F[row][h_i .. h_i + w_i)
// for the 16 lanes of a row (lane l: columns h_i + 2 l + 32 u), with
// h_i = h + i dir kLuGW and w_i = min(kLuGW, mp - h_i) (a multiple of 32).
// Step i + 1's row loads and its first reads of a are issued before step
// i's products, so they are in flight while step i waits and computes.
__device__ __forceinline__ double lu_pipe_span(const double2* __restrict__ f, int n, int h, int dir, int mp, double* A,
                                               double* ag, int l, int* err) {
  double2 cur[kLuGW / 32], nxt[kLuGW / 32];
  unsigned long long pv[2];
  auto issue = [&](int i, double2 (&fv)[kLuGW / 32]) {
    const int h0 = h + i * dir * kLuGW, w = min(kLuGW, mp - h0);
#pragma unroll
    for (int u = 0; u < kLuGW / 32; ++u)
      if (32 * u < w) fv[u] = f[(h0 + 2 * l + 32 * u) >> 1];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int c = threadIdx.x + 256 * k;
      pv[k] = c < w ? lu_peek(A + h0 + c) : 0ull;
    }
  };
  double acc = 0.0;
  if (n <= 0) return acc;
  issue(0, cur);
  for (int i = 0; i < n; ++i) {
    const int h0 = h + i * dir * kLuGW, w = min(kLuGW, mp - h0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int c = threadIdx.x + 256 * k;
      if (c < w) ag[c] = lu_poll(A + h0 + c, pv[k], err);
    }
    __syncthreads();
    if (i + 1 < n) issue(i + 1, nxt);
#pragma unroll
    for (int u = 0; u < kLuGW / 32; ++u)
      if (32 * u < w) {
        acc = fma(cur[u].x, ag[2 * l + 32 * u], acc);
        acc = fma(cur[u].y, ag[2 * l + 32 * u + 1], acc);
      }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kLuGW / 32; ++u) cur[u] = nxt[u];
  }
  return acc;
}

// a[c0 .. c0 + w) . F[row][c0 .. c0 + w) in one step (w <= kLuGW, a multiple of 32)
__device__ __forceinline__ double lu_pipe_dot(const double2* __restrict__ f, int c0, int w, double* A, double* ag,
                                              int l, int* err) {
  return lu_pipe_span(f, 1, c0, 1, c0 + w, A, ag, l, err);
}

__global__ void __launch_bounds__(256, 3) k_lu_fwd_pipe(int mp, const double* __restrict__ F,
                                                     const GmresState* __restrict__ st, const double* __restrict__ t,
                                                     double* A, double* __restrict__ y, double* Anext,
                                                     unsigned* tick, int* err) {
  if (gm_inactive(st)) return;
  __shared__ double ag[kLuGW];
  __shared__ int s_sp;
  if (threadIdx.x == 0) s_sp = (int)atomicAdd(&tick[0], 1u);
  __syncthreads();
  const int sp = s_sp, r0 = 16 * sp;
  if (sp == 0 && threadIdx.x == 0) __hip_atomic_store(&tick[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int row = r0 + (threadIdx.x >> 4), l = threadIdx.x & 15;
  if (l == 0) lu_publish(Anext + row, lu_pending());
  const int c0 = (r0 / kLuGW) * kLuGW, rb = r0 & ~127;
  const double2* f = reinterpret_cast<const double2*>(F + (size_t)row * mp);
  const double acc = group_sum<16>(lu_pipe_span(f, c0 / kLuGW, 0, 1, mp, A, ag, l, err));
  const double a = t[row] - acc;
  if (l == 0) lu_publish(A + row, a);
  double acc2 = 0.0;
  if (rb > c0) acc2 = group_sum<16>(lu_pipe_dot(f, c0, rb - c0, A, ag, l, err));
  if (l == 0) y[row] = a + acc2;
}

__global__ void __launch_bounds__(256, 3) k_lu_bwd_pipe(int mp, const double* __restrict__ F,
                                                     const double* __restrict__ Pall,
                                                     const GmresState* __restrict__ st, const double* __restrict__ y,
                                                     double* A, double* __restrict__ t, double* Anext,
                                                     unsigned* tick, int* err) {
  if (gm_inactive(st)) return;
  __shared__ double ag[kLuGW];
  __shared__ int s_sp;
  if (threadIdx.x == 0) s_sp = (int)atomicAdd(&tick[1], 1u);
  __syncthreads();
  const int sp = s_sp, r0 = mp - 16 * (sp + 1);
  if (sp == 0 && threadIdx.x == 0) __hip_atomic_store(&tick[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int row = r0 + (threadIdx.x >> 4), l = threadIdx.x & 15;
  if (l == 0) lu_publish(Anext + row, lu_pending());
  const int c0 = (r0 / kLuGW) * kLuGW, c1 = min(c0 + kLuGW, mp), rb = r0 & ~127;
  // (P y)_row with the row's inverted pivot block
  const double2* pr = reinterpret_cast<const double2*>(Pall + (size_t)(rb / 128) * 128 * 128 + (size_t)(row - rb) * 128);
  double p = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double2 v = pr[l + 16 * u];
    const int c = rb + 2 * (l + 16 * u);
    p = fma(v.x, y[c], p);
    p = fma(v.y, y[c + 1], p);
  }
  p = group_sum<16>(p);
  const double2* f = reinterpret_cast<const double2*>(F + (size_t)row * mp);
  const int hlast = ((mp - 1) / kLuGW) * kLuGW;
  const double acc = group_sum<16>(lu_pipe_span(f, hlast >= c1 ? (hlast - c1) / kLuGW + 1 : 0, hlast, -1, mp, A, ag,
                                                l, err));
  const double a = p - acc;
  if (l == 0) lu_publish(A + row, a);
  double acc2 = 0.0;
  if (c1 > rb + 128) acc2 = group_sum<16>(lu_pipe_dot(f, rb + 128, c1 - rb - 128, A, ag, l, err));
  if (l == 0) t[row] = a + acc2;
}

__global__ void k_lu_pipe_init(int mp, double* __restrict__ A0, double* __restrict__ A1, unsigned* __restrict__ tick) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < mp) {
    A0[i] = lu_pending();
    A1[i] = lu_pending();
  }
  if (i < 2) tick[i] = 0u;
}

// Buffers of the pipelined passes to their starting state (both pending,
// tickets zero): once per setup; each pass then leaves the other's ready.
void launch_lu_pipe_init(hipStream_t s, int mp, double* A0, double* A1, unsigned* tick) {
  k_lu_pipe_init<<<(mp + 255) / 256, 256, 0, s>>>(mp, A0, A1, tick);
}

// The pipelined form of launch_wb_lu (group of four 128-blocks): A0, A1 hold
// mp doubles each, tick two counters, err[2] the wait flag.
void launch_wb_lu_pipe(hipStream_t s, int m, int mp, const int* row_c, const int* row_i, const int* vid,
                       const double* Q, const double* F, const double* P, const double* u, const GmresState* st,
                       double* t, double* y, double* A0, double* A1, unsigned* tick, int* err) {
  k_wb_hq<<<(m + 255) / 256, 256, 0, s>>>(m, row_c, row_i, vid, Q, u, st, t);
  k_lu_fwd_pipe<<<mp / 16, 256, 0, s>>>(mp, F, st, t, A0, y, A1, tick, err);
  k_lu_bwd_pipe<<<mp / 16, 256, 0, s>>>(mp, F, P, st, y, A1, t, A0, tick, err);
}

// w[cv_a] = sum over the contacts c at contact vertex a of Q_c^T t_c (H^T t
// in world coordinates; w is zero elsewhere).  One thread per contact vertex.
__global__ void k_scatter_ht(int ncv, const int* __restrict__ cv, const int* __restrict__ cv_ptr,
                             const int* __restrict__ c_row0, const int* __restrict__ c_nrow,
                             const double* __restrict__ Q, const double* __restrict__ t,
                             const GmresState* __restrict__ st, double* __restrict__ w) {
  if (gm_inactive(st)) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ncv) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int c = cv_ptr[a]; c < cv_ptr[a + 1]; ++c)
    for (int i = 0; i < c_nrow[c]; ++i) {
      const double tv = t[c_row0[c] + i];
      const double* q = Q + 9 * c + 3 * i;
      s0 += q[0] * tv;
      s1 += q[1] * tv;
      s2 += q[2] * tv;
    }
  const int v = cv[a];
  w[3 * v] = s0;
  w[3 * v + 1] = s1;
  w[3 * v + 2] = s2;
}

void launch_scatter_ht(hipStream_t s, int ncv, const int* cv, const int* cv_ptr, const int* c_row0,
                       const int* c_nrow, const double* Q, const double* t, const GmresState* st, double* w) {
  if (ncv <= 0) return;
  k_scatter_ht<<<(ncv + 255) / 256, 256, 0, s>>>(ncv, cv, cv_ptr, c_row0, c_nrow, Q, t, st, w);
}

void launch_wb_correct(hipStream_t s, int nv, int ncv, const int* cv_ptr, const int* c_row0, const int* c_nrow,
                       const double* Q, const double* t, const double* Z, double h2, const double* u,
                       const GmresState* st, double* y) {
  wb_correct_impl(s, nv, ncv, cv_ptr, c_row0, c_nrow, Q, t, Z, h2, u, st, y);
}
template <class MT>
static void bsr_impl(hipStream_t s, int lanes, int nv, const int* rowptr, const int* col, const MT* val,
                     const double* val64, long long soa, const double* x, double* outbase, long long stride,
                     const GmresState* st) {
  const int rows = 256 / lanes;
  const unsigned g = (unsigned)((nv + rows - 1) / rows);
  switch (lanes) {
    case 4: k_bsr_spmv<MT, 4><<<g, 256, 0, s>>>(nv, rowptr, col, val, val64, soa, x, outbase, stride, st); break;
    case 8: k_bsr_spmv<MT, 8><<<g, 256, 0, s>>>(nv, rowptr, col, val, val64, soa, x, outbase, stride, st); break;
    case 32: k_bsr_spmv<MT, 32><<<g, 256, 0, s>>>(nv, rowptr, col, val, val64, soa, x, outbase, stride, st); break;
    default: k_bsr_spmv<MT, 16><<<g, 256, 0, s>>>(nv, rowptr, col, val, val64, soa, x, outbase, stride, st); break;
  }
}
// soa: 0 for block-major values (val[9 p + k]), else the number of blocks
// of the entry-major copy (val[k soa + p])
void launch_bsr_spmv(hipStream_t s, int lanes, int nv, const int* rowptr, const int* col, const double* val,
                     long long soa, const double* x, double* outbase, long long stride, const GmresState* st) {
  bsr_impl(s, lanes, nv, rowptr, col, val, (const double*)nullptr, soa, x, outbase, stride, st);
}
// FP32 block values with the diagonal blocks from val64 (see block_madd)
void launch_bsr_spmv(hipStream_t s, int lanes, int nv, const int* rowptr, const int* col, const float* val,
                     const double* val64, long long soa, const double* x, double* outbase, long long stride,
                     const GmresState* st) {
  bsr_impl(s, lanes, nv, rowptr, col, val, val64, soa, x, outbase, stride, st);
}

// Entry-major copies of the block values (the Krylov products' layout):
// soa[k nnzb + p] = aos[9 p + k], and the same rounded to FP32 into soa32
// when it is given.  A block transposes 256 consecutive blocks through LDS:
// it reads their 2304 contiguous values and writes nine contiguous runs of
// 256, so both sides coalesce.
__global__ void __launch_bounds__(256) k_bsr_soa(long long nnzb, const double* __restrict__ aos,
                                                 double* __restrict__ soa, float* __restrict__ soa32) {
  __shared__ double tile[9 * 256];
  const long long p0 = (long long)blockIdx.x * 256;
  const int nloc = (int)min(256LL, nnzb - p0);
  const double* src = aos + 9 * p0;
  for (int i = threadIdx.x; i < 9 * nloc; i += 256) tile[i] = src[i];
  __syncthreads();
  if ((int)threadIdx.x >= nloc) return;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double v = tile[9 * threadIdx.x + k];
    soa[k * nnzb + p0 + threadIdx.x] = v;
    if (soa32) soa32[k * nnzb + p0 + threadIdx.x] = (float)v;
  }
}
void launch_bsr_soa(hipStream_t s, long long nnzb, const double* aos, double* soa, float* soa32) {
  if (nnzb <= 0) return;
  k_bsr_soa<<<(unsigned)((nnzb + 255) / 256), 256, 0, s>>>(nnzb, aos, soa, soa32);
}

__global__ void k_to_f32(long long n, const double* __restrict__ a, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)a[i];
}
void launch_to_f32(hipStream_t s, long long n, const double* a, float* out) {
  if (n <= 0) return;
  k_to_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, a, out);
}

// Partial sums of many blocks folded once: entry i (i <= j + extra, j the
// current basis index) of P[b * ld + i] summed over the nb blocks in fixed
// order into P[i] (block row 0), one 256-thread block per entry.  The
// consumers then read one partial instead of re-adding nb of them in each of
// their own blocks, which costs nb x (j + 1) loads per block on large scenes.
__global__ void __launch_bounds__(256) k_fold_partials(double* __restrict__ P, int nb, int ld,
                                                       const GmresState* __restrict__ st, int extra) {
  if (st->active == 0) return;
  const int i = blockIdx.x;
  if (i > st->j + extra) return;
  __shared__ double tmp[256];
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) a += P[(size_t)b * ld + i];
  a = block_sum(a, tmp);
  if (threadIdx.x == 0) P[i] = a;
}

void launch_fold_partials(hipStream_t s, double* P, int nb, const GmresState* st, int extra) {
  k_fold_partials<<<kLd, 256, 0, s>>>(P, nb, kLd, st, extra);
}

int gm_blocks(long long n, int rpb) { return (int)((n + rpb - 1) / rpb); }
int bsr_blocks(int nv, int lanes) { return (nv + 256 / lanes - 1) / (256 / lanes); }

template <class MT>
static void bsr_dots_impl(hipStream_t s, int lanes, int nv, const int* rowptr, const int* col, const MT* val,
                          const double* val64, long long soa, const double* y, double* Vt, long long stride,
                          const GmresState* st, int jfix, double* P, double* Zb) {
  const unsigned g = (unsigned)bsr_blocks(nv, lanes);
  switch (lanes) {
    case 4: k_bsr_dots<MT, 4><<<g, 256, 0, s>>>(nv, rowptr, col, val, val64, soa, y, Vt, stride, st, jfix, P, Zb); break;
    case 8: k_bsr_dots<MT, 8><<<g, 256, 0, s>>>(nv, rowptr, col, val, val64, soa, y, Vt, stride, st, jfix, P, Zb); break;
    case 32: k_bsr_dots<MT, 32><<<g, 256, 0, s>>>(nv, rowptr, col, val, val64, soa, y, Vt, stride, st, jfix, P, Zb); break;
    default: k_bsr_dots<MT, 16><<<g, 256, 0, s>>>(nv, rowptr, col, val, val64, soa, y, Vt, stride, st, jfix, P, Zb); break;
  }
}
void launch_bsr_dots(hipStream_t s, int lanes, int nv, const int* rowptr, const int* col, const double* val,
                     long long soa, const double* y, double* Vt, long long stride, const GmresState* st, int jfix,
                     double* P, double* Zb) {
  bsr_dots_impl(s, lanes, nv, rowptr, col, val, (const double*)nullptr, soa, y, Vt, stride, st, jfix, P, Zb);
}
void launch_bsr_dots(hipStream_t s, int lanes, int nv, const int* rowptr, const int* col, const float* val,
                     const double* val64, long long soa, const double* y, double* Vt, long long stride,
                     const GmresState* st, int jfix, double* P, double* Zb) {
  bsr_dots_impl(s, lanes, nv, rowptr, col, val, val64, soa, y, Vt, stride, st, jfix, P, Zb);
}

void launch_gm_update(hipStream_t s, long long n, int rpb, double* Vt, long long stride, const double* scale,
                      const GmresState* st, const double* Pin, int nbin, double* Pout, double* hbuf, int mode) {
  k_gm_update<<<gm_blocks(n, rpb), 256, 0, s>>>(n, rpb, Vt, stride, scale, st, Pin, nbin, Pout, hbuf, mode);
}

void launch_gm_givens(hipStream_t s, GmresState* st, const double* P, int nb, double* scale, const double* hbuf,
                      double* H, double* cs, double* sn, double* gvec) {
  k_gm_givens<<<1, 256, 0, s>>>(st, P, nb, scale, hbuf, H, cs, sn, gvec);
}

void launch_gm_finish(hipStream_t s, long long n, const GmresState* st, const double* H,
                      const double* gvec, const double* scale, const double* Vt, long long stride,
                      double* coef, double* out) {
  k_gm_solve_small<<<1, 64, 0, s>>>(st, H, gvec, scale, coef);
  k_gm_combine<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, Vt, stride, coef, out);
}

void launch_axpy(hipStream_t s, long long n, double a, const double* x, double* y) {
  k_axpy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, a, x, y);
}

int vec_blocks(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < 512 ? b : 512);
}

// r = b - r, v0 = r (when given), |r| into the state (and the GMRES start
// vector scale and g when scale is given)
void launch_residual(hipStream_t s, long long n, const double* b, double* r, double* v0, double* P,
                     GmresState* st, double* scale, double* gvec) {
  const int nb = vec_blocks(n);
  k_residual<<<nb, 256, 0, s>>>(n, b, r, v0, P);
  k_residual_finish<<<1, 256, 0, s>>>(P, nb, st, scale, gvec);
}

void launch_pcg_xr(hipStream_t s, long long n, double* x, double* r, const double* p, const double* w,
                   const double* Ppw, int nbpw, const GmresState* st, const double* sc, double* Prr) {
  k_pcg_xr<<<vec_blocks(n), 256, 0, s>>>(n, x, r, p, w, Ppw, nbpw, st, sc, Prr);
}
void launch_dot_partials(hipStream_t s, long long n, const double* a, const double* b, const GmresState* st,
                         double* P) {
  k_dot_partials<<<vec_blocks(n), 256, 0, s>>>(n, a, b, st, P);
}
void launch_pcg_scalar(hipStream_t s, GmresState* st, const double* Prz, int nbrz, const double* Prr, int nbrr,
                       const double* Ppw, int nbpw, double* sc, int first) {
  k_pcg_scalar<<<1, 256, 0, s>>>(st, Prz, nbrz, Prr, nbrr, Ppw, nbpw, sc, first);
}
void launch_pcg_p(hipStream_t s, long long n, const double* z, double* p, const GmresState* st,
                  const double* sc) {
  k_pcg_p<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, z, p, st, sc);
}

}  // namespace adj
