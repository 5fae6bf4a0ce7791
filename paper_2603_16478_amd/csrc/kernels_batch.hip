// Batched adjoint solves: many independent scenes in one launch per phase.
//
// The scenes are packed into one disjoint union (vertices, tets and
// contacts of scene s are contiguous, in scene order), so every per-tet,
// per-contact and sparse-matrix kernel of the single-scene path runs over
// all scenes at once: A, S and Acal^T are block diagonal.  What is per
// scene is dense or scalar: the Delassus matrix D_s, the Woodbury factors
// Z_s and X_s (packed with per-scene offsets), and the Krylov state (one
// GMRES per scene, Sec. 5.4).  Kernels of those parts walk tables whose
// blocks never straddle two scenes; a scene whose cycle has stopped has its
// blocks return at once (per-scene convergence mask).
//
// Tables are int4 {scene, begin, end, first}: rows [begin, end) of one
// scene, `first` = 1 for the first block of the scene in the table.  Per
// scene, rng[s] = [first block, end block) of a table, so consumers of the
// per-block partials sum exactly the blocks of their scene.
#include "device_common.h"
#include "krylov_state.h"

#include <algorithm>

namespace adj {

constexpr int kBLd = 130;  // partials per block (basis index i)

// ---------------------------------------------------------------------------
// Sparse-inverse products over the union: y = S x with x the scene's current
// basis vector Vt_{j_s} * scale_s[j_s] (use_j) or x = xbase; rows of stopped
// scenes are skipped.  rscene: scene of each row (the rows of S are in
// elimination order, those of S^T in vertex order).  ACC: y[row] += alpha
// (row . x) instead (the first phase of a sweep level).
template <class MT, bool ACC = false>
__global__ void __launch_bounds__(256) kb_spmv_tasks(const int4* __restrict__ tasks,
                                                     const long long* __restrict__ rp,
                                                     const int* __restrict__ cj, const MT* __restrict__ cx,
                                                     const double* __restrict__ xbase, long long stride,
                                                     const double* __restrict__ scale, int lds_scale,
                                                     const GmresState* __restrict__ st,
                                                     const int* __restrict__ rscene, int use_j,
                                                     double* __restrict__ y, double alpha = 0.0) {
  __shared__ double lds[32];
  const int4 t = tasks[blockIdx.x];
  constexpr int kBig = 0x40000000;
  if (t.x >= 0 && (t.x & kBig)) {
    const int row = t.x & ~kBig;
    const int s = rscene[row];
    if (st[s].active == 0) return;
    const double* x = xbase + (use_j ? (long long)st[s].j * stride : 0);
    const double sc = use_j ? scale[(size_t)s * lds_scale + st[s].j] : 1.0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
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
  const int s = rscene[row];
  if (st[s].active == 0) return;
  const double* x = xbase + (use_j ? (long long)st[s].j * stride : 0);
  const double sc = use_j ? scale[(size_t)s * lds_scale + st[s].j] : 1.0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
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

// Permutations of the sweeps over the union (elimination position i of the
// scene pscene[i] holds vertex perm[i]); entries of stopped scenes are left
// as they are.  Gather: t = scale_s x (x the scene's current basis vector
// with use_j, else xbase); scatter: out = z back in vertex order.
__global__ void kb_perm_gather(int n, const int* __restrict__ perm, const int* __restrict__ pscene,
                               const double* __restrict__ xbase, long long stride, const double* __restrict__ scale,
                               int lds_scale, const GmresState* __restrict__ st, int use_j, double* __restrict__ t) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  const int i = e / 3, c = e - 3 * i;
  const int s = pscene[i];
  if (st[s].active == 0) return;
  const double* x = xbase + (use_j ? (long long)st[s].j * stride : 0);
  const double sc = use_j ? scale[(size_t)s * lds_scale + st[s].j] : 1.0;
  t[e] = sc * x[3 * perm[i] + c];
}

__global__ void kb_perm_scatter(int n, const int* __restrict__ perm, const int* __restrict__ pscene,
                                const double* __restrict__ z, const GmresState* __restrict__ st,
                                double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  const int i = e / 3, c = e - 3 * i;
  if (st[pscene[i]].active == 0) return;
  out[3 * perm[i] + c] = z[e];
}

// ---------------------------------------------------------------------------
// Woodbury correction, per scene.
// t = X_s (Hq u) on the capacitance rows of one scene (table over union
// capacitance rows, 4 rows per block, one wavefront per row); g = Hq u for
// all m_s rows of the scene is staged in LDS first.
__global__ void __launch_bounds__(256) kb_wb_gather(const int4* __restrict__ tab, const int* __restrict__ moff,
                                                    const long long* __restrict__ xpos,
                                                    const int* __restrict__ mps, const int* __restrict__ row_c,
                                                    const int* __restrict__ row_i, const int* __restrict__ vid,
                                                    const double* __restrict__ Q, const double* __restrict__ Xb,
                                                    const double* __restrict__ u,
                                                    const GmresState* __restrict__ st, double* __restrict__ t) {
  extern __shared__ double g[];
  const int4 e = tab[blockIdx.x];
  const int s = e.x;
  if (st[s].active == 0) return;
  const int r0 = moff[s], m = moff[s + 1] - r0;
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    const int c = row_c[r0 + r];
    const double* q = Q + 9 * c + 3 * row_i[r0 + r];
    const int v = vid[c];
    g[r] = q[0] * u[3 * v] + q[1] * u[3 * v + 1] + q[2] * u[3 * v + 2];
  }
  __syncthreads();
  // union capacitance rows e.y .. e.z - 1
  wb_gather_rows(e.y, e.z, m, Xb + xpos[s] + (size_t)(e.y - r0) * mps[s], mps[s], g, t);
}

// y = u - h^2 Z_s t' on the vertex rows of one scene (4 per block, one
// wavefront per vertex); t'_a = sum over the contacts at contact vertex a of
// Q_c^T t_c, for the scene's contact vertices, staged in LDS.  Scenes
// without contacts copy u.
__global__ void __launch_bounds__(256) kb_wb_correct(const int4* __restrict__ tab, const int* __restrict__ voff,
                                                     const int* __restrict__ cvoff, const int* __restrict__ cv_ptr,
                                                     const int* __restrict__ c_row0, const int* __restrict__ c_nrow,
                                                     const double* __restrict__ Q, const double* __restrict__ t,
                                                     const double* __restrict__ Zb, const long long* __restrict__ yoff,
                                                     double h2, const double* __restrict__ u,
                                                     const GmresState* __restrict__ st, double* __restrict__ y) {
  extern __shared__ double tp[];
  const int4 e = tab[blockIdx.x];
  const int s = e.x;
  if (st[s].active == 0) return;
  const int a0 = cvoff[s], ncv = cvoff[s + 1] - a0;
  for (int a = threadIdx.x; a < ncv; a += blockDim.x) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int c = cv_ptr[a0 + a]; c < cv_ptr[a0 + a + 1]; ++c)
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
  const double* Zr = Zb + yoff[s] + (size_t)(e.y - voff[s]) * ncv;
  wb_rows(e.y, e.z, ncv, Zr, tp, h2, u, y);
}

// ---------------------------------------------------------------------------
// Krylov kernels of the batch (per-scene GMRES, lockstep cycles).

// w = Acal^T y on the vertex rows of one scene (LANES lanes per row), fused
// with the first Gram-Schmidt dots Vt_i . w (i <= j_s) over the block's rows.
template <class MT, int LANES>
__global__ void __launch_bounds__(256) kb_bsr_dots(const int4* __restrict__ tab, const int* __restrict__ rowptr,
                                                   const int* __restrict__ col, const MT* __restrict__ val,
                                                   const double* __restrict__ val64,
                                                   const double* __restrict__ y, double* __restrict__ Vt,
                                                   long long stride, const GmresState* __restrict__ st,
                                                   double* __restrict__ P) {
  constexpr int R = 256 / LANES;
  __shared__ double wl[3 * R];
  const int4 e = tab[blockIdx.x];
  const int s = e.x;
  if (st[s].active == 0) return;
  const int j = st[s].j;
  double* w = Vt + (long long)(j + 1) * stride;
  const int sub = threadIdx.x & (LANES - 1), rl = threadIdx.x / LANES;
  const int row = e.y + rl;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (row < e.z) {
    for (int p = rowptr[row] + sub; p < rowptr[row + 1]; p += LANES) {
      const int c = col[p];
      const double x0 = y[3 * c], x1 = y[3 * c + 1], x2 = y[3 * c + 2];
      block_madd<MT>(val, val64, (size_t)p, c == row, x0, x1, x2, a0, a1, a2);
    }
  }
  a0 = group_sum<LANES>(a0);
  a1 = group_sum<LANES>(a1);
  a2 = group_sum<LANES>(a2);
  if (sub == 0) {
    const bool ok = row < e.z;
    wl[3 * rl] = ok ? a0 : 0.0;
    wl[3 * rl + 1] = ok ? a1 : 0.0;
    wl[3 * rl + 2] = ok ? a2 : 0.0;
    if (ok) {
      w[3 * row] = a0;
      w[3 * row + 1] = a1;
      w[3 * row + 2] = a2;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
  const long long e0 = 3LL * e.y;
  const int ne = 3 * (e.z - e.y);
  for (int i = wid; i <= j; i += 4) {
    const double* vi = Vt + (long long)i * stride + e0;
    double d = 0.0;
    for (int k = lane; k < ne; k += 64) d += vi[k] * wl[k];
    d = wave_sum(d);
    if (lane == 0) P[(size_t)blockIdx.x * kBLd + i] = d;
  }
}

// Gram-Schmidt update on the DOF rows [begin, end) of one scene (T = 256 /
// rows-per-block threads per row): c_i = scale_i^2 * (sum of the scene's
// partials Pin), w -= sum_i c_i Vt_i; the scene's first block records
// h_i = scale_i * sum in hbuf_s[hoff + i].  mode 0: partial dots of the new
// w; mode 1: partial |w|^2.
__global__ void __launch_bounds__(256) kb_gm_update(const int4* __restrict__ tab, int rpb,
                                                    const int2* __restrict__ rng_in,
                                                    const double* __restrict__ Pin, double* __restrict__ Pout,
                                                    double* __restrict__ Vt, long long stride,
                                                    const double* __restrict__ scale, int lds_scale,
                                                    const GmresState* __restrict__ st,
                                                    double* __restrict__ hbuf, int mode) {
  __shared__ double hs[kBLd];
  __shared__ double tmp[256];
  const int4 e = tab[blockIdx.x];
  const int s = e.x;
  if (st[s].active == 0) return;
  const int j = st[s].j;
  double* w = Vt + (long long)(j + 1) * stride;
  const double* sc = scale + (size_t)s * lds_scale;
  const int2 rg = rng_in[s];
  sum_partials(Pin + (size_t)rg.x * kBLd, rg.y - rg.x, kBLd, j + 1, hs, tmp);
  if (e.w)
    for (int i = threadIdx.x; i <= j; i += blockDim.x) hbuf[(size_t)s * 2 * kBLd + (mode == 0 ? 0 : kBLd) + i] = sc[i] * hs[i];
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += blockDim.x) hs[i] *= sc[i] * sc[i];
  __syncthreads();
  const int T = blockDim.x / rpb;
  const int rl = threadIdx.x % rpb, part = threadIdx.x / rpb;
  const long long r = (long long)e.y + rl;
  double acc = 0.0;
  if (r < e.z)
    for (int i = part; i <= j; i += T) acc += hs[i] * Vt[(long long)i * stride + r];
  tmp[threadIdx.x] = acc;
  __syncthreads();
  if (part == 0 && r < e.z) {
    double a = tmp[rl];
    for (int q = 1; q < T; ++q) a += tmp[rl + q * rpb];
    w[r] -= a;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64, nw = blockDim.x / 64;
  if (mode == 0) {
    for (int i = wid; i <= j; i += nw) {
      const double* vi = Vt + (long long)i * stride;
      double d = 0.0;
      for (long long rr = e.y + lane; rr < e.z; rr += 64) d += vi[rr] * w[rr];
      d = wave_sum(d);
      if (lane == 0) Pout[(size_t)blockIdx.x * kBLd + i] = d;
    }
  } else {
    double d = 0.0;
    for (long long rr = e.y + threadIdx.x; rr < e.z; rr += blockDim.x) d += w[rr] * w[rr];
    d = block_sum(d, tmp);
    if (threadIdx.x == 0) Pout[(size_t)blockIdx.x * kBLd] = d;
  }
}

// One block per scene: |w| from the scene's partial norms, the Hessenberg
// column, Givens rotations, residual estimate and the scene's state.
__global__ void __launch_bounds__(256) kb_gm_givens(GmresState* __restrict__ st, const int2* __restrict__ rng,
                                                    const double* __restrict__ P, double* __restrict__ scale,
                                                    int lds_scale, const double* __restrict__ hbuf,
                                                    double* __restrict__ H, double* __restrict__ cs,
                                                    double* __restrict__ sn, double* __restrict__ gvec) {
  const int s = blockIdx.x;
  if (st[s].active == 0) return;
  __shared__ double nn[1];
  __shared__ double tmp[256];
  const int2 rg = rng[s];
  sum_partials(P + (size_t)rg.x * kBLd, rg.y - rg.x, kBLd, 1, nn, tmp);
  if (threadIdx.x != 0) return;
  GmresState& S = st[s];
  const int j = S.j, R = S.restart;
  const double nrm = sqrt(nn[0]);
  double* sc = scale + (size_t)s * lds_scale;
  double* Hs = H + (size_t)s * (R + 1) * R;
  double* css = cs + (size_t)s * (R + 1);
  double* sns = sn + (size_t)s * (R + 1);
  double* gs = gvec + (size_t)s * lds_scale;
  const double* hb = hbuf + (size_t)s * 2 * kBLd;
  double* Hc = Hs + (size_t)j * (R + 1);
  for (int i = 0; i <= j; ++i) Hc[i] = hb[i] + hb[kBLd + i];
  Hc[j + 1] = nrm;
  sc[j + 1] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
  for (int i = 0; i < j; ++i) {
    const double a = Hc[i], b = Hc[i + 1];
    Hc[i] = css[i] * a + sns[i] * b;
    Hc[i + 1] = -sns[i] * a + css[i] * b;
  }
  const double a = Hc[j], b = Hc[j + 1];
  const double rr = sqrt(a * a + b * b);
  const double c = (rr > 0.0) ? a / rr : 1.0, sv = (rr > 0.0) ? b / rr : 0.0;
  css[j] = c;
  sns[j] = sv;
  Hc[j] = rr;
  Hc[j + 1] = 0.0;
  gs[j + 1] = -sv * gs[j];
  gs[j] = c * gs[j];
  S.res = fabs(gs[j + 1]);
  S.j = j + 1;
  if (S.res <= S.tol || j + 1 >= R || !(nrm > 0.0) || !isfinite(S.res)) S.active = 0;
}

// r = b - r, v0 = r on the DOF rows of one scene; partial |r|^2 per block.
// Scenes already converged (done) keep their residual untouched.
__global__ void __launch_bounds__(256) kb_residual(const int4* __restrict__ tab, const double* __restrict__ b,
                                                   double* __restrict__ r, double* __restrict__ v0,
                                                   const GmresState* __restrict__ st, double* __restrict__ P) {
  __shared__ double lds[32];
  const int4 e = tab[blockIdx.x];
  if (st[e.x].done) return;
  double acc = 0.0;
  for (long long i = e.y + threadIdx.x; i < e.z; i += blockDim.x) {
    const double v = b[i] - r[i];
    r[i] = v;
    v0[i] = v;
    acc += v * v;
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) P[(size_t)blockIdx.x * kBLd] = acc;
}

// One block per scene: |r| -> rnorm, res, scale_s[0], g_s; restart the cycle
// (j = 0, active) unless the residual meets the tolerance (done).  With
// set_tol = 1 (first call) the tolerance becomes rtol * |r|.
__global__ void __launch_bounds__(256) kb_residual_finish(GmresState* __restrict__ st, const int2* __restrict__ rng,
                                                          const double* __restrict__ P, double* __restrict__ scale,
                                                          int lds_scale, double* __restrict__ gvec,
                                                          const double* __restrict__ rtol, double* __restrict__ bnorm,
                                                          int set_tol) {
  const int s = blockIdx.x;
  GmresState& S = st[s];
  if (S.done) return;
  __shared__ double nn[1];
  __shared__ double tmp[256];
  const int2 rg = rng[s];
  sum_partials(P + (size_t)rg.x * kBLd, rg.y - rg.x, kBLd, 1, nn, tmp);
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(nn[0]);
  if (set_tol) {  // first residual of a solve: r = b, tolerance relative to |b_s|
    S.tol = rtol[s] * nrm;
    bnorm[s] = nrm;
  }
  S.rnorm = nrm;
  S.res = nrm;
  S.j = 0;
  const bool ok = !(nrm > S.tol);
  S.done = ok ? 1 : 0;
  S.active = ok ? 0 : 1;
  scale[(size_t)s * lds_scale] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
  gvec[(size_t)s * lds_scale] = nrm;
}

// One wavefront per scene: y = H^{-1} g (back substitution, column
// oriented), coef_s[i] = y_i scale_s[i], coef_s[128] = k_s.  Scenes that
// ran no iteration this cycle get k_s = 0.
__global__ void __launch_bounds__(64) kb_gm_solve_small(const GmresState* __restrict__ st,
                                                        const double* __restrict__ H,
                                                        const double* __restrict__ gvec,
                                                        const double* __restrict__ scale, int lds_scale,
                                                        double* __restrict__ coef) {
  __shared__ double y[130];
  const int s = blockIdx.x;
  const GmresState S = st[s];
  const int k = S.done ? 0 : S.j, R = S.restart;
  const double* Hs = H + (size_t)s * (R + 1) * R;
  const double* gs = gvec + (size_t)s * lds_scale;
  const double* sc = scale + (size_t)s * lds_scale;
  double* cf = coef + (size_t)s * kBLd;
  const int t = threadIdx.x;
  for (int i = t; i < k; i += 64) y[i] = gs[i];
  __syncthreads();
  for (int l = k - 1; l >= 0; --l) {
    const double* Hl = Hs + (size_t)l * (R + 1);
    const double yl = y[l] / Hl[l];
    __syncthreads();
    for (int i = t; i < l; i += 64) y[i] -= Hl[i] * yl;
    if (t == 0) y[l] = yl;
    __syncthreads();
  }
  for (int i = t; i < k; i += 64) cf[i] = y[i] * sc[i];
  if (t == 0) cf[128] = (double)k;
}

// out_r = sum_{i < k_s} coef_s[i] Vt_i[r] for the scene s of DOF row r.
__global__ void kb_gm_combine(long long n, const int* __restrict__ vscene, const double* __restrict__ Vt,
                              long long stride, const double* __restrict__ coef, double* __restrict__ out) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double* cf = coef + (size_t)vscene[r / 3] * kBLd;
  const int k = (int)cf[128];
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += cf[i] * Vt[(long long)i * stride + r];
  out[r] = acc;
}

// ---------------------------------------------------------------------------
// Delassus matrices and capacitance inverses of the scenes.

// Y_s[rloc[r]][a] = S[r][cv_a] (column a of the scene's contact vertices),
// one block per union contact vertex, from the rows of S^T.  The rows r of S
// are elimination positions; rloc[r] numbers the positions of each scene
// from 0, so Y_s has the scene's n_v rows.
__global__ void kb_fill_Y(int ncv_total, const int* __restrict__ cv, const int* __restrict__ cvscene,
                          const int* __restrict__ cvoff, const int* __restrict__ rloc,
                          const long long* __restrict__ yoff, const long long* __restrict__ STp,
                          const int* __restrict__ STj, const double* __restrict__ STx, double* __restrict__ Yb) {
  const int a = blockIdx.x;
  if (a >= ncv_total) return;
  const int s = cvscene[a];
  const int la = a - cvoff[s], ncv = cvoff[s + 1] - cvoff[s];
  const int v = cv[a];
  double* Y = Yb + yoff[s];
  for (long long p = STp[v] + threadIdx.x; p < STp[v + 1]; p += blockDim.x)
    Y[(size_t)rloc[STj[p]] * ncv + la] = STx[p];
}

// D_s = Y_s^T Y_s on FP64 matrix cores; one 256-thread block per 64x64
// lower-triangle tile of one scene (table entries {scene, ti, tj, -}), the
// whole K range of the scene's rows; both triangles are written.  Same
// operand/result layouts as the single-scene kernel (row lane/16 + 4 e).
typedef double bd4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) kb_syrk(const int4* __restrict__ tiles, const int* __restrict__ voff,
                                               const int* __restrict__ cvoff, const long long* __restrict__ yoff,
                                               const long long* __restrict__ doff, const double* __restrict__ Yb,
                                               double* __restrict__ Db) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int4 e = tiles[blockIdx.x];
  const int s = e.x, ti = e.y, tj = e.z;
  const int nv = voff[s + 1] - voff[s], ncv = cvoff[s + 1] - cvoff[s];
  const double* Y = Yb + yoff[s];
  double* D = Db + doff[s];
  const int a0 = ti * 64, b0 = tj * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wa = 32 * (w >> 1), wb = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
  bd4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = bd4{0, 0, 0, 0};
  for (int r0 = 0; r0 < nv; r0 += 16) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int idx = tid + 256 * k;
      const int kr = idx / 64, c = idx % 64;
      const int r = r0 + kr;
      const bool rin = r < nv;
      As[kr][c] = (rin && a0 + c < ncv) ? Y[(size_t)r * ncv + a0 + c] : 0.0;
      Bs[kr][c] = (rin && b0 + c < ncv) ? Y[(size_t)r * ncv + b0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        av[p] = As[k4 + lk][wa + 16 * p + li];
        bv[p] = Bs[k4 + lk][wb + 16 * p + li];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = a0 + wa + 16 * p + lk + 4 * k;
        const int jj = b0 + wb + 16 * q + li;
        if (i < ncv && jj < ncv) {
          D[(size_t)i * ncv + jj] = acc[p][q][k];
          if (ti != tj) D[(size_t)jj * ncv + i] = acc[p][q][k];
        }
      }
}

// Z_s[v - voff_s][c] = sum_p S^T[v][p] Y_s[rloc[p]][c], one block per
// union vertex of a scene with contacts (list zv).
__global__ void __launch_bounds__(256) kb_spmm_Z(int nzv, const int* __restrict__ zv, const int* __restrict__ vscene,
                                                 const int* __restrict__ voff, const int* __restrict__ rloc,
                                                 const int* __restrict__ cvoff,
                                                 const long long* __restrict__ yoff, const long long* __restrict__ STp,
                                                 const int* __restrict__ STj, const double* __restrict__ STx,
                                                 const double* __restrict__ Yb, double* __restrict__ Zb) {
  const int k = blockIdx.x;
  if (k >= nzv) return;
  const int v = zv[k];
  const int s = vscene[v];
  const int ncv = cvoff[s + 1] - cvoff[s];
  const double* Y = Yb + yoff[s];
  double* Z = Zb + yoff[s];
  const int lv = v - voff[s];
  for (int c = threadIdx.x; c < ncv; c += blockDim.x) {
    double acc = 0.0;
    for (long long p = STp[v]; p < STp[v + 1]; ++p) acc += STx[p] * Y[(size_t)rloc[STj[p]] * ncv + c];
    Z[(size_t)lv * ncv + c] = acc;
  }
}

// Capacitance of every scene (transposed system): padded row list entries
// {scene, local row, -, -}; columns j < mp_s; padding rows and columns are
// the identity.  Same entries as the single-scene kernel.
__global__ void kb_capacitance(const int4* __restrict__ prow, const int* __restrict__ moff,
                               const int* __restrict__ mps, const long long* __restrict__ xoff,
                               const int* __restrict__ cvoff, const int* __restrict__ coff,
                               const int* __restrict__ row_c, const int* __restrict__ row_i,
                               const int* __restrict__ cmap, const long long* __restrict__ doff,
                               const double* __restrict__ Db, const double* __restrict__ Q,
                               const double* __restrict__ kh, const double* __restrict__ mu_c, double h2,
                               double* __restrict__ Cb) {
  const int4 e = prow[blockIdx.x];
  const int s = e.x, i = e.y;
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  const int mp = mps[s];
  if (j >= mp) return;
  const int m = moff[s + 1] - moff[s];
  double* C = Cb + xoff[s];
  if (i >= m || j >= m) {
    C[(size_t)i * mp + j] = (i == j) ? 1.0 : 0.0;
    return;
  }
  const int ncv = cvoff[s + 1] - cvoff[s];
  const int cb = cvoff[s];
  const int ri = moff[s] + i, rj = moff[s] + j;
  const int c = row_c[ri], a = row_i[ri];
  const int c2 = row_c[rj], b = row_i[rj];
  const double* q1 = Q + 9 * c + 3 * a;
  const double* q2 = Q + 9 * c2 + 3 * b;
  const double* D = Db + doff[s];
  double v = h2 * D[(size_t)(cmap[c] - cb) * ncv + (cmap[c2] - cb)] * (q1[0] * q2[0] + q1[1] * q2[1] + q1[2] * q2[2]);
  if (c == c2) {
    const double ka = kh[4 * c], kb = kh[4 * c + 1], kc = kh[4 * c + 2];
    if (a == 0 && b == 0) v += 1.0 / ka;
    else if (a == 0 && b == 1) v += mu_c[c] / kb;
    else if (a == 1 && b == 1) v += 1.0 / kb;
    else if (a == 2 && b == 2) v += (kc > 1e-200) ? 1.0 / kc : 1e200;
  }
  C[(size_t)i * mp + j] = v;
  (void)coff;
}

// one block per scene: grad[3 s + 0] += sum of tE over the scene's tets,
// grad[3 s + 1] += sum of tN, grad[3 s + 2] += sum of gmu over its contacts
__global__ void __launch_bounds__(256) kb_param_sums(const int* __restrict__ toff, const int* __restrict__ coff,
                                                     const double* __restrict__ tE, const double* __restrict__ tN,
                                                     const double* __restrict__ gmu, double* __restrict__ grad) {
  __shared__ double lds[32];
  const int s = blockIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int t = toff[s] + threadIdx.x; t < toff[s + 1]; t += blockDim.x) {
    a += tE[t];
    b += tN[t];
  }
  for (int k = coff[s] + threadIdx.x; k < coff[s + 1]; k += blockDim.x) c += gmu[k];
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  c = block_sum(c, lds);
  if (threadIdx.x == 0) {
    grad[3 * s] += a;
    grad[3 * s + 1] += b;
    grad[3 * s + 2] += c;
  }
}

// Union contact arrays from every scene's arrays in one launch: thread c
// finds its scene (ns is small: linear scan of the ranges), shifts the
// vertex id by the scene's first union vertex and copies the frame, gap,
// and multiplier rows.
__global__ void kb_gather_contacts(int nc, int ns, const ContactSrc* __restrict__ src, int* __restrict__ vid,
                                   int* __restrict__ fric, double* __restrict__ frame, double* __restrict__ delta,
                                   double* __restrict__ lam) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int s = 0;
  while (s + 1 < ns && src[s + 1].off <= c) ++s;
  const ContactSrc& S = src[s];
  const int k = c - S.off;
  vid[c] = S.vid[k] + S.voff;
  fric[c] = S.fric[k];
#pragma unroll
  for (int e = 0; e < 9; ++e) frame[9 * c + e] = S.frame[9 * k + e];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    delta[3 * c + e] = S.delta[3 * k + e];
    lam[3 * c + e] = S.lam[3 * k + e];
  }
}

// active = 1 for every scene not yet converged (before the end-of-cycle
// products), 0 for the others
__global__ void kb_set_active(int ns, GmresState* __restrict__ st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < ns) st[s].active = st[s].done ? 0 : 1;
}

// y += x on the rows of active scenes
__global__ void kb_axpy_active(long long n, const int* __restrict__ vscene, const GmresState* __restrict__ st,
                               const double* __restrict__ x, double* __restrict__ y) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || st[vscene[r / 3]].active == 0) return;
  y[r] += x[r];
}

// w = Acal^T x on the rows of active scenes (16 lanes per vertex row)
template <class MT>
__global__ void __launch_bounds__(256) kb_bsr_active(int nv, const int* __restrict__ vscene,
                                                     const GmresState* __restrict__ st,
                                                     const int* __restrict__ rowptr, const int* __restrict__ col,
                                                     const MT* __restrict__ val,
                                                     const double* __restrict__ val64, const double* __restrict__ x,
                                                     double* __restrict__ out) {
  const int sub = threadIdx.x & 15;
  const int row = blockIdx.x * 16 + threadIdx.x / 16;
  const bool on = row < nv && st[vscene[row < nv ? row : 0]].active != 0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (on) {
    for (int p = rowptr[row] + sub; p < rowptr[row + 1]; p += 16) {
      const int c = col[p];
      const double x0 = x[3 * c], x1 = x[3 * c + 1], x2 = x[3 * c + 2];
      block_madd<MT>(val, val64, (size_t)p, c == row, x0, x1, x2, a0, a1, a2);
    }
  }
  a0 = group_sum<16>(a0);
  a1 = group_sum<16>(a1);
  a2 = group_sum<16>(a2);
  if (on && sub == 0) {
    out[3 * row] = a0;
    out[3 * row + 1] = a1;
    out[3 * row + 2] = a2;
  }
}

// per-scene |x|^2 partials on a DOF table (for the refinement norms)
__global__ void __launch_bounds__(256) kb_norm_partials(const int4* __restrict__ tab, const double* __restrict__ x,
                                                        double* __restrict__ P) {
  __shared__ double lds[32];
  const int4 e = tab[blockIdx.x];
  double acc = 0.0;
  for (long long i = e.y + threadIdx.x; i < e.z; i += blockDim.x) acc += x[i] * x[i];
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) P[(size_t)blockIdx.x * kBLd] = acc;
}

// one block per scene: out[s] = sqrt(sum of the scene's partials)
__global__ void __launch_bounds__(256) kb_norm_finish(const int2* __restrict__ rng, const double* __restrict__ P,
                                                      double* __restrict__ out) {
  __shared__ double nn[1];
  __shared__ double tmp[256];
  const int2 rg = rng[blockIdx.x];
  sum_partials(P + (size_t)rg.x * kBLd, rg.y - rg.x, kBLd, 1, nn, tmp);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(nn[0]);
}

// host-side launchers ------------------------------------------------------

void launchb_spmv(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                  const double* cx, const double* xbase, long long stride, const double* scale, int lds,
                  const GmresState* st, const int* vscene, int use_j, double* y) {
  kb_spmv_tasks<double><<<ntasks, 256, 0, s>>>(tasks, rp, cj, cx, xbase, stride, scale, lds, st, vscene, use_j, y);
}
void launchb_spmv(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                  const float* cx, const double* xbase, long long stride, const double* scale, int lds,
                  const GmresState* st, const int* vscene, int use_j, double* y) {
  kb_spmv_tasks<float><<<ntasks, 256, 0, s>>>(tasks, rp, cj, cx, xbase, stride, scale, lds, st, vscene, use_j, y);
}
void launchb_spmv_acc(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                      const double* cx, const double* x, double alpha, const GmresState* st, const int* rscene,
                      double* y) {
  if (ntasks <= 0) return;
  kb_spmv_tasks<double, true><<<ntasks, 256, 0, s>>>(tasks, rp, cj, cx, x, 0, nullptr, 0, st, rscene, 0, y, alpha);
}
void launchb_spmv_acc(hipStream_t s, int ntasks, const int4* tasks, const long long* rp, const int* cj,
                      const float* cx, const double* x, double alpha, const GmresState* st, const int* rscene,
                      double* y) {
  if (ntasks <= 0) return;
  kb_spmv_tasks<float, true><<<ntasks, 256, 0, s>>>(tasks, rp, cj, cx, x, 0, nullptr, 0, st, rscene, 0, y, alpha);
}
void launchb_perm_gather(hipStream_t s, int n, const int* perm, const int* pscene, const double* xbase,
                         long long stride, const double* scale, int lds_scale, const GmresState* st, int use_j,
                         double* t) {
  kb_perm_gather<<<(3 * n + 255) / 256, 256, 0, s>>>(n, perm, pscene, xbase, stride, scale, lds_scale, st, use_j, t);
}
void launchb_perm_scatter(hipStream_t s, int n, const int* perm, const int* pscene, const double* z,
                          const GmresState* st, double* out) {
  kb_perm_scatter<<<(3 * n + 255) / 256, 256, 0, s>>>(n, perm, pscene, z, st, out);
}
void launchb_wb_gather(hipStream_t s, int nblk, int max_m, const int4* tab, const int* moff, const long long* xpos,
                       const int* mps, const int* row_c, const int* row_i, const int* vid, const double* Q,
                       const double* Xb, const double* u, const GmresState* st, double* t) {
  if (nblk == 0) return;
  kb_wb_gather<<<nblk, 256, (size_t)max_m * sizeof(double), s>>>(tab, moff, xpos, mps, row_c, row_i, vid, Q, Xb, u,
                                                                  st, t);
}
void launchb_wb_correct(hipStream_t s, int nblk, int max_ncv, const int4* tab, const int* voff, const int* cvoff,
                        const int* cv_ptr, const int* c_row0, const int* c_nrow, const double* Q, const double* t,
                        const double* Zb, const long long* yoff, double h2, const double* u, const GmresState* st,
                        double* y) {
  kb_wb_correct<<<nblk, 256, (size_t)3 * std::max(max_ncv, 1) * sizeof(double), s>>>(
      tab, voff, cvoff, cv_ptr, c_row0, c_nrow, Q, t, Zb, yoff, h2, u, st, y);
}
void launchb_bsr_dots(hipStream_t s, int nblk, const int4* tab, const int* rowptr, const int* col, const double* val,
                      const double* y, double* Vt, long long stride, const GmresState* st, double* P) {
  kb_bsr_dots<double, 16><<<nblk, 256, 0, s>>>(tab, rowptr, col, val, nullptr, y, Vt, stride, st, P);
}
void launchb_bsr_dots(hipStream_t s, int nblk, const int4* tab, const int* rowptr, const int* col, const float* val,
                      const double* val64, const double* y, double* Vt, long long stride, const GmresState* st,
                      double* P) {
  kb_bsr_dots<float, 16><<<nblk, 256, 0, s>>>(tab, rowptr, col, val, val64, y, Vt, stride, st, P);
}
void launchb_gm_update(hipStream_t s, int nblk, const int4* tab, int rpb, const int2* rng_in, const double* Pin,
                       double* Pout, double* Vt, long long stride, const double* scale, int lds, const GmresState* st,
                       double* hbuf, int mode) {
  kb_gm_update<<<nblk, 256, 0, s>>>(tab, rpb, rng_in, Pin, Pout, Vt, stride, scale, lds, st, hbuf, mode);
}
void launchb_gm_givens(hipStream_t s, int ns, GmresState* st, const int2* rng, const double* P, double* scale,
                       int lds, const double* hbuf, double* H, double* cs, double* sn, double* g) {
  kb_gm_givens<<<ns, 256, 0, s>>>(st, rng, P, scale, lds, hbuf, H, cs, sn, g);
}
void launchb_residual(hipStream_t s, int nblk, int ns, const int4* tab, const int2* rng, const double* b, double* r,
                      double* v0, GmresState* st, double* P, double* scale, int lds, double* g, const double* rtol,
                      double* bnorm, int set_tol) {
  kb_residual<<<nblk, 256, 0, s>>>(tab, b, r, v0, st, P);
  kb_residual_finish<<<ns, 256, 0, s>>>(st, rng, P, scale, lds, g, rtol, bnorm, set_tol);
}
void launchb_finish(hipStream_t s, int ns, long long n, const int* vscene, const GmresState* st, const double* H,
                    const double* g, const double* scale, int lds, const double* Vt, long long stride, double* coef,
                    double* out) {
  kb_gm_solve_small<<<ns, 64, 0, s>>>(st, H, g, scale, lds, coef);
  kb_gm_combine<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, vscene, Vt, stride, coef, out);
}
void launchb_set_active(hipStream_t s, int ns, GmresState* st) {
  kb_set_active<<<(ns + 255) / 256, 256, 0, s>>>(ns, st);
}
void launchb_axpy_active(hipStream_t s, long long n, const int* vscene, const GmresState* st, const double* x,
                         double* y) {
  kb_axpy_active<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, vscene, st, x, y);
}
void launchb_bsr_active(hipStream_t s, int nv, const int* vscene, const GmresState* st, const int* rowptr,
                        const int* col, const double* val, const double* x, double* out) {
  kb_bsr_active<double><<<(nv + 15) / 16, 256, 0, s>>>(nv, vscene, st, rowptr, col, val, nullptr, x, out);
}
void launchb_bsr_active(hipStream_t s, int nv, const int* vscene, const GmresState* st, const int* rowptr,
                        const int* col, const float* val, const double* val64, const double* x, double* out) {
  kb_bsr_active<float><<<(nv + 15) / 16, 256, 0, s>>>(nv, vscene, st, rowptr, col, val, val64, x, out);
}
void launchb_norms(hipStream_t s, int nblk, int ns, const int4* tab, const int2* rng, const double* x, double* P,
                   double* out) {
  kb_norm_partials<<<nblk, 256, 0, s>>>(tab, x, P);
  kb_norm_finish<<<ns, 256, 0, s>>>(rng, P, out);
}
// w[cv_a] = sum over the contacts at union contact vertex a of Q_c^T t_c for
// the active scenes (w zero elsewhere); one thread per contact vertex.
__global__ void kb_scatter_ht(int ncv, const int* __restrict__ cv, const int* __restrict__ cvscene,
                              const int* __restrict__ cv_ptr, const int* __restrict__ c_row0,
                              const int* __restrict__ c_nrow, const double* __restrict__ Q,
                              const double* __restrict__ t, const GmresState* __restrict__ st,
                              double* __restrict__ w) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ncv || st[cvscene[a]].active == 0) return;
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

void launchb_scatter_ht(hipStream_t s, int ncv, const int* cv, const int* cvscene, const int* cv_ptr,
                        const int* c_row0, const int* c_nrow, const double* Q, const double* t, const GmresState* st,
                        double* w) {
  if (ncv > 0) kb_scatter_ht<<<(ncv + 255) / 256, 256, 0, s>>>(ncv, cv, cvscene, cv_ptr, c_row0, c_nrow, Q, t, st, w);
}

void launchb_delassus(hipStream_t s, int ncv_total, int ntiles, int nzv, const int* cv, const int* cvscene,
                      const int* cvoff, const int* voff, const int* vscene, const int* rloc, const long long* yoff,
                      const long long* doff, const int4* tiles, const int* zv, const long long* STp, const int* STj,
                      const double* STx, double* Yb, double* Db, double* Zb) {
  if (ncv_total == 0) return;
  kb_fill_Y<<<ncv_total, 256, 0, s>>>(ncv_total, cv, cvscene, cvoff, rloc, yoff, STp, STj, STx, Yb);
  if (ntiles) kb_syrk<<<ntiles, 256, 0, s>>>(tiles, voff, cvoff, yoff, doff, Yb, Db);
  if (nzv) kb_spmm_Z<<<nzv, 256, 0, s>>>(nzv, zv, vscene, voff, rloc, cvoff, yoff, STp, STj, STx, Yb, Zb);
}
void launchb_capacitance(hipStream_t s, int nprow, int max_mp, const int4* prow, const int* moff, const int* mps,
                         const long long* xoff, const int* cvoff, const int* coff, const int* row_c,
                         const int* row_i, const int* cmap, const long long* doff, const double* Db,
                         const double* Q, const double* kh, const double* mu_c, double h2, double* Cb) {
  if (nprow == 0) return;
  dim3 g(nprow, (max_mp + 255) / 256);
  kb_capacitance<<<g, 256, 0, s>>>(prow, moff, mps, xoff, cvoff, coff, row_c, row_i, cmap, doff, Db, Q, kh, mu_c,
                                   h2, Cb);
}
void launchb_param_sums(hipStream_t s, int ns, const int* toff, const int* coff, const double* tE,
                        const double* tN, const double* gmu, double* grad) {
  kb_param_sums<<<ns, 256, 0, s>>>(toff, coff, tE, tN, gmu, grad);
}
void launchb_gather_contacts(hipStream_t s, int nc, int ns, const ContactSrc* src, int* vid, int* fric, double* frame,
                             double* delta, double* lam) {
  if (nc > 0) kb_gather_contacts<<<(nc + 255) / 256, 256, 0, s>>>(nc, ns, src, vid, fric, frame, delta, lam);
}

}  // namespace adj
