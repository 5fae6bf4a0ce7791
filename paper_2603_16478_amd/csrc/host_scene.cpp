// Host-side scene construction (see host_scene.h).
//
// A = M + h^2 sum_i w_i G_i^T G_i with G_i = Bt_i^T (x) I_3 (vec F = G_i q,
// column-major vec) is A_s (x) I_3 for the scalar n_v x n_v matrix
//     A_s = diag(m) + h^2 sum_i w_i Bt_i Bt_i^T,
// so one scalar factorisation serves all three coordinates.  The factor is
// computed once per scene (A does not depend on the state, eq:dynamics) and
// its inverse S = L^{-1} P gives A^{-1} = S^T S (Sec. 3.4).
#include "host_scene.h"

#include <thread>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>

namespace adj {

const int kPairK[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
const int kPairL[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

int pair_index(int k, int l) {
  static const int tbl[4][4] = {{0, 1, 2, 3}, {-1, 4, 5, 6}, {-1, -1, 7, 8}, {-1, -1, -1, 9}};
  return tbl[k][l];
}

namespace {

void inv3(const double* a, double* out, double* det_out) {
  double c00 = a[4] * a[8] - a[5] * a[7];
  double c01 = a[5] * a[6] - a[3] * a[8];
  double c02 = a[3] * a[7] - a[4] * a[6];
  double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  double id = 1.0 / det;
  out[0] = c00 * id;
  out[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  out[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  out[3] = c01 * id;
  out[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  out[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  out[6] = c02 * id;
  out[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  out[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  *det_out = det;
}

// Geometric nested dissection on the vertex graph: split the longest axis of
// the bounding box at the median, take as separator the vertices of the
// first half that touch the second half, recurse, separator last.  Every
// leaf subdomain and every separator is recorded as a segment of the
// ordering with its height in the separator tree (leaves 0, a separator one
// above the higher of its two halves); returns the height of the subtree
// (-1 when it recorded no segment).  L couples a segment only with its
// descendants and ancestors, so segments of equal height are independent.
int nested_dissection(const std::vector<int32_t>& verts, const std::vector<double>& pos,
                      const std::vector<std::vector<int32_t>>& adj, std::vector<int32_t>& out,
                      std::vector<int8_t>& side, std::vector<NdSegment>& segs) {
  const size_t kLeaf = 48;
  if (verts.empty()) return -1;
  if (verts.size() <= kLeaf) {
    std::vector<int32_t> v = verts;
    std::sort(v.begin(), v.end());
    segs.push_back({(int32_t)out.size(), (int32_t)v.size(), 0});
    out.insert(out.end(), v.begin(), v.end());
    return 0;
  }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int32_t v : verts)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], pos[3 * v + c]);
      hi[c] = std::max(hi[c], pos[3 * v + c]);
    }
  int ax = 0;
  for (int c = 1; c < 3; ++c)
    if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
  std::vector<int32_t> v = verts;
  std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) {
    if (pos[3 * a + ax] != pos[3 * b + ax]) return pos[3 * a + ax] < pos[3 * b + ax];
    return a < b;
  });
  size_t half = v.size() / 2;
  // keep vertices with the same coordinate together: the separator is a layer
  double cut = pos[3 * v[half] + ax];
  size_t split = half;
  while (split > 0 && pos[3 * v[split - 1] + ax] == cut) --split;
  if (split == 0) split = half;
  for (size_t i = 0; i < v.size(); ++i) side[v[i]] = (i < split) ? 1 : 2;
  std::vector<int32_t> left, right, sep;
  for (size_t i = 0; i < v.size(); ++i) {
    int32_t a = v[i];
    if (side[a] == 2) {
      right.push_back(a);
      continue;
    }
    bool touches = false;
    for (int32_t b : adj[a])
      if (side[b] == 2) {
        touches = true;
        break;
      }
    (touches ? sep : left).push_back(a);
  }
  for (int32_t a : v) side[a] = 0;
  if (left.empty() || right.empty()) {
    std::sort(v.begin(), v.end());
    segs.push_back({(int32_t)out.size(), (int32_t)v.size(), 0});
    out.insert(out.end(), v.begin(), v.end());
    return 0;
  }
  const int hl = nested_dissection(left, pos, adj, out, side, segs);
  const int hr = nested_dissection(right, pos, adj, out, side, segs);
  const int h = std::max(hl, hr);
  if (sep.empty()) return h;
  std::sort(sep.begin(), sep.end());
  segs.push_back({(int32_t)out.size(), (int32_t)sep.size(), h + 1});
  out.insert(out.end(), sep.begin(), sep.end());
  return h + 1;
}

}  // namespace

std::vector<int32_t> make_row_tasks(const std::vector<int64_t>& rowptr, int64_t big,
                                    const std::vector<int32_t>* rows, bool skip_empty) {
  std::vector<int32_t> t;
  std::vector<int32_t> small;
  // longest rows first: blocks are dispatched in grid order, so the rows that
  // bound the launch start earliest, and the rows sharing a block have
  // similar lengths
  std::vector<int32_t> order;
  if (rows) {
    order = *rows;
  } else {
    const int n = (int)rowptr.size() - 1;
    order.reserve(n);
    for (int r = 0; r < n; ++r)
      if (!skip_empty || rowptr[r + 1] > rowptr[r]) order.push_back(r);
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return rowptr[a + 1] - rowptr[a] > rowptr[b + 1] - rowptr[b]; });
  for (int r : order) {
    if (rowptr[r + 1] - rowptr[r] > big) {
      t.insert(t.end(), {r | 0x40000000, -1, -1, -1});
    } else {
      small.push_back(r);
      if (small.size() == 4) {
        t.insert(t.end(), small.begin(), small.end());
        small.clear();
      }
    }
  }
  if (!small.empty()) {
    while (small.size() < 4) small.push_back(-1);
    t.insert(t.end(), small.begin(), small.end());
  }
  return t;
}

// Level-scheduled triangular sweeps with the Cholesky factor (A_s^{-1} =
// P^T L^{-T} L^{-1} P).  Per segment of the nested dissection (a leaf
// subdomain or a separator, contiguous in the elimination order) the
// diagonal block L_ss is inverted densely; the remaining entries of L couple
// a segment only to its descendants (rows) or ancestors (columns).  Forward
// sweep, levels by increasing height:  t_s -= L_{s,desc} y_desc, then
// y_s = L_ss^{-1} t_s.  Backward, levels by decreasing height:
// t_s -= L_{anc,s}^T z_anc, then z_s = L_ss^{-T} t_s.  All four parts are
// CSR over elimination rows, with per-level task lists of the rows that
// have entries.
void build_sweeps(HostScene& s) {
  const int nv = s.nv;
  std::vector<int32_t> seg_of(nv, -1);
  int levels = 0;
  for (size_t g = 0; g < s.segs.size(); ++g) {
    for (int32_t i = 0; i < s.segs[g].len; ++i) seg_of[s.segs[g].start + i] = (int32_t)g;
    levels = std::max(levels, s.segs[g].height + 1);
  }
  for (int i = 0; i < nv; ++i)
    if (seg_of[i] < 0) return;  // not a complete segmentation: no sweeps
  // off-diagonal-block entries: forward rows (row i of L, columns j < i in
  // other segments) by counting from the CSC columns; backward rows (column
  // j of L below its segment) straight from the columns
  s.Fp.assign(nv + 1, 0);
  s.Bp.assign(nv + 1, 0);
  for (int j = 0; j < nv; ++j)
    for (int32_t p = s.Lp[j] + 1; p < s.Lp[j + 1]; ++p)
      if (seg_of[s.Li[p]] != seg_of[j]) {
        s.Fp[s.Li[p] + 1]++;
        s.Bp[j + 1]++;
      }
  for (int i = 0; i < nv; ++i) {
    s.Fp[i + 1] += s.Fp[i];
    s.Bp[i + 1] += s.Bp[i];
  }
  s.Fj.resize(s.Fp[nv]);
  s.Fx.resize(s.Fp[nv]);
  s.Bj.resize(s.Bp[nv]);
  s.Bx.resize(s.Bp[nv]);
  {
    std::vector<int64_t> fpos(s.Fp.begin(), s.Fp.end() - 1);
    for (int j = 0; j < nv; ++j) {
      int64_t b = s.Bp[j];
      for (int32_t p = s.Lp[j] + 1; p < s.Lp[j + 1]; ++p)
        if (seg_of[s.Li[p]] != seg_of[j]) {
          const int64_t o = fpos[s.Li[p]]++;
          s.Fj[o] = j;
          s.Fx[o] = s.Lx[p];
          s.Bj[b] = s.Li[p];
          s.Bx[b++] = s.Lx[p];
        }
    }
  }
  // dense inverses of the diagonal blocks, segments spread over host threads
  const size_t nseg = s.segs.size();
  std::vector<std::vector<double>> inv(nseg);
  auto invert = [&](size_t g) {
    const int32_t s0 = s.segs[g].start, n = s.segs[g].len;
    std::vector<double> Ld((size_t)n * n, 0.0);  // row-major lower-triangular block
    for (int32_t c = 0; c < n; ++c)
      for (int32_t p = s.Lp[s0 + c]; p < s.Lp[s0 + c + 1]; ++p) {
        const int32_t r = s.Li[p] - s0;
        if (r < n) Ld[(size_t)r * n + c] = s.Lx[p];
      }
    std::vector<double>& X = inv[g];
    X.assign((size_t)n * n, 0.0);  // row-major inverse, lower-triangular
    for (int32_t c = 0; c < n; ++c) {
      // column c of the inverse: forward substitution of e_c
      X[(size_t)c * n + c] = 1.0 / Ld[(size_t)c * n + c];
      for (int32_t r = c + 1; r < n; ++r) {
        double acc = 0.0;
        for (int32_t k = c; k < r; ++k) acc += Ld[(size_t)r * n + k] * X[(size_t)k * n + c];
        X[(size_t)r * n + c] = -acc / Ld[(size_t)r * n + r];
      }
    }
  };
  {
    std::vector<size_t> order(nseg);
    for (size_t g = 0; g < nseg; ++g) order[g] = g;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return s.segs[a].len > s.segs[b].len; });
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nthreads = (int)std::min<unsigned>(16u, hw);
    std::atomic<size_t> next{0};
    auto work = [&]() {
      for (size_t k = next++; k < nseg; k = next++) invert(order[k]);
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nthreads; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
  }
  s.Ip.assign(nv + 1, 0);
  s.ITp.assign(nv + 1, 0);
  for (size_t g = 0; g < nseg; ++g) {
    const int32_t s0 = s.segs[g].start, n = s.segs[g].len;
    const std::vector<double>& X = inv[g];
    for (int32_t r = 0; r < n; ++r)
      for (int32_t c = 0; c < n; ++c)
        if (X[(size_t)r * n + c] != 0.0) {
          s.Ip[s0 + r + 1]++;
          s.ITp[s0 + c + 1]++;
        }
  }
  for (int i = 0; i < nv; ++i) {
    s.Ip[i + 1] += s.Ip[i];
    s.ITp[i + 1] += s.ITp[i];
  }
  s.Ij.resize(s.Ip[nv]);
  s.Ix.resize(s.Ip[nv]);
  s.ITj.resize(s.ITp[nv]);
  s.ITx.resize(s.ITp[nv]);
  {
    std::vector<int64_t> ip(s.Ip.begin(), s.Ip.end() - 1), itp(s.ITp.begin(), s.ITp.end() - 1);
    for (size_t g = 0; g < nseg; ++g) {
      const int32_t s0 = s.segs[g].start, n = s.segs[g].len;
      const std::vector<double>& X = inv[g];
      for (int32_t r = 0; r < n; ++r)
        for (int32_t c = 0; c < n; ++c) {
          const double v = X[(size_t)r * n + c];
          if (v == 0.0) continue;
          const int64_t o = ip[s0 + r]++;
          s.Ij[o] = s0 + c;
          s.Ix[o] = v;
          const int64_t o2 = itp[s0 + c]++;  // row s0 + c of L_ss^{-T}: columns s0 + r >= s0 + c
          s.ITj[o2] = s0 + r;
          s.ITx[o2] = v;
        }
    }
  }
  // per-level task lists of each phase
  s.n_levels = levels;
  std::vector<std::vector<int32_t>> rows(levels);
  for (size_t g = 0; g < nseg; ++g)
    for (int32_t i = 0; i < s.segs[g].len; ++i) rows[s.segs[g].height].push_back(s.segs[g].start + i);
  auto lists = [&](const std::vector<int64_t>& rp, std::vector<int32_t>& tasks, std::vector<int32_t>& off) {
    tasks.clear();
    off.assign(levels + 1, 0);
    for (int l = 0; l < levels; ++l) {
      std::vector<int32_t> r;
      for (int32_t i : rows[l])
        if (rp[i + 1] > rp[i]) r.push_back(i);
      const std::vector<int32_t> t = make_row_tasks(rp, 1024, &r);
      tasks.insert(tasks.end(), t.begin(), t.end());
      off[l + 1] = (int32_t)(tasks.size() / 4);
    }
  };
  lists(s.Fp, s.fA_tasks, s.fA_off);
  lists(s.Ip, s.fB_tasks, s.fB_off);
  lists(s.Bp, s.bA_tasks, s.bA_off);
  lists(s.ITp, s.bB_tasks, s.bB_off);
}

int sweep_parts(const HostScene& s, int k, std::vector<int32_t>& rows, std::vector<int32_t>& off) {
  rows.clear();
  off.clear();
  const int nv = s.nv;
  if (k <= 0 || s.n_levels == 0 || (int)s.Fp.size() != nv + 1) return 0;
  std::vector<int32_t> height(nv, -1), up(nv);
  for (const NdSegment& g : s.segs)
    for (int32_t i = 0; i < g.len; ++i) height[g.start + i] = g.height;
  for (int i = 0; i < nv; ++i) up[i] = i;
  auto find = [&](int a) {
    while (up[a] != a) {
      up[a] = up[up[a]];
      a = up[a];
    }
    return a;
  };
  auto join = [&](int a, int b) {
    a = find(a);
    b = find(b);
    if (a != b) up[std::max(a, b)] = std::min(a, b);
  };
  for (const NdSegment& g : s.segs)
    if (g.height < k)
      for (int32_t i = 1; i < g.len; ++i) join(g.start, g.start + i);
  for (int i = 0; i < nv; ++i)
    if (height[i] < k)
      for (int64_t p = s.Fp[i]; p < s.Fp[i + 1]; ++p) join(i, s.Fj[p]);  // descendants: heights < height[i]
  // parts in order of their smallest row; rows by (part, height, row)
  std::vector<int32_t> part(nv, -1);
  int np = 0;
  for (int i = 0; i < nv; ++i)
    if (height[i] >= 0 && height[i] < k) {
      const int r = find(i);
      if (part[r] < 0) part[r] = np++;
      part[i] = part[r];
    }
  std::vector<int32_t> cnt((size_t)np * k + 1, 0);
  for (int i = 0; i < nv; ++i)
    if (part[i] >= 0) cnt[(size_t)part[i] * k + height[i] + 1]++;
  for (size_t e = 1; e < cnt.size(); ++e) cnt[e] += cnt[e - 1];
  rows.assign(cnt.back(), 0);
  std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
  for (int i = 0; i < nv; ++i)
    if (part[i] >= 0) rows[pos[(size_t)part[i] * k + height[i]]++] = i;
  off.assign((size_t)np * (k + 1), 0);
  for (int c = 0; c < np; ++c) {
    for (int h = 0; h < k; ++h) off[(size_t)c * (k + 1) + h] = cnt[(size_t)c * k + h];
    off[(size_t)c * (k + 1) + k] = cnt[(size_t)(c + 1) * k];
  }
  return np;
}

adj_status build_host_scene(const adj_scene_desc* d, HostScene& s, std::string& err) {
  if (!d || d->n_verts <= 0 || d->n_tets <= 0 || !d->rest_pos || !d->tets || !d->E || !d->nu) {
    err = "scene_desc: missing arrays or non-positive sizes";
    return ADJ_E_ARG;
  }
  if (!(d->h > 0) || !(d->eps > 0) || !(d->density > 0) || d->n_planes < 0 ||
      (d->n_planes > 0 && !d->planes)) {
    err = "scene_desc: h, eps, density must be positive";
    return ADJ_E_ARG;
  }
  const int nv = d->n_verts, nt = d->n_tets;
  s.nv = nv;
  s.nt = nt;
  s.h = d->h;
  s.eps = d->eps;
  s.density = d->density;
  s.margin = d->contact_margin;
  for (int c = 0; c < 3; ++c) s.gravity[c] = d->gravity[c];
  s.planes.assign(d->planes, d->planes + 4 * d->n_planes);
  s.rest.assign(d->rest_pos, d->rest_pos + 3 * (size_t)nv);
  s.tets.assign(d->tets, d->tets + 4 * (size_t)nt);
  for (int32_t v : s.tets)
    if (v < 0 || v >= nv) {
      err = "tet references a vertex out of range";
      return ADJ_E_ARG;
    }
  if (d->material < 0 || d->material > 2) {
    err = "scene_desc: material must be 0 (Neo-Hookean), 1 (ARAP) or 2 (co-rotational)";
    return ADJ_E_ARG;
  }
  s.material = d->material;
  if (d->n_bindings < 0 || (d->n_bindings > 0 && (!d->binding_vid || !d->binding_E))) {
    err = "scene_desc: binding arrays missing";
    return ADJ_E_ARG;
  }
  s.bvid.assign(d->binding_vid, d->binding_vid + std::max(0, d->n_bindings));
  s.bE.assign(d->binding_E, d->binding_E + std::max(0, d->n_bindings));
  {
    std::vector<char> seen(nv, 0);
    for (size_t b = 0; b < s.bvid.size(); ++b) {
      const int32_t v = s.bvid[b];
      if (v < 0 || v >= nv || seen[v] || !(s.bE[b] > 0) || !std::isfinite(s.bE[b])) {
        err = "bindings: vertex out of range or repeated, or compliance not positive";
        return ADJ_E_ARG;
      }
      seen[v] = 1;
    }
  }
  s.Bm.resize(9 * (size_t)nt);
  s.Bt.resize(12 * (size_t)nt);
  s.vol.resize(nt);
  s.lmu.resize(nt);
  s.llam.resize(nt);
  s.E.resize(nt);
  s.nu.resize(nt);
  s.mass.assign(nv, 0.0);
  for (int t = 0; t < nt; ++t) {
    const int32_t* tv = &s.tets[4 * (size_t)t];
    double Dm[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Dm[3 * r + c] = s.rest[3 * tv[c + 1] + r] - s.rest[3 * tv[0] + r];
    double det;
    inv3(Dm, &s.Bm[9 * (size_t)t], &det);
    if (!(det > 0)) {
      err = "rest tet " + std::to_string(t) + " has non-positive orientation";
      return ADJ_E_INVERTED;
    }
    s.vol[t] = det / 6.0;
    const double* B = &s.Bm[9 * (size_t)t];
    double* Bt = &s.Bt[12 * (size_t)t];
    for (int c = 0; c < 3; ++c) {
      Bt[c] = -(B[c] + B[3 + c] + B[6 + c]);
      for (int k = 0; k < 3; ++k) Bt[3 * (k + 1) + c] = B[3 * k + c];
    }
    double E = d->per_tet_material ? d->E[t] : d->E[0];
    double nu = d->per_tet_material ? d->nu[t] : d->nu[0];
    if (!(E > 0) || !(nu > -1.0 && nu < 0.5)) {
      err = "material out of range";
      return ADJ_E_ARG;
    }
    s.E[t] = E;
    s.nu[t] = nu;
    s.lmu[t] = E / (2.0 * (1.0 + nu));
    s.llam[t] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    for (int k = 0; k < 4; ++k) s.mass[tv[k]] += d->density * s.vol[t] / 4.0;
  }
  // vertex adjacency and block pattern
  std::vector<std::vector<int32_t>> adj(nv);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 4; ++k)
      for (int l = 0; l < 4; ++l) adj[s.tets[4 * t + k]].push_back(s.tets[4 * t + l]);
  s.rowptr.assign(nv + 1, 0);
  for (int v = 0; v < nv; ++v) {
    auto& a = adj[v];
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
    s.rowptr[v + 1] = s.rowptr[v] + (int32_t)a.size();
  }
  const int nnzb = s.rowptr[nv];
  s.col.resize(nnzb);
  s.row_of_slot.resize(nnzb);
  s.diag_slot.resize(nv);
  for (int v = 0; v < nv; ++v)
    for (int32_t p = s.rowptr[v]; p < s.rowptr[v + 1]; ++p) {
      s.col[p] = adj[v][p - s.rowptr[v]];
      s.row_of_slot[p] = v;
      if (s.col[p] == v) s.diag_slot[v] = p;
    }
  auto slot_of = [&](int a, int b) {
    auto first = s.col.begin() + s.rowptr[a], last = s.col.begin() + s.rowptr[a + 1];
    return (int32_t)(std::lower_bound(first, last, b) - s.col.begin());
  };
  // element -> slot map (gather lists) and the scalar A_s
  std::vector<int32_t> cnt(nnzb + 1, 0);
  std::vector<int32_t> tslot(16 * (size_t)nt);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 4; ++k)
      for (int l = 0; l < 4; ++l) {
        int32_t sl = slot_of(s.tets[4 * t + k], s.tets[4 * t + l]);
        tslot[16 * (size_t)t + 4 * k + l] = sl;
        cnt[sl + 1]++;
      }
  s.slot_ptr.assign(nnzb + 1, 0);
  for (int i = 0; i < nnzb; ++i) s.slot_ptr[i + 1] = s.slot_ptr[i] + cnt[i + 1];
  s.slot_code.resize(s.slot_ptr[nnzb]);
  std::vector<int32_t> fill(s.slot_ptr.begin(), s.slot_ptr.end() - 1);
  s.As.assign(nnzb, 0.0);
  const double h2 = d->h * d->h;
  for (int t = 0; t < nt; ++t) {
    const double* Bt = &s.Bt[12 * (size_t)t];
    double w = 2.0 * s.lmu[t] * s.vol[t];
    for (int k = 0; k < 4; ++k)
      for (int l = 0; l < 4; ++l) {
        int32_t sl = tslot[16 * (size_t)t + 4 * k + l];
        int pr = k <= l ? pair_index(k, l) : pair_index(l, k);
        int tr = k <= l ? 0 : 1;
        s.slot_code[fill[sl]++] = t * 32 + pr * 2 + tr;
        double bb = Bt[3 * k] * Bt[3 * l] + Bt[3 * k + 1] * Bt[3 * l + 1] + Bt[3 * k + 2] * Bt[3 * l + 2];
        s.As[sl] += h2 * w * bb;
      }
  }
  for (int v = 0; v < nv; ++v) s.As[s.diag_slot[v]] += s.mass[v];
  // bindings: h^2 J_b^T E_b^{-1} J_b (a scalar on the vertex's diagonal)
  for (size_t b = 0; b < s.bvid.size(); ++b) s.As[s.diag_slot[s.bvid[b]]] += h2 / s.bE[b];
  // vertex incidence (for gathering element forces)
  s.vptr.assign(nv + 1, 0);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 4; ++k) s.vptr[s.tets[4 * t + k] + 1]++;
  for (int v = 0; v < nv; ++v) s.vptr[v + 1] += s.vptr[v];
  s.vcode.resize(4 * (size_t)nt);
  {
    std::vector<int32_t> pos(s.vptr.begin(), s.vptr.end() - 1);
    for (int t = 0; t < nt; ++t)
      for (int k = 0; k < 4; ++k) s.vcode[pos[s.tets[4 * t + k]]++] = t * 4 + k;
  }

  // ordering
  {
    std::vector<int32_t> all(nv);
    std::iota(all.begin(), all.end(), 0);
    std::vector<int8_t> side(nv, 0);
    s.perm.clear();
    s.perm.reserve(nv);
    nested_dissection(all, s.rest, adj, s.perm, side, s.segs);
    s.iperm.assign(nv, -1);
    for (int i = 0; i < nv; ++i) s.iperm[s.perm[i]] = i;
  }
  // Permuted upper triangle by columns: column k holds rows i <= k of P A_s P^T.
  std::vector<std::vector<std::pair<int32_t, double>>> ucol(nv);
  for (int v = 0; v < nv; ++v)
    for (int32_t p = s.rowptr[v]; p < s.rowptr[v + 1]; ++p) {
      int i = s.iperm[v], j = s.iperm[s.col[p]];
      if (i <= j) ucol[j].push_back({i, s.As[p]});
    }
  for (auto& c : ucol) std::sort(c.begin(), c.end());
  // elimination tree (ancestor path compression)
  s.parent.assign(nv, -1);
  {
    std::vector<int32_t> anc(nv, -1);
    for (int k = 0; k < nv; ++k)
      for (auto& e : ucol[k]) {
        int i = e.first;
        while (i != -1 && i < k) {
          int nxt = anc[i];
          anc[i] = k;
          if (nxt == -1) {
            s.parent[i] = k;
            break;
          }
          i = nxt;
        }
      }
  }
  // row patterns via the elimination tree, column counts
  std::vector<int32_t> mark(nv, -1), colcount(nv, 1);
  auto row_pattern = [&](int k, std::vector<int32_t>& pat) {
    pat.clear();
    mark[k] = k;
    for (auto& e : ucol[k]) {
      int i = e.first;
      while (i < k && mark[i] != k) {
        pat.push_back(i);
        mark[i] = k;
        i = s.parent[i];
      }
    }
    std::sort(pat.begin(), pat.end());
  };
  std::vector<int32_t> pat;
  for (int k = 0; k < nv; ++k) {
    row_pattern(k, pat);
    for (int j : pat) colcount[j]++;
  }
  s.Lp.assign(nv + 1, 0);
  for (int j = 0; j < nv; ++j) s.Lp[j + 1] = s.Lp[j] + colcount[j];
  s.Li.assign(s.Lp[nv], 0);
  s.Lx.assign(s.Lp[nv], 0.0);
  std::vector<int32_t> next(nv);
  std::fill(mark.begin(), mark.end(), -1);
  std::vector<double> x(nv, 0.0);
  for (int k = 0; k < nv; ++k) {
    row_pattern(k, pat);
    double dk = 0.0;
    for (auto& e : ucol[k]) {
      if (e.first == k)
        dk = e.second;
      else
        x[e.first] = e.second;
    }
    for (int j : pat) {
      double yj = x[j] / s.Lx[s.Lp[j]];
      x[j] = 0.0;
      for (int32_t p = s.Lp[j] + 1; p < next[j]; ++p) x[s.Li[p]] -= s.Lx[p] * yj;
      dk -= yj * yj;
      s.Li[next[j]] = k;
      s.Lx[next[j]++] = yj;
    }
    if (!(dk > 0) || !std::isfinite(dk)) {
      err = "elastic system matrix is not positive definite";
      return ADJ_E_SINGULAR;
    }
    s.Li[s.Lp[k]] = k;
    s.Lx[s.Lp[k]] = std::sqrt(dk);
    next[k] = s.Lp[k] + 1;
  }
  // S = L^{-1} P column by column: column v of S is L^{-1} e_{iperm[v]},
  // nonzero exactly on the elimination-tree path from iperm[v] to the root.
  s.STp.assign(nv + 1, 0);
  for (int v = 0; v < nv; ++v) {
    int len = 0;
    for (int j = s.iperm[v]; j != -1; j = s.parent[j]) ++len;
    s.STp[v + 1] = s.STp[v] + len;
  }
  s.STj.resize(s.STp[nv]);
  s.STx.resize(s.STp[nv]);
  // the columns are independent: spread them over host threads, each with
  // its own work vector, writing disjoint slices of STj/STx
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nthreads = (int)std::min<unsigned>(16u, hw);
  auto columns = [&](int t0) {
    std::vector<double> xw(nv, 0.0);
    std::vector<int32_t> pth;
    for (int v = t0; v < nv; v += nthreads) {
      pth.clear();
      for (int j = s.iperm[v]; j != -1; j = s.parent[j]) pth.push_back(j);
      xw[pth[0]] = 1.0;
      for (int j : pth) {
        xw[j] /= s.Lx[s.Lp[j]];
        const double xj = xw[j];
        for (int32_t p = s.Lp[j] + 1; p < s.Lp[j + 1]; ++p) xw[s.Li[p]] -= s.Lx[p] * xj;
      }
      int64_t o = s.STp[v];
      for (int j : pth) {
        s.STj[o] = j;
        s.STx[o++] = xw[j];
        xw[j] = 0.0;
      }
    }
  };
  if (nthreads == 1 || nv < 4096) {
    for (int t = 0; t < nthreads; ++t) columns(t);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) pool.emplace_back(columns, t);
    for (auto& th : pool) th.join();
  }
  // transpose: CSR of S (rows = internal index)
  s.Sp.assign(nv + 1, 0);
  for (int64_t p = 0; p < s.STp[nv]; ++p) s.Sp[s.STj[p] + 1]++;
  for (int i = 0; i < nv; ++i) s.Sp[i + 1] += s.Sp[i];
  s.Sj.resize(s.STp[nv]);
  s.Sx.resize(s.STp[nv]);
  std::vector<int64_t> pos(s.Sp.begin(), s.Sp.end() - 1);
  for (int v = 0; v < nv; ++v)
    for (int64_t p = s.STp[v]; p < s.STp[v + 1]; ++p) {
      int64_t o = pos[s.STj[p]]++;
      s.Sj[o] = v;
      s.Sx[o] = s.STx[p];
    }
  s.S_tasks = make_row_tasks(s.Sp, 1024);
  s.ST_tasks = make_row_tasks(s.STp, 1024);
  build_sweeps(s);
  return ADJ_OK;
}

}  // namespace adj
