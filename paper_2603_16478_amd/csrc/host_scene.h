// Host-side scene construction: rest-shape operators, lumped mass, the
// constant scalar system matrix, its fill-reducing ordering, sparse Cholesky
// factor and sparse inverse, and the block pattern of the adjoint matrix with
// its element-to-entry map.  Plain C++, runs once per scene.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "adjoint.h"

namespace adj {

// The 10 blocks (k <= l) of a symmetric 4x4 block element matrix.
extern const int kPairK[10];
extern const int kPairL[10];
int pair_index(int k, int l);  // k <= l

// A segment of the nested-dissection ordering: a leaf subdomain or a
// separator, positions [start, start + len), with its separator-tree height.
struct NdSegment {
  int32_t start, len, height;
};

struct HostScene {
  int nv = 0, nt = 0;
  double h = 0, eps = 0, density = 0;
  double gravity[3] = {0, 0, 0};
  double margin = 0;
  std::vector<double> planes;  // [n_planes*4]
  std::vector<double> rest;    // [nv*3]
  std::vector<int32_t> tets;   // [nt*4]
  std::vector<double> Bm;      // [nt*9] row-major B_m = D_m^{-1}
  std::vector<double> Bt;      // [nt*12] row-major 4x3: [-1^T B_m; B_m]
  std::vector<double> vol, lmu, llam, E, nu;  // per tet (Lame mu, lambda; E, nu)
  std::vector<double> mass;    // per vertex
  // bilateral bindings: vertex and compliance per binding
  std::vector<int32_t> bvid;
  std::vector<double> bE;
  int material = 0;            // adj_material
  // Block pattern of Acal: rows = vertices, sorted columns, diagonal included.
  std::vector<int32_t> rowptr, col, diag_slot, row_of_slot;
  // Element-to-entry map: contributions to each block slot, ordered by
  // (tet, local pair); code = tet*32 + pair*2 + transpose.
  std::vector<int32_t> slot_ptr, slot_code;
  std::vector<double> As;      // scalar A_s per slot (A = A_s (x) I_3)
  // vertex -> incident (tet, corner) list, code = tet*4 + corner, tet order
  std::vector<int32_t> vptr, vcode;
  // Fill-reducing ordering (internal index -> vertex) and its inverse.
  std::vector<int32_t> perm, iperm;
  // Cholesky factor of P A_s P^T, CSC, diagonal first in every column.
  std::vector<int32_t> Lp, Li, parent;
  std::vector<double> Lx;
  // S = L^{-1} P: CSR by internal row (columns = vertices) and CSR of S^T
  // (rows = vertices, columns = internal rows).
  std::vector<int64_t> Sp, STp;
  std::vector<int32_t> Sj, STj;
  std::vector<double> Sx, STx;
  // load-balanced row tasks for the S and S^T products (4 ints per block)
  std::vector<int32_t> S_tasks, ST_tasks;
  // Level-scheduled sweeps with L (build_sweeps): nested-dissection segments;
  // off-diagonal-block rows of L (F) and of L^T (B); rows of the inverted
  // diagonal blocks L_ss^{-1} (I) and L_ss^{-T} (IT); per phase the row tasks
  // of every level, concatenated, with task offsets [n_levels + 1].  Empty
  // when the ordering has no complete segmentation.
  std::vector<NdSegment> segs;
  int n_levels = 0;
  std::vector<int64_t> Fp, Bp, Ip, ITp;
  std::vector<int32_t> Fj, Bj, Ij, ITj;
  std::vector<double> Fx, Bx, Ix, ITx;
  std::vector<int32_t> fA_tasks, fB_tasks, bA_tasks, bB_tasks;
  std::vector<int32_t> fA_off, fB_off, bA_off, bB_off;
};

void build_sweeps(HostScene& s);

// Rows of the k lowest sweep levels (heights < k) grouped into independent
// parts: rows joined by an entry of L between different segments, and the
// rows of one segment, fall in one part, so each part's sweep through those
// levels reads only its own rows (and, backwards, rows above height k - 1).
// rows: the parts one after another, each sorted by height then row; off:
// [n_parts * (k + 1)] start of height h of part c at off[c (k + 1) + h],
// the part's end at off[c (k + 1) + k].  Returns the number of parts.
int sweep_parts(const HostScene& s, int k, std::vector<int32_t>& rows, std::vector<int32_t>& off);

// Pack CSR rows into blocks: rows longer than `big` get a block each (flag
// 0x40000000), shorter rows go four to a block; -1 marks an empty slot.
// Tasks are ordered by decreasing row length.  `rows` restricts the tasks to
// the listed rows; `skip_empty` leaves out rows without entries.
std::vector<int32_t> make_row_tasks(const std::vector<int64_t>& rowptr, int64_t big,
                                    const std::vector<int32_t>* rows = nullptr, bool skip_empty = false);

// Returns ADJ_OK or an error code with a message in err.
adj_status build_host_scene(const adj_scene_desc* d, HostScene& s, std::string& err);

}  // namespace adj
